// The float32 pair kernel: every (query sphere, kept Gaussian) pair of the
// neighbourhood ball evaluated with Eq. 5, 7, 8 and folded into per-query
// reductions (count/label of Sec. II-E, min and the stable softmin of
// Sec. II-B, the averaged cost of Eq. 11).
//
// Layout and mapping on gfx950:
//  * 256 lanes (4 waves) per block, a few queries per lane; each query's
//    centre, r^2 and accumulators live in VGPRs;
//  * the Gaussian records are wave-uniform: every lane of a wave needs the
//    same Gaussian at the same time, so they are fetched with scalar loads
//    into SGPRs and used directly as VALU operands (no LDS round trip, no
//    VGPRs spent on them, no bank conflicts);
//  * the Gaussian list is cut into `splits` contiguous ranges so that small
//    query batches still fill the 256 CUs; blocks are mapped XCD-major so the
//    blocks of one XCD share a range in their L2; partial reductions are
//    merged in a fixed order by combine_kernel (bit-reproducible results).
#include <cmath>

#include "pair_core.h"

namespace csplat {

namespace {

using namespace pair;

template <int M, bool FULL, bool BALL>
void launch_pair(dim3 grid, hipStream_t st, const float *gs, int n, int per_split, int n_tiles,
                 const float *c, const float *r, int q, const EvalParams &p, const Part &part, float mu_max)
{
    constexpr int QPL = FULL ? kQplFull : kQplLabels;
    pair_kernel<M, FULL, BALL, QPL><<<grid, kBlock, 0, st>>>(gs, n, per_split, n_tiles, c, r, q, p, part, mu_max);
}

template <int M>
void launch_m(csplat_ctx *ctx, bool full, bool ball, dim3 grid, hipStream_t st, const float *gs, int n,
              int per_split, int n_tiles, const float *c, const float *r, int q,
              const EvalParams &p, const Part &part, int S, const EvalOut &out, float mu_max)
{
    if (n > 0) {
        timing_begin(ctx);
        if (full && ball) launch_pair<M, true, true>(grid, st, gs, n, per_split, n_tiles, c, r, q, p, part, mu_max);
        else if (full) launch_pair<M, true, false>(grid, st, gs, n, per_split, n_tiles, c, r, q, p, part, mu_max);
        else if (ball) launch_pair<M, false, true>(grid, st, gs, n, per_split, n_tiles, c, r, q, p, part, mu_max);
        else launch_pair<M, false, false>(grid, st, gs, n, per_split, n_tiles, c, r, q, p, part, mu_max);
        timing_end(ctx);
    }
    const int cb = (q + 255) / 256;
    if (full) combine_kernel<M, true><<<cb, 256, 0, st>>>(q, S, p, part, out);
    else combine_kernel<M, false><<<cb, 256, 0, st>>>(q, S, p, part, out);
}

}  // namespace

csplat_status fp32_eval(csplat_ctx *ctx, const csplat_scene *sc, int64_t q64, const float *centers,
                        const float *radii, const EvalParams &p, const EvalOut &out,
                        bool labels_only)
{
    const int q = (int)q64;
    const int n = (int)sc->n;
    const bool full = !labels_only;
    const bool ball = std::isfinite(p.rn2);
    const SplitPlan sp = split_plan(ctx_target_blocks(ctx), q, n, full);
    const int n_tiles = sp.n_tiles, per_split = sp.per_split, qpl = sp.qpl;
    const int S = std::max(sp.S, 1);
    const int M = p.m;
    const size_t words = (size_t)S * q * part_words(M, full);
    if (words > 0) {
        hipError_t e = ctx->partial.reserve(words * 4);
        if (e != hipSuccess) return hip_fail(e, "partial workspace");
    }
    const Part part = part_views(ctx->partial.ptr, S, q, M, full);
    ctx->stats.splits = S;
    ctx->stats.queries_per_lane = qpl;
    ctx->stats.kernel_pairs = (int64_t)q * n;
    dim3 grid((unsigned)(n_tiles * S));
    hipStream_t st = ctx->stream;
    const float *gs = sc->gauss;
    const int S_used = sp.S;
    switch (M) {
    case 1: launch_m<1>(ctx, full, ball, grid, st, gs, n, per_split, n_tiles, centers, radii, q, p, part, S_used, out, sc->mu_max); break;
    case 2: launch_m<2>(ctx, full, ball, grid, st, gs, n, per_split, n_tiles, centers, radii, q, p, part, S_used, out, sc->mu_max); break;
    case 3: launch_m<3>(ctx, full, ball, grid, st, gs, n, per_split, n_tiles, centers, radii, q, p, part, S_used, out, sc->mu_max); break;
    case 4: launch_m<4>(ctx, full, ball, grid, st, gs, n, per_split, n_tiles, centers, radii, q, p, part, S_used, out, sc->mu_max); break;
    case 5: launch_m<5>(ctx, full, ball, grid, st, gs, n, per_split, n_tiles, centers, radii, q, p, part, S_used, out, sc->mu_max); break;
    case 6: launch_m<6>(ctx, full, ball, grid, st, gs, n, per_split, n_tiles, centers, radii, q, p, part, S_used, out, sc->mu_max); break;
    case 7: launch_m<7>(ctx, full, ball, grid, st, gs, n, per_split, n_tiles, centers, radii, q, p, part, S_used, out, sc->mu_max); break;
    case 8: launch_m<8>(ctx, full, ball, grid, st, gs, n, per_split, n_tiles, centers, radii, q, p, part, S_used, out, sc->mu_max); break;
    default: return fail(CSPLAT_E_INVALID, "m out of range");
    }
    CSPLAT_HIP(hipGetLastError());
    return CSPLAT_OK;
}

}  // namespace csplat
