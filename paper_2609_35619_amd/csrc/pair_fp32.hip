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
#include <hipcub/hipcub.hpp>

#include <cmath>

#include "pair_core.h"

namespace csplat {

namespace {

using namespace pair;

struct Launch {
    dim3 grid;
    hipStream_t st;
    const float *gs;
    int n, n_tiles;
    const float *c, *r;
    int q;
    EvalParams p;
    Part part;
    float mu_max;
    const float *cull;
    unsigned long long *chunk_count;
    int S;
    EvalOut out;
    const int32_t *perm;
};

template <int M, bool FULL, bool BALL, bool CULL>
void launch_pair(const Launch &L)
{
    constexpr int QPL = FULL ? kQplFull : kQplLabels;
    pair_kernel<M, FULL, BALL, QPL, CULL><<<L.grid, kBlock, 0, L.st>>>(L.gs, L.n, L.S, L.n_tiles, L.c, L.r,
                                                                       L.q, L.p, L.part, L.mu_max, L.cull,
                                                                       L.chunk_count);
}

template <int M>
void launch_m(csplat_ctx *ctx, bool full, bool ball, bool cull, const Launch &L)
{
    if (L.n > 0) {
        timing_begin(ctx);
        if (full && ball) {
            if (cull) launch_pair<M, true, true, true>(L);
            else launch_pair<M, true, true, false>(L);
        } else if (full) {
            launch_pair<M, true, false, false>(L);
        } else if (ball) {
            if (cull) launch_pair<M, false, true, true>(L);
            else launch_pair<M, false, true, false>(L);
        } else {
            if (cull) launch_pair<M, false, false, true>(L);
            else launch_pair<M, false, false, false>(L);
        }
        timing_end(ctx);
    }
    const unsigned cb = (unsigned)(((int64_t)L.q * M + 255) / 256);
    if (full) combine_kernel<M, true><<<cb, 256, 0, L.st>>>(L.q, L.S, L.p, L.part, L.out, L.perm);
    else combine_kernel<M, false><<<cb, 256, 0, L.st>>>(L.q, L.S, L.p, L.part, L.out, L.perm);
}

__device__ inline uint32_t spread3(uint32_t v)  // 10 bits -> every third bit
{
    v &= 0x3FF;
    v = (v | (v << 16)) & 0x030000FF;
    v = (v | (v << 8)) & 0x0300F00F;
    v = (v | (v << 4)) & 0x030C30C3;
    v = (v | (v << 2)) & 0x09249249;
    return v;
}

// Morton code of each query centre on the scene's quantisation grid.
__global__ void query_code_kernel(int q, const float *__restrict__ c, float3 lo, float3 scale,
                                  uint32_t *__restrict__ code, int32_t *__restrict__ idx)
{
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= q) return;
    const float fx = (c[3 * j] - lo.x) * scale.x, fy = (c[3 * j + 1] - lo.y) * scale.y,
                fz = (c[3 * j + 2] - lo.z) * scale.z;
    const uint32_t ix = (uint32_t)fminf(fmaxf(fx, 0.f), 1023.f), iy = (uint32_t)fminf(fmaxf(fy, 0.f), 1023.f),
                   iz = (uint32_t)fminf(fmaxf(fz, 0.f), 1023.f);
    code[j] = spread3(ix) | (spread3(iy) << 1) | (spread3(iz) << 2);
    idx[j] = j;
}

__global__ void query_gather_kernel(int q, const int32_t *__restrict__ perm, const float *__restrict__ c,
                                    const float *__restrict__ r, float *__restrict__ sc, float *__restrict__ sr)
{
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= q) return;
    const int i = perm[j];
    sc[3 * j] = c[3 * i];
    sc[3 * j + 1] = c[3 * i + 1];
    sc[3 * j + 2] = c[3 * i + 2];
    sr[j] = r[i];
}

}  // namespace

csplat_status sort_queries(csplat_ctx *ctx, const csplat_scene *sc, int q, const float *centers,
                           const float *radii, SortedQueries *out)
{
    hipStream_t st = ctx->stream;
    size_t tbytes = 0;
    CSPLAT_HIP(hipcub::DeviceRadixSort::SortPairs(nullptr, tbytes, (uint32_t *)nullptr, (uint32_t *)nullptr,
                                                  (int32_t *)nullptr, (int32_t *)nullptr, q, 0, 30, st));
    const size_t qn = (size_t)q;
    const size_t off_code2 = qn * 4, off_idx = qn * 8, off_perm = qn * 12, off_c = qn * 16, off_r = qn * 28,
                 off_cnt = (qn * 32 + 255) & ~(size_t)255, off_tmp = off_cnt + 256;
    hipError_t e = ctx->sortbuf.reserve(off_tmp + tbytes);
    if (e != hipSuccess) return hip_fail(e, "sort workspace");
    char *b = ctx->sortbuf.as<char>();
    uint32_t *code = reinterpret_cast<uint32_t *>(b), *code2 = reinterpret_cast<uint32_t *>(b + off_code2);
    int32_t *idx = reinterpret_cast<int32_t *>(b + off_idx), *perm = reinterpret_cast<int32_t *>(b + off_perm);
    float *sc_c = reinterpret_cast<float *>(b + off_c), *sc_r = reinterpret_cast<float *>(b + off_r);
    auto *counter = reinterpret_cast<unsigned long long *>(b + off_cnt);
    const unsigned qb = (unsigned)((q + 255) / 256);
    query_code_kernel<<<qb, 256, 0, st>>>(q, centers, make_float3(sc->box_lo[0], sc->box_lo[1], sc->box_lo[2]),
                                          make_float3(sc->box_scale[0], sc->box_scale[1], sc->box_scale[2]), code,
                                          idx);
    CSPLAT_HIP(hipGetLastError());
    CSPLAT_HIP(hipcub::DeviceRadixSort::SortPairs(b + off_tmp, tbytes, code, code2, idx, perm, q, 0, 30, st));
    query_gather_kernel<<<qb, 256, 0, st>>>(q, perm, centers, radii, sc_c, sc_r);
    CSPLAT_HIP(hipGetLastError());
    CSPLAT_HIP(zero_words(reinterpret_cast<int32_t *>(counter), 2, st));
    out->c = sc_c;
    out->r = sc_r;
    out->perm = perm;
    out->counter = counter;
    return CSPLAT_OK;
}

csplat_status fp32_eval(csplat_ctx *ctx, const csplat_scene *sc, int64_t q64, const float *centers,
                        const float *radii, const EvalParams &p, const EvalOut &out,
                        bool labels_only)
{
    const int q = (int)q64;
    const int n = (int)sc->n;
    const bool full = !labels_only;
    const bool ball = std::isfinite(p.rn2);
    // culling applies to labels, and to full outputs over a finite ball
    const bool cull = p.cull && n > 0 && sc->cull && (!full || ball);
    const SplitPlan sp = split_plan(ctx_target_blocks(ctx), q, n, full);
    const int S = std::max(sp.S, 1);
    const int M = p.m;
    const size_t words = (size_t)S * q * part_words(M, full);
    if (words > 0) {
        hipError_t e = ctx->partial.reserve(words * 4);
        if (e != hipSuccess) return hip_fail(e, "partial workspace");
    }
    hipStream_t st = ctx->stream;
    Launch L{};
    L.grid = dim3((unsigned)(sp.n_tiles * S));
    L.st = st;
    L.gs = sc->gauss;
    L.n = n;
    L.n_tiles = sp.n_tiles;
    L.c = centers;
    L.r = radii;
    L.q = q;
    L.p = p;
    L.part = part_views(ctx->partial.ptr, S, q, M, full);
    L.mu_max = sc->mu_max;
    L.S = sp.S;
    L.out = out;
    ctx->stats.splits = S;
    ctx->stats.queries_per_lane = sp.qpl;
    ctx->stats.kernel_pairs = (int64_t)q * n;
    ctx->chunk_counter = nullptr;
    if (cull) {
        // evaluate a copy of the queries sorted along the scene's Morton curve
        // (the lanes of a wave then hold nearby queries), scatter the outputs
        SortedQueries sq;
        csplat_status s = sort_queries(ctx, sc, q, centers, radii, &sq);
        if (s != CSPLAT_OK) return s;
        L.c = sq.c;
        L.r = sq.r;
        L.perm = sq.perm;
        L.cull = sc->cull;
        L.chunk_count = sq.counter;
        ctx->chunk_counter = sq.counter;
        ctx->pairs_per_chunk = (int64_t)kCull * 64 * sp.qpl;
    }
    switch (M) {
    case 1: launch_m<1>(ctx, full, ball, cull, L); break;
    case 2: launch_m<2>(ctx, full, ball, cull, L); break;
    case 3: launch_m<3>(ctx, full, ball, cull, L); break;
    case 4: launch_m<4>(ctx, full, ball, cull, L); break;
    case 5: launch_m<5>(ctx, full, ball, cull, L); break;
    case 6: launch_m<6>(ctx, full, ball, cull, L); break;
    case 7: launch_m<7>(ctx, full, ball, cull, L); break;
    case 8: launch_m<8>(ctx, full, ball, cull, L); break;
    default: return fail(CSPLAT_E_INVALID, "m out of range");
    }
    CSPLAT_HIP(hipGetLastError());
    return CSPLAT_OK;
}

}  // namespace csplat
