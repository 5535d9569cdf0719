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
//  * the Gaussian chunks are dealt to S splits (split s takes every S-th
//    chunk) so that small query batches still fill the 256 CUs and every work
//    item gets an even share; partial reductions are merged in a fixed order
//    by combine_kernel (bit-reproducible results).
// Robot bodies are spheres (centre, radius) or ellipsoids (centre, orientation
// quaternion, semi-axes; Eq. 5-6), prepared into records of kBodyFloats.
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
    bool ell;
    const float *cull;
    unsigned long long *chunk_count;
    int S, G, parts;  // splits, splits per work item, partial records per query
    EvalOut out;
    const int32_t *perm;
};

template <int M, bool FULL, bool BALL, bool CULL>
void launch_pair(const Launch &L)
{
    constexpr int QPL = FULL ? kQplFull : kQplLabels;
    if constexpr (QPL == 1 && (BALL || !FULL)) {
        if (L.ell && !uses_tasks<FULL, BALL, QPL, true>())
            pair_kernel<M, FULL, BALL, QPL, CULL, true><<<L.grid, kBlock, 0, L.st>>>(
                L.gs, L.n, L.S, L.G, L.n_tiles, L.c, L.r, L.q, L.p, L.part, L.cull, L.chunk_count);
        else if (L.ell)
            pair_task_kernel<M, FULL, BALL, CULL, true><<<L.grid, task_block<FULL>(), 0, L.st>>>(
                L.gs, L.n, L.S, L.G, L.n_tiles, L.c, L.r, L.q, L.p, L.part, L.cull, L.chunk_count);
        else
            pair_task_kernel<M, FULL, BALL, CULL, false><<<L.grid, task_block<FULL>(), 0, L.st>>>(
                L.gs, L.n, L.S, L.G, L.n_tiles, L.c, L.r, L.q, L.p, L.part, L.cull, L.chunk_count);
    } else {
        if (L.ell)
            pair_kernel<M, FULL, BALL, QPL, CULL, true><<<L.grid, kBlock, 0, L.st>>>(
                L.gs, L.n, L.S, L.G, L.n_tiles, L.c, L.r, L.q, L.p, L.part, L.cull, L.chunk_count);
        else
            pair_kernel<M, FULL, BALL, QPL, CULL, false><<<L.grid, kBlock, 0, L.st>>>(
                L.gs, L.n, L.S, L.G, L.n_tiles, L.c, L.r, L.q, L.p, L.part, L.cull, L.chunk_count);
    }
}

template <int M>
csplat_status launch_m(csplat_ctx *ctx, bool full, bool ball, bool cull, const Launch &L,
                       const std::function<csplat_status()> &gate)
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
    if (gate) {
        const csplat_status s = gate();
        if (s != CSPLAT_OK) return s;
    }
    const unsigned cb = (unsigned)(((int64_t)L.q * M + 255) / 256);
    if (full) combine_kernel<M, true><<<cb, 256, 0, L.st>>>(L.q, L.parts, L.p, L.part, L.out, L.perm);
    else combine_kernel<M, false><<<cb, 256, 0, L.st>>>(L.q, L.parts, L.p, L.part, L.out, L.perm);
    return CSPLAT_OK;
}

// Hilbert key of each query centre on the scene's grid (the scene's curve);
// thread 0 also clears the pair kernel's task counter.
__device__ __forceinline__ uint32_t query_key(const float *__restrict__ c, int stride, float3 lo, float3 scale, int j)
{
    const float *cj = c + (size_t)stride * j;
    const float fx = (cj[0] - lo.x) * scale.x, fy = (cj[1] - lo.y) * scale.y, fz = (cj[2] - lo.z) * scale.z;
    const uint32_t ix = (uint32_t)fminf(fmaxf(fx, 0.f), 1023.f), iy = (uint32_t)fminf(fmaxf(fy, 0.f), 1023.f),
                   iz = (uint32_t)fminf(fmaxf(fz, 0.f), 1023.f);
    return hilbert_key(ix, iy, iz);
}

__global__ void query_code_kernel(int q, const float *__restrict__ c, int stride, float3 lo, float3 scale,
                                  uint32_t *__restrict__ code, int32_t *__restrict__ idx,
                                  unsigned long long *__restrict__ counter)
{
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j == 0) *counter = 0;
    if (j >= q) return;
    code[j] = query_key(c, stride, lo, scale, j);
    idx[j] = j;
}

// Batches of 2 to kSortRuns runs of kSortRun queries are sorted by two
// kernels instead of the library's radix sort (which, at these sizes, is a
// block sort followed by one launch per merge level: about 43 us for 32,768
// keys):
//  1. each run of kSortRun consecutive queries is sorted in LDS (a block
//     radix sort, stable), its keys computed on the way in;
//  2. a query at position p of run r goes to p plus, for every other run,
//     the number of its keys below the query's key (runs after r) or at most
//     equal to it (runs before r): equal keys keep their input order, so the
//     permutation is the one a stable sort of all keys gives.  A block holds
//     64 consecutive queries of one run; its wave w binary-searches runs w,
//     w + 16, ... for all 64 (neighbouring keys share the search's cache
//     lines), the counts are summed in LDS, and the query's record is
//     gathered to its rank.
// Measured on 32,768 keys (kernel averages under the tracer, sort + merge):
// runs of 4,096 keys 25.9 + 5.4 us, 2,048 14.6 + 5.6 us, 1,024 9.4 + 8.4 us
// (8-bit radix passes no better); wall time per evaluation with runs of
// 1,024: the navigation batch 0.995 -> 0.987 ms, the paper-shaped batches of
// 32,768 and 4,096 spheres 0.429 -> 0.412 ms and 0.150 -> 0.147 ms.  Larger
// batches stay with the library, whose merge levels cost less than the
// searches there (262,144 spheres in runs of 4,096: 1.249 against 1.223 ms).
#ifndef CSPLAT_SORT_ITEMS
#define CSPLAT_SORT_ITEMS 4
#endif
constexpr int kSortThreads = 256, kSortItems = CSPLAT_SORT_ITEMS;
constexpr int kSortRun = kSortThreads * kSortItems;  // keys per run
constexpr int kMergeWaves = 16;                       // 1,024 threads per merge block
#ifndef CSPLAT_SORT_MAX_RUNS
#define CSPLAT_SORT_MAX_RUNS 64
#endif
#ifndef CSPLAT_SORT_RADIX_BITS
#define CSPLAT_SORT_RADIX_BITS 4
#endif
constexpr int kSortRuns = CSPLAT_SORT_MAX_RUNS;       // at most kSortRuns / 16 searches per wave and query
constexpr uint32_t kSortPad = 1u << 30;               // above every 30-bit key: padding sorts last

// (the keys are computed here, as query_code_kernel computes them; thread 0
// of block 0 also clears the pair kernel's task counter)
__global__ void __launch_bounds__(kSortThreads) run_sort_kernel(int q, const float *__restrict__ c, int stride,
                                                                float3 lo, float3 scale,
                                                                uint32_t *__restrict__ code2,
                                                                int32_t *__restrict__ idx,
                                                                unsigned long long *__restrict__ counter)
{
    using Sort = hipcub::BlockRadixSort<uint32_t, kSortThreads, kSortItems, int32_t, CSPLAT_SORT_RADIX_BITS>;
    __shared__ typename Sort::TempStorage tmp;
    if (blockIdx.x == 0 && threadIdx.x == 0) *counter = 0;
    const int base = blockIdx.x * kSortRun + (int)threadIdx.x * kSortItems;  // blocked arrangement
    uint32_t k[kSortItems];
    int32_t v[kSortItems];
#pragma unroll
    for (int i = 0; i < kSortItems; ++i) {
        const int j = base + i;
        k[i] = j < q ? query_key(c, stride, lo, scale, j) : kSortPad;
        v[i] = j;
    }
    Sort(tmp).Sort(k, v, 0, 31);  // 31 bits: the padding's key among them
#pragma unroll
    for (int i = 0; i < kSortItems; ++i)
        if (base + i < q) {  // the run's real keys fill its first positions
            code2[base + i] = k[i];
            idx[base + i] = v[i];
        }
}

// (each query's record is gathered to its rank here: centre and radius, or
// the 16-float body record when sc_r is NULL)
__global__ void __launch_bounds__(64 * kMergeWaves) run_merge_kernel(int q, int n_runs,
                                                                     const uint32_t *__restrict__ code2,
                                                                     const int32_t *__restrict__ idx,
                                                                     int32_t *__restrict__ perm,
                                                                     const float *__restrict__ src_c,
                                                                     const float *__restrict__ src_r,
                                                                     float *__restrict__ sc_c,
                                                                     float *__restrict__ sc_r)
{
    __shared__ int s_cnt[kMergeWaves][64];
    const int lane = (int)(threadIdx.x & 63u), w = (int)(threadIdx.x >> 6);
    const int g = blockIdx.x * 64 + lane;  // position in the run-sorted array
    const int gg = g < q ? g : q - 1;
    const int r = gg / kSortRun;
    const uint32_t key = code2[gg];
    int cnt = 0;
    for (int x = w; x < n_runs; x += kMergeWaves) {
        if (x == r) {
            cnt += gg - r * kSortRun;
            continue;
        }
        const uint32_t *run = code2 + (size_t)x * kSortRun;
        int lo = 0, hi = min(kSortRun, q - x * kSortRun);
        const bool upper = x < r;  // runs before r: keys <= key go first
        while (lo < hi) {
            const int mid = (lo + hi) >> 1;
            const uint32_t km = run[mid];
            if (upper ? km <= key : km < key) lo = mid + 1;
            else hi = mid;
        }
        cnt += lo;
    }
    s_cnt[w][lane] = cnt;
    __syncthreads();
    if (w == 0 && g < q) {
        int rank = 0;
#pragma unroll
        for (int k = 0; k < kMergeWaves; ++k) rank += s_cnt[k][lane];
        const int i = idx[g];
        perm[rank] = i;
        if (sc_r) {
            sc_c[3 * rank] = src_c[3 * i];
            sc_c[3 * rank + 1] = src_c[3 * i + 1];
            sc_c[3 * rank + 2] = src_c[3 * i + 2];
            sc_r[rank] = src_r[i];
        } else {
            const float4 *src = reinterpret_cast<const float4 *>(src_c) + (size_t)i * (kBodyFloats / 4);
            float4 *dst = reinterpret_cast<float4 *>(sc_c) + (size_t)rank * (kBodyFloats / 4);
#pragma unroll
            for (int k = 0; k < kBodyFloats / 4; ++k) dst[k] = src[k];
        }
    }
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

// Ellipsoid records in sorted order: one float4 of a record per thread.
__global__ void body_gather_kernel(int q, const int32_t *__restrict__ perm, const float4 *__restrict__ rec,
                                   float4 *__restrict__ out)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (int64_t)q * 4) return;
    const int j = (int)(t >> 2), k = (int)(t & 3);
    out[t] = rec[(size_t)perm[j] * 4 + k];
}

// Ellipsoid records (Eq. 5-6): centre, L = diag(1/a, 1/b, 1/c) R^T with R the
// rotation of the normalised (w, x, y, z) quaternion, so that A = L^T L =
// R diag(1/a^2, 1/b^2, 1/c^2) R^T; qa = (smallest semi-axis)^2 and qk =
// largest / smallest semi-axis for the reach bound, both rounded up.
// Computed in double, stored in float32.
__global__ void body_prep_kernel(int q, const float *__restrict__ centers, const float *__restrict__ quats,
                                 const float *__restrict__ axes, float *__restrict__ rec)
{
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= q) return;
    double w = quats[4 * j], x = quats[4 * j + 1], y = quats[4 * j + 2], z = quats[4 * j + 3];
    const double inv = 1.0 / sqrt(w * w + x * x + y * y + z * z);
    w *= inv, x *= inv, y *= inv, z *= inv;
    const double R[3][3] = {{1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)},
                            {2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)},
                            {2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)}};
    const double a[3] = {axes[3 * j], axes[3 * j + 1], axes[3 * j + 2]};
    float *o = rec + (size_t)kBodyFloats * j;
    o[0] = centers[3 * j];
    o[1] = centers[3 * j + 1];
    o[2] = centers[3 * j + 2];
    for (int k = 0; k < 3; ++k)      // row k of L: column k of R over a_k
        for (int c = 0; c < 3; ++c) o[3 + 3 * k + c] = (float)(R[c][k] / a[k]);
    const double amin = fmin(a[0], fmin(a[1], a[2])), amax = fmax(a[0], fmax(a[1], a[2]));
    o[12] = (float)(amin * amin * (1.0 + 1e-6));
    o[13] = (float)(amax / amin * (1.0 + 1e-6));
    o[14] = 0.f;
    o[15] = 0.f;
}

}  // namespace

csplat_status sort_queries(csplat_ctx *ctx, const csplat_scene *sc, int q, const float *centers,
                           const float *radii, SortedQueries *out)
{
    return sort_bodies(ctx, sc, q, centers, radii, false, out);
}

namespace {
// Layout of the sort workspace: keys, their sorted copy, indices, the
// permutation, the sorted records, a counter, then the radix-sort scratch.
struct SortLayout {
    size_t off_code2, off_idx, off_perm, off_c, off_r, off_cnt, off_tmp, tbytes;
    size_t total() const { return off_tmp + tbytes; }
};

csplat_status sort_layout(int q, bool ell, hipStream_t st, SortLayout &L)
{
    L.tbytes = 0;
    CSPLAT_HIP(hipcub::DeviceRadixSort::SortPairs(nullptr, L.tbytes, (uint32_t *)nullptr, (uint32_t *)nullptr,
                                                  (int32_t *)nullptr, (int32_t *)nullptr, q, 0, 30, st));
    const size_t qn = (size_t)q;
    const size_t rec_bytes = ell ? qn * kBodyFloats * 4 : qn * 16;  // sorted records, or centres + radii
    L.off_code2 = qn * 4, L.off_idx = qn * 8, L.off_perm = qn * 12, L.off_c = (qn * 16 + 255) & ~(size_t)255;
    L.off_r = L.off_c + qn * 12, L.off_cnt = (L.off_c + rec_bytes + 255) & ~(size_t)255;
    L.off_tmp = L.off_cnt + 256;
    return CSPLAT_OK;
}
}  // namespace

csplat_status sort_workspace_bytes(int q, bool ell, hipStream_t st, size_t *bytes)
{
    SortLayout L;
    csplat_status s = sort_layout(q, ell, st, L);
    if (s != CSPLAT_OK) return s;
    *bytes = (L.total() + 255) & ~(size_t)255;
    return CSPLAT_OK;
}

csplat_status sort_bodies(csplat_ctx *ctx, const csplat_scene *sc, int q, const float *centers,
                          const float *radii, bool ell, SortedQueries *out, const Workspace *ws)
{
    hipStream_t st = ctx->stream;
    SortLayout Ly;
    csplat_status ls = sort_layout(q, ell, st, Ly);
    if (ls != CSPLAT_OK) return ls;
    size_t tbytes = Ly.tbytes;
    const size_t off_code2 = Ly.off_code2, off_idx = Ly.off_idx, off_perm = Ly.off_perm, off_c = Ly.off_c,
                 off_r = Ly.off_r, off_cnt = Ly.off_cnt, off_tmp = Ly.off_tmp;
    char *b = nullptr;
    if (ws) {
        if (ws->bytes < Ly.total()) return fail(CSPLAT_E_INVALID, "sort workspace: supplied memory too small");
        b = ws->base;
    } else {
        hipError_t e = ctx->sortbuf.reserve(Ly.total());
        if (e != hipSuccess) return hip_fail(e, "sort workspace");
        b = ctx->sortbuf.as<char>();
    }
    uint32_t *code = reinterpret_cast<uint32_t *>(b), *code2 = reinterpret_cast<uint32_t *>(b + off_code2);
    int32_t *idx = reinterpret_cast<int32_t *>(b + off_idx), *perm = reinterpret_cast<int32_t *>(b + off_perm);
    float *sc_c = reinterpret_cast<float *>(b + off_c), *sc_r = reinterpret_cast<float *>(b + off_r);
    auto *counter = reinterpret_cast<unsigned long long *>(b + off_cnt);
    const unsigned qb = (unsigned)((q + 255) / 256);
    const int stride = ell ? kBodyFloats : 3;
    const float3 lo = make_float3(sc->box_lo[0], sc->box_lo[1], sc->box_lo[2]);
    const float3 scale = make_float3(sc->box_scale[0], sc->box_scale[1], sc->box_scale[2]);
    if (q > kSortRun && q <= kSortRuns * kSortRun) {
        // keys computed by the run sort, records gathered by the merge
        const int n_runs = (q + kSortRun - 1) / kSortRun;
        run_sort_kernel<<<(unsigned)n_runs, kSortThreads, 0, st>>>(q, centers, stride, lo, scale, code2, idx, counter);
        CSPLAT_HIP(hipGetLastError());
        run_merge_kernel<<<(unsigned)((q + 63) / 64), 64 * kMergeWaves, 0, st>>>(
            q, n_runs, code2, idx, perm, centers, ell ? nullptr : radii, sc_c, ell ? nullptr : sc_r);
        CSPLAT_HIP(hipGetLastError());
    } else {
        query_code_kernel<<<qb, 256, 0, st>>>(q, centers, stride, lo, scale, code, idx, counter);
        CSPLAT_HIP(hipGetLastError());
        CSPLAT_HIP(hipcub::DeviceRadixSort::SortPairs(b + off_tmp, tbytes, code, code2, idx, perm, q, 0, 30, st));
        if (ell)
            body_gather_kernel<<<(unsigned)(((size_t)q * 4 + 255) / 256), 256, 0, st>>>(
                q, perm, reinterpret_cast<const float4 *>(centers), reinterpret_cast<float4 *>(sc_c));
        else
            query_gather_kernel<<<qb, 256, 0, st>>>(q, perm, centers, radii, sc_c, sc_r);
        CSPLAT_HIP(hipGetLastError());
    }
    out->c = sc_c;
    out->r = ell ? nullptr : sc_r;
    out->perm = perm;
    out->counter = counter;
    return CSPLAT_OK;
}

csplat_status prepare_bodies(csplat_ctx *ctx, int q, const float *centers, const float *quats, const float *axes,
                             float *rec)
{
    CSPLAT_HIP(prepare_bodies_on(ctx->stream, q, centers, quats, axes, rec));
    return CSPLAT_OK;
}

hipError_t prepare_bodies_on(hipStream_t st, int q, const float *centers, const float *quats, const float *axes,
                             float *rec)
{
    if (q <= 0) return hipSuccess;
    body_prep_kernel<<<(unsigned)((q + 255) / 256), 256, 0, st>>>(q, centers, quats, axes, rec);
    return hipGetLastError();
}

namespace {
// pairs of a pass over the unresolved queries below which the minimum search
// finishes them with one dense pass
constexpr double kDenseMinPairs = 2147483648.0;  // 2^31

template <int M>
csplat_status min_search(csplat_ctx *ctx, const csplat_scene *sc, int q, const float *c, const float *r,
                         const int32_t *perm, bool cull, unsigned long long *counter, const EvalParams &p,
                         const EvalOut &out, const std::function<csplat_status()> &gate)
{
    hipStream_t st = ctx->stream;
    const int n = (int)sc->n;
    const bool want_count = out.label || out.count;
    const size_t qn = (size_t)q;
    // search state, lists and gathered queries in the min workspace
    size_t sel_bytes = 0;
    CSPLAT_HIP(hipcub::DeviceSelect::Flagged(nullptr, sel_bytes, hipcub::CountingInputIterator<int32_t>(0),
                                             (const uint8_t *)nullptr, (int32_t *)nullptr, (int32_t *)nullptr, q,
                                             st));
    auto al = [](size_t b) { return (b + 255) & ~(size_t)255; };
    const size_t o_mt = 0, o_thr = o_mt + al(qn * M * 4), o_flag = o_thr + al(qn * 4), o_list = o_flag + al(qn),
                 o_nl = o_list + al(qn * 4), o_cc = o_nl + 256, o_rr = o_cc + al(qn * 12), o_tt = o_rr + al(qn * 4),
                 o_sel = o_tt + al(qn * 4), total = o_sel + al(sel_bytes);
    hipError_t e = ctx->minbuf.reserve(total);
    if (e != hipSuccess) return hip_fail(e, "minimum-search workspace");
    char *b = ctx->minbuf.as<char>();
    float *st_mt = reinterpret_cast<float *>(b + o_mt), *st_thr = reinterpret_cast<float *>(b + o_thr);
    uint8_t *flag = reinterpret_cast<uint8_t *>(b + o_flag);
    int32_t *list = reinterpret_cast<int32_t *>(b + o_list), *n_list = reinterpret_cast<int32_t *>(b + o_nl);
    float *cc = reinterpret_cast<float *>(b + o_cc), *rr = reinterpret_cast<float *>(b + o_rr),
          *tt = reinterpret_cast<float *>(b + o_tt);
    void *sel_tmp = b + o_sel;
    float total_ms = 0.f;
    // one pass of the walk over nq queries (thr: their thresholds, NULL = 1;
    // culled: skip what lies beyond the thresholds' reach)
    auto pass = [&](bool first, int nq, const float *pc, const float *pr, const float *pt, Part &part, int &S,
                    bool culled) {
        SplitPlan sp = split_plan(ctx_target_blocks(ctx), nq, n, false, false, false, !culled);
        S = std::max(sp.S, 1);
        const size_t words = (size_t)S * nq * M * (first && want_count ? 2 : 1);
        hipError_t pe = ctx->partial.reserve(words * 4);
        if (pe != hipSuccess) return hip_fail(pe, "partial workspace");
        char *pb = ctx->partial.as<char>();
        part = Part{};
        part.cnt = reinterpret_cast<int32_t *>(pb);
        part.mt = reinterpret_cast<float *>(pb + (first && want_count ? (size_t)S * nq * M * 4 : 0));
        if (n == 0) return CSPLAT_OK;
        const dim3 grid((unsigned)(sp.n_tiles * S));
        if (ctx->timing) (void)hipEventRecord(ctx->ev0, st);
        if (first && want_count) {
            if (culled) pair_min_kernel<M, true, true><<<grid, kBlock, 0, st>>>(sc->gauss, n, S, sp.n_tiles, pc, pr, pt, nq, p, part, sc->cull, counter);
            else pair_min_kernel<M, true, false><<<grid, kBlock, 0, st>>>(sc->gauss, n, S, sp.n_tiles, pc, pr, pt, nq, p, part, sc->cull, counter);
        } else {
            if (culled) pair_min_kernel<M, false, true><<<grid, kBlock, 0, st>>>(sc->gauss, n, S, sp.n_tiles, pc, pr, pt, nq, p, part, sc->cull, counter);
            else pair_min_kernel<M, false, false><<<grid, kBlock, 0, st>>>(sc->gauss, n, S, sp.n_tiles, pc, pr, pt, nq, p, part, sc->cull, counter);
        }
        CSPLAT_HIP(hipGetLastError());
        if (ctx->timing) (void)hipEventRecord(ctx->ev1, st);
        if (first) ctx->stats.splits = S;
        return CSPLAT_OK;
    };
    auto pass_ms = [&]() {
        if (!ctx->timing || n == 0) return CSPLAT_OK;
        float ms = 0.f;
        CSPLAT_HIP(hipEventSynchronize(ctx->ev1));
        CSPLAT_HIP(hipEventElapsedTime(&ms, ctx->ev0, ctx->ev1));
        total_ms += ms;
        return CSPLAT_OK;
    };
    Part part;
    int S = 0;
    csplat_status s = pass(true, q, c, r, nullptr, part, S, cull);
    if (s != CSPLAT_OK) return s;
    s = pass_ms();
    if (s != CSPLAT_OK) return s;
    if (gate) {  // nothing that writes an output is queued before the input check passed
        s = gate();
        if (s != CSPLAT_OK) return s;
    }
    const unsigned qb = (unsigned)((q + 255) / 256);
    const int Sf = n > 0 ? S : 0;
    if (want_count)
        min_first_combine_kernel<M, true><<<qb, 256, 0, st>>>(q, Sf, p, part, r, perm, out.label, out.count, st_mt,
                                                              st_thr, flag);
    else
        min_first_combine_kernel<M, false><<<qb, 256, 0, st>>>(q, Sf, p, part, r, perm, nullptr, nullptr, st_mt,
                                                               st_thr, flag);
    CSPLAT_HIP(hipGetLastError());
    int passes = 1;
    for (; n > 0; ++passes) {
        CSPLAT_HIP(hipcub::DeviceSelect::Flagged(sel_tmp, sel_bytes, hipcub::CountingInputIterator<int32_t>(0), flag,
                                                 list, n_list, q, st));
        int nl = 0;
        CSPLAT_HIP(hipMemcpyAsync(&nl, n_list, sizeof(int), hipMemcpyDeviceToHost, st));
        CSPLAT_HIP(hipStreamSynchronize(st));
        if (nl == 0) break;
        // every pass either resolves a query or quadruples its threshold; 64
        // passes cover any float32 threshold
        if (passes >= 64) return fail(CSPLAT_E_DEVICE, "minimum search: thresholds did not converge");
        // A short list (the queries far from every Gaussian, whose thresholds
        // grow four times a pass) is finished by one dense pass: every pair,
        // no threshold, which resolves each listed query (a culled pass over a
        // few queries costs about as much as a dense one over a few hundred:
        // passes of 48 and 6 queries took 0.2 ms each on the precision
        // workload).  A minimum is order-free, so the results keep their bits.
        const bool dense = (double)nl * (double)n <= kDenseMinPairs;
        const unsigned lb = (unsigned)((nl + 255) / 256);
        min_gather_kernel<M><<<lb, 256, 0, st>>>(nl, list, c, r, st_mt, st_thr, cc, rr, tt, dense);
        CSPLAT_HIP(hipGetLastError());
        s = pass(false, nl, cc, rr, tt, part, S, cull && !dense);
        if (s != CSPLAT_OK) return s;
        s = pass_ms();
        if (s != CSPLAT_OK) return s;
        min_next_combine_kernel<M><<<(unsigned)((nl + 3) / 4), 256, 0, st>>>(nl, S, part, list, r, st_thr, st_mt,
                                                                            flag);
        CSPLAT_HIP(hipGetLastError());
        if (dense) {
            ++passes;
            break;
        }
    }
    min_output_kernel<M><<<qb, 256, 0, st>>>(q, p.m, r, perm, st_mt, out.min);
    CSPLAT_HIP(hipGetLastError());
    ctx->stats.min_passes = passes;
    if (ctx->timing) {
        ctx->timed = true;
        ctx->timed_ms = total_ms;
    }
    return CSPLAT_OK;
}
}  // namespace

csplat_status fp32_min_eval(csplat_ctx *ctx, const csplat_scene *sc, int64_t q64, const float *centers,
                            const float *radii, const EvalParams &p, const EvalOut &out,
                            const std::function<csplat_status()> &gate)
{
    const int q = (int)q64;
    const int n = (int)sc->n;
    const bool cull = p.cull && n > 0 && sc->cull;
    ctx->stats.queries_per_lane = 1;
    ctx->stats.kernel_pairs = (int64_t)q * n;
    ctx->chunk_counter = nullptr;
    const float *c = centers, *r = radii;
    const int32_t *perm = nullptr;
    unsigned long long *counter = nullptr;
    if (cull) {
        SortedQueries sq;
        csplat_status s = sort_queries(ctx, sc, q, centers, radii, &sq);
        if (s != CSPLAT_OK) return s;
        c = sq.c;
        r = sq.r;
        perm = sq.perm;
        counter = sq.counter;
        ctx->chunk_counter = sq.counter;
        ctx->pairs_per_chunk = kFine;  // the counter counts (query, sub-chunk) tasks of every pass
    }
    switch (p.m) {
    case 1: return min_search<1>(ctx, sc, q, c, r, perm, cull, counter, p, out, gate);
    case 2: return min_search<2>(ctx, sc, q, c, r, perm, cull, counter, p, out, gate);
    case 3: return min_search<3>(ctx, sc, q, c, r, perm, cull, counter, p, out, gate);
    case 4: return min_search<4>(ctx, sc, q, c, r, perm, cull, counter, p, out, gate);
    case 5: return min_search<5>(ctx, sc, q, c, r, perm, cull, counter, p, out, gate);
    case 6: return min_search<6>(ctx, sc, q, c, r, perm, cull, counter, p, out, gate);
    case 7: return min_search<7>(ctx, sc, q, c, r, perm, cull, counter, p, out, gate);
    case 8: return min_search<8>(ctx, sc, q, c, r, perm, cull, counter, p, out, gate);
    default: return fail(CSPLAT_E_INVALID, "m out of range");
    }
}

csplat_status fp32_eval(csplat_ctx *ctx, const csplat_scene *sc, int64_t q64, const float *centers,
                        const float *radii, const EvalParams &p, const EvalOut &out,
                        bool labels_only, bool ell, const std::function<csplat_status()> &gate,
                        const Workspace *ws)
{
    // the minimum over every kept Gaussian (labels optional): threshold passes
    // of the task walk instead of the dense walk
    if (!ws && !ell && !std::isfinite(p.rn2) && out.min && !out.softmin && !out.cost && !out.nbr)
        return fp32_min_eval(ctx, sc, q64, centers, radii, p, out, gate);
    const int q = (int)q64;
    const int n = (int)sc->n;
    const bool full = !labels_only;
    const bool ball = std::isfinite(p.rn2);
    // culling applies to labels, and to full outputs over a finite ball
    const bool cull = p.cull && n > 0 && sc->cull && (!full || ball);
    SplitPlan sp = split_plan(ctx_target_blocks(ctx), q, n, full, ball, ell, !cull);
    const int M = p.m;
    // the sorted queries and the partials: the context's buffers, or the
    // caller's workspace (sort first, then as many splits as fit)
    size_t sort_bytes = 0;
    void *part_base = nullptr;
    if (ws) {
        if (cull) {
            csplat_status s = sort_workspace_bytes(q, ell, ctx->stream, &sort_bytes);
            if (s != CSPLAT_OK) return s;
        }
        const size_t per_part = (size_t)q * part_words(M, full) * 4;
        const size_t avail = ws->bytes > sort_bytes ? ws->bytes - sort_bytes : 0;
        const size_t fit = per_part ? avail / per_part : 0;
        if (fit < 1) return fail(CSPLAT_E_INVALID, "workspace too small for one split of the partials");
        if ((size_t)sp.parts > fit) {
            sp.parts = (int)fit;
            sp.S = sp.parts * sp.G;
        }
        part_base = ws->base + sort_bytes;
    }
    const int S = std::max(sp.S, 1);
    const int parts = std::max(sp.parts, 1);
    const size_t words = (size_t)parts * q * part_words(M, full);
    if (!ws && words > 0) {
        hipError_t e = ctx->partial.reserve(words * 4);
        if (e != hipSuccess) return hip_fail(e, "partial workspace");
        part_base = ctx->partial.ptr;
    }
    hipStream_t st = ctx->stream;
    Launch L{};
    L.grid = dim3((unsigned)(sp.n_tiles * parts));
    L.st = st;
    L.gs = sc->gauss;
    L.n = n;
    L.n_tiles = sp.n_tiles;
    L.c = centers;
    L.r = radii;
    L.q = q;
    L.p = p;
    L.part = part_views(part_base, parts, q, M, full);
    L.ell = ell;
    L.S = sp.S;
    L.G = sp.G;
    L.parts = sp.parts;  // 0 for an empty scene: the combine then folds nothing
    L.out = out;
    ctx->stats.splits = S;
    ctx->stats.queries_per_lane = sp.qpl;
    ctx->stats.kernel_pairs = (int64_t)q * n;
    ctx->chunk_counter = nullptr;
    if (cull) {
        // evaluate a copy of the queries sorted along the scene's Hilbert curve
        // (the lanes of a wave then hold nearby queries), scatter the outputs
        SortedQueries sq;
        Workspace sw{ws ? ws->base : nullptr, sort_bytes};
        csplat_status s = sort_bodies(ctx, sc, q, centers, radii, ell, &sq, ws ? &sw : nullptr);
        if (s != CSPLAT_OK) return s;
        L.c = sq.c;
        L.r = sq.r;
        L.perm = sq.perm;
        L.cull = sc->cull;
        L.chunk_count = sq.counter;
        ctx->chunk_counter = sq.counter;
        // the counter counts visited (wave, chunk) steps, or in the task
        // walk (query, sub-chunk) tasks
        const bool tasks = sp.qpl == 1 && (!full || (ball && (!ell || CSPLAT_ELL_FULL_TASKS)));
        ctx->pairs_per_chunk = tasks ? (int64_t)kFine : (int64_t)kCull * 64 * sp.qpl;
    }
    csplat_status s = CSPLAT_OK;
    switch (M) {
    case 1: s = launch_m<1>(ctx, full, ball, cull, L, gate); break;
    case 2: s = launch_m<2>(ctx, full, ball, cull, L, gate); break;
    case 3: s = launch_m<3>(ctx, full, ball, cull, L, gate); break;
    case 4: s = launch_m<4>(ctx, full, ball, cull, L, gate); break;
    case 5: s = launch_m<5>(ctx, full, ball, cull, L, gate); break;
    case 6: s = launch_m<6>(ctx, full, ball, cull, L, gate); break;
    case 7: s = launch_m<7>(ctx, full, ball, cull, L, gate); break;
    case 8: s = launch_m<8>(ctx, full, ball, cull, L, gate); break;
    default: return fail(CSPLAT_E_INVALID, "m out of range");
    }
    if (s != CSPLAT_OK) return s;
    CSPLAT_HIP(hipGetLastError());
    return CSPLAT_OK;
}

}  // namespace csplat
