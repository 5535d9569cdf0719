// Device code of the float32 pair path shared by the evaluation kernels and
// the serving step kernels (one definition, identical arithmetic).
//
// Layout and mapping on gfx950:
//  * 256 lanes (4 waves) per block, a few queries per lane; each query's
//    centre, r^2 and accumulators live in VGPRs;
//  * the Gaussian records are wave-uniform: every lane of a wave needs the
//    same Gaussian at the same time, so they are fetched with scalar loads
//    into SGPRs and used directly as VALU operands (no LDS round trip, no
//    VGPRs spent on them, no bank conflicts);
//  * the Gaussian list is cut into `splits` contiguous ranges so that small
//    query batches still fill the 256 CUs; partial reductions are merged in a
//    fixed order (bit-reproducible results).
#pragma once

#include <algorithm>
#include <cmath>

#include "internal.h"

namespace csplat {
namespace pair {

constexpr int kBlock = 256;
// Threads of a full-output task block (its waves' splits are folded into
// one partial record; labels and the wave walk keep kBlock).  Eight waves
// (512) halve the partials again but measured slower: 0.893 against 0.868 ms
// on the navigation batch, 23.2 against 21.7 ms on the manipulation batch.
#ifndef CSPLAT_FULL_TASK_BLOCK
#define CSPLAT_FULL_TASK_BLOCK 256
#endif
constexpr int kFullTaskBlock = CSPLAT_FULL_TASK_BLOCK;
static_assert(kFullTaskBlock == 256 || kFullTaskBlock == 512, "four or eight waves per full-output task block");
template <bool FULL>
constexpr int task_block()
{
    return FULL ? kFullTaskBlock : kBlock;
}
constexpr int kChunk = 512;  // Gaussians per first-level softmin/cost sum
constexpr int kCull = 64;    // Gaussians per culling chunk (consecutive on the curve)
constexpr int kPiece = kChunk / kCull;  // culling chunks per first-level sum
constexpr int kCullFloats = 8;  // per chunk: centre (3), radius, largest scale, 0 0 0
// relative widening of the culling thresholds: far above float32 rounding, so
// no pair the float32 test would accept is ever culled
constexpr float kCullMargin = 1.0000153f;  // 1 + 2^-16
// Launch-shape constants (overridable at build time for tuning sweeps).
#ifndef CSPLAT_UNROLL
#define CSPLAT_UNROLL 4
#endif
#ifndef CSPLAT_QPL_FULL
#define CSPLAT_QPL_FULL 1
#endif
#ifndef CSPLAT_QPL_LABELS
#define CSPLAT_QPL_LABELS 1  // 1: the task walk; 2: the wave walk with two queries per lane
#endif
#ifndef CSPLAT_PIPELINE
#define CSPLAT_PIPELINE 0
#endif
// Optional register cap: at least N waves of the pair kernels per SIMD.
#ifdef CSPLAT_WAVES_PER_EU
#define CSPLAT_OCCUPANCY __attribute__((amdgpu_waves_per_eu(CSPLAT_WAVES_PER_EU)))
#else
#define CSPLAT_OCCUPANCY
#endif
// The task walk (full outputs over a ball) at 5 or more waves per SIMD: its
// vector loads want the latency hiding.  Records are loaded four at a time
// with one conservatism value and two at a time with more, where four would
// spill.  With three values the kernel fits in 78 VGPRs and runs 6 waves
// (LDS holds six of its blocks per CU).  Measured on MI355X: navigation
// workload, m = 3: no cap 1.25 ms, 4 waves 1.10, later 4 waves 1.002 ms and
// 5 waves 0.987 ms, now 6 waves 0.906 ms, 7 waves (partial rows without bank
// padding, 32 spilled bytes) 0.92-0.93; one value (manipulation 21.6 ms,
// serving 633 requests/s): 6 waves with 24 spilled bytes 22.2 ms and 599,
// two records per group at 8 waves 22.1 ms and 585.
#ifndef CSPLAT_TASK_WAVES_PER_EU
#define CSPLAT_TASK_WAVES_PER_EU 5
#endif
#ifndef CSPLAT_TASK_UNROLL
#define CSPLAT_TASK_UNROLL 0  // 0: by the number of conservatism values
#endif
// Full outputs for ellipsoids over a ball: task walk (1) or wave walk (0).
// The tabletop workload puts 88% of the pairs the task walk evaluates inside
// the ball, so the wave walk's masked lanes cost little there, while the
// task walk's per-lane record loads (48 B per pair against ~50 operations)
// approach the vector-memory return rate (measured: 5.2 ms wave walk, 5.95
// ms task walk; 5.74 ms after the task walk's register and load-order work).
#ifndef CSPLAT_ELL_FULL_TASKS
#define CSPLAT_ELL_FULL_TASKS 0
#endif
// Work items of the task walk per compute unit (fewer, longer splits keep
// its task queues full; measured: 32 beats 16 and 64).
#ifndef CSPLAT_TASK_BLOCKS_PER_CU
#define CSPLAT_TASK_BLOCKS_PER_CU 32
#endif
constexpr int kUnroll = CSPLAT_UNROLL;       // Gaussians per group of scalar loads
// records per group of loads in a full-output task with M conservatism values
template <int M>
constexpr int task_unroll()
{
    return CSPLAT_TASK_UNROLL > 0 ? CSPLAT_TASK_UNROLL : (M == 1 ? 4 : 2);
}
constexpr int kQplFull = CSPLAT_QPL_FULL;    // queries per lane, all outputs
constexpr int kQplLabels = CSPLAT_QPL_LABELS;  // queries per lane, labels only
constexpr bool kPipeline = CSPLAT_PIPELINE != 0;

__device__ inline float fast_exp2(float x) { return __builtin_amdgcn_exp2f(x); }
__device__ inline float fast_sqrt(float x) { return __builtin_amdgcn_sqrtf(x); }
__device__ inline float fast_log2(float x) { return __builtin_amdgcn_logf(x); }

struct Part {
    int32_t *cnt;  // [split][v][q]
    float *mt;     // running minimum of t = s~^2 * kt
    float *sm;     // sum of 2^(mt - t)
    float *cs;     // sum of the base-2 cost terms
    int32_t *nb;   // [split][q] neighbourhood size
};

// Ball membership and the per-pair metric, with d = mu - c.
//  * Sphere of radius r (Eq. 6 with a = b = c = r): terms in "r^2 units", with
//    D = |d|^2 and V = |M d|^2 = d^T Sigma d,
//      r^2 s^2 = D,  r^2 n sqrt(sigma^2) = 2 n sqrt(V),  r^2 s~^2 = max(0, D - 2 n sqrt(V)).
//  * Ellipsoid A = L^T L with L = diag(1/a, 1/b, 1/c) R^T (Eq. 5-6): e = L d,
//    s^2 = |e|^2 and the gradient of s^2 is 2 A d = 2 L^T e (Eq. 7), so
//    sqrt(sigma^2) = 2 |M L^T e| and s~^2 = max(0, s^2 - 2 n |M L^T e|)
//    (dimensionless: threshold 1).
//
// Each lane holds QPL queries (slot u of lane l in wave w of tile b is query
// (b*kBlock + w*64)*QPL + u*64 + l: a wave holds 64*QPL consecutive queries,
// which after the spatial sort are one compact region),
// so every scalar-loaded Gaussian feeds QPL pairs per lane; the Gaussian loop is
// unrolled by kUnroll (the group's records in scalar loads).  In FULL mode a single branch per
// Gaussian skips the metric when no query of the wave has it in its ball.
template <int M, int QPL>
struct Acc {
    int cnt[QPL][M];
    float mt[QPL][M], sm[QPL][M], cs[QPL][M];   // lane totals
    float cmt[QPL][M], csm[QPL][M], ccs[QPL][M]; // current chunk
    int nb[QPL];
};

// Per-lane query state.  r2, kq: the collision threshold and the factor that
// turns the metric into t = s~^2 * kt (sphere: r^2 and kt / r^2; ellipsoid: 1
// and kt).  qa, qk: the reach-bound constants, the smallest semi-axis squared
// and largest / smallest semi-axis (sphere: r^2 and 1).  L: the ellipsoid's
// matrix diag(1/a) R^T, row-major.
template <int QPL, bool ELL>
struct QState {
    float cx[QPL], cy[QPL], cz[QPL], r2[QPL], kq[QPL], qa[QPL], qk[QPL];
    float L[ELL ? QPL : 1][9];
};

// D: the metric's squared term, W: its variance term (see above), from d
// (L: the body's matrix, ellipsoids only).
template <bool ELL>
__device__ __forceinline__ void metric_dw(const float *__restrict__ gp, const float *L, float dx, float dy,
                                          float dz, float D_sphere, float &D, float &W)
{
    if constexpr (ELL) {
        const float e0 = fmaf(L[2], dz, fmaf(L[1], dy, L[0] * dx));
        const float e1 = fmaf(L[5], dz, fmaf(L[4], dy, L[3] * dx));
        const float e2 = fmaf(L[8], dz, fmaf(L[7], dy, L[6] * dx));
        D = fmaf(e2, e2, fmaf(e1, e1, e0 * e0));
        const float hx = fmaf(L[6], e2, fmaf(L[3], e1, L[0] * e0));  // L^T e = A d
        const float hy = fmaf(L[7], e2, fmaf(L[4], e1, L[1] * e0));
        const float hz = fmaf(L[8], e2, fmaf(L[5], e1, L[2] * e0));
        const float g0 = fmaf(gp[5], hz, fmaf(gp[4], hy, gp[3] * hx));
        const float g1 = fmaf(gp[8], hz, fmaf(gp[7], hy, gp[6] * hx));
        const float g2 = fmaf(gp[11], hz, fmaf(gp[10], hy, gp[9] * hx));
        W = fmaf(g2, g2, fmaf(g1, g1, g0 * g0));
    } else {
        D = D_sphere;
        const float e0 = fmaf(gp[5], dz, fmaf(gp[4], dy, gp[3] * dx));
        const float e1 = fmaf(gp[8], dz, fmaf(gp[7], dy, gp[6] * dx));
        const float e2 = fmaf(gp[11], dz, fmaf(gp[10], dy, gp[9] * dx));
        W = fmaf(e2, e2, fmaf(e1, e1, e0 * e0));
    }
}

template <bool ELL, int QPL>
__device__ __forceinline__ void metric_terms(const float *__restrict__ gp, const QState<QPL, ELL> &Q, int u,
                                             float dx, float dy, float dz, float D_sphere, float &D, float &W)
{
    metric_dw<ELL>(gp, Q.L[ELL ? u : 0], dx, dy, dz, D_sphere, D, W);
}

template <int M, bool FULL, bool BALL, int QPL, bool ELL>
__device__ __forceinline__ void pair_step(const float *__restrict__ gp, const QState<QPL, ELL> &Q,
                                          const EvalParams &p, Acc<M, QPL> &A)
{
    if constexpr (FULL) {
        bool any = !BALL;
        if constexpr (BALL) {
#pragma unroll
            for (int u = 0; u < QPL; ++u) {
                const float dx = gp[0] - Q.cx[u], dy = gp[1] - Q.cy[u], dz = gp[2] - Q.cz[u];
                any |= fmaf(dz, dz, fmaf(dy, dy, dx * dx)) <= p.rn2;
            }
        }
        if (any) {
#pragma unroll
            for (int u = 0; u < QPL; ++u) {
                const float dx = gp[0] - Q.cx[u], dy = gp[1] - Q.cy[u], dz = gp[2] - Q.cz[u];
                const float Db = fmaf(dz, dz, fmaf(dy, dy, dx * dx));
                if (!BALL || Db <= p.rn2) {
                    ++A.nb[u];
                    float D, W;
                    metric_terms<ELL, QPL>(gp, Q, u, dx, dy, dz, Db, D, W);
                    const float sv = fast_sqrt(W);
#pragma unroll
                    for (int v = 0; v < M; ++v) {
                        const float x = fmaf(-p.two_n[v], sv, D);  // (r^2) (s^2 - n sqrt(sigma^2))
                        A.cnt[u][v] += x < Q.r2[u];                  // s~^2 < 1
                        const float t = fmaxf(x, 0.f) * Q.kq[u];
                        // stable log-sum-exp about the running chunk minimum (one exp per pair)
                        const float e = fast_exp2(-fabsf(t - A.cmt[u][v]));
                        const bool lower = t < A.cmt[u][v];
                        A.csm[u][v] = lower ? fmaf(A.csm[u][v], e, 1.f) : A.csm[u][v] + e;
                        A.cmt[u][v] = lower ? t : A.cmt[u][v];
                        A.ccs[u][v] += fast_exp2(fminf(fmaf(t, -p.g1, p.g0), 0.f));
                    }
                }
            }
        }
    } else {
#pragma unroll
        for (int u = 0; u < QPL; ++u) {
            const float dx = gp[0] - Q.cx[u], dy = gp[1] - Q.cy[u], dz = gp[2] - Q.cz[u];
            // labels only: s~^2 < 1  <=>  a |a| < 4 n^2 W  with a = (r^2)(s^2 - 1) (exact rewrite)
            float a, W;
            bool in = true;
            if constexpr (ELL) {
                float D;
                metric_terms<ELL, QPL>(gp, Q, u, dx, dy, dz, 0.f, D, W);
                a = D - 1.f;
                if constexpr (BALL) in = fmaf(dz, dz, fmaf(dy, dy, dx * dx)) <= p.rn2;
            } else {
                a = fmaf(dz, dz, fmaf(dy, dy, fmaf(dx, dx, -Q.r2[u])));
                float D;
                metric_terms<ELL, QPL>(gp, Q, u, dx, dy, dz, 0.f, D, W);
                if constexpr (BALL) in = a + Q.r2[u] <= p.rn2;
            }
            const float aa = a * fabsf(a);
#pragma unroll
            for (int v = 0; v < M; ++v) A.cnt[u][v] += in && (aa < p.four_n2[v] * W);
        }
    }
}

// Culling metadata of one chunk of kCull Gaussians consecutive on the curve: the
// centre of their bounding box, the largest distance of a mean from it and the
// largest scale (all rounded up at load time).
struct ChunkMeta {
    float x, y, z, rad, smax;
};

__device__ __forceinline__ ChunkMeta load_chunk(const float *__restrict__ cull, int ci)
{
    const float4 a = *reinterpret_cast<const float4 *>(cull + (size_t)kCullFloats * ci);
    return ChunkMeta{a.x, a.y, a.z, a.w, cull[(size_t)kCullFloats * ci + 4]};
}

__device__ __forceinline__ float lane_value(float v, int lane)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), lane));
}

// A value equal on every lane, held in a scalar register (the empty asm
// keeps the arithmetic that made it ahead of the read, so the scalar
// register is what later code uses).
__device__ __forceinline__ float wave_uniform(float v)
{
    asm volatile("" : "+v"(v));
    return __builtin_bit_cast(float, __builtin_amdgcn_readfirstlane(__builtin_bit_cast(int, v)));
}

// The metadata held by lane `lane`, as wave-uniform values.
__device__ __forceinline__ ChunkMeta lane_chunk(const ChunkMeta &m, int lane)
{
    return ChunkMeta{lane_value(m.x, lane), lane_value(m.y, lane), lane_value(m.z, lane), lane_value(m.rad, lane),
                     lane_value(m.smax, lane)};
}

// Bounding sphere of every query the wave holds (centre w = middle of their
// bounding box, radius `spread`) and their largest r^2; with `half`, also the
// half extents of that box about w.
template <int QPL>
__device__ __forceinline__ void wave_sphere(const float (&cx)[QPL], const float (&cy)[QPL], const float (&cz)[QPL],
                                            const float (&r2)[QPL], float &wx, float &wy, float &wz, float &spread,
                                            float &r2max, float *half = nullptr)
{
    float lo[3] = {cx[0], cy[0], cz[0]}, hi[3] = {cx[0], cy[0], cz[0]};
    r2max = r2[0];
#pragma unroll
    for (int u = 1; u < QPL; ++u) {
        lo[0] = fminf(lo[0], cx[u]), hi[0] = fmaxf(hi[0], cx[u]);
        lo[1] = fminf(lo[1], cy[u]), hi[1] = fmaxf(hi[1], cy[u]);
        lo[2] = fminf(lo[2], cz[u]), hi[2] = fmaxf(hi[2], cz[u]);
        r2max = fmaxf(r2max, r2[u]);
    }
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            lo[k] = fminf(lo[k], __shfl_xor(lo[k], off));
            hi[k] = fmaxf(hi[k], __shfl_xor(hi[k], off));
        }
        r2max = fmaxf(r2max, __shfl_xor(r2max, off));
    }
    // after the butterflies every lane holds the same values
    wx = wave_uniform(0.5f * (lo[0] + hi[0])), wy = wave_uniform(0.5f * (lo[1] + hi[1]));
    wz = wave_uniform(0.5f * (lo[2] + hi[2])), r2max = wave_uniform(r2max);
    if (half) {
        half[0] = wave_uniform(fmaxf(hi[0] - wx, wx - lo[0]));
        half[1] = wave_uniform(fmaxf(hi[1] - wy, wy - lo[1]));
        half[2] = wave_uniform(fmaxf(hi[2] - wz, wz - lo[2]));
    }
    spread = 0.f;
#pragma unroll
    for (int u = 0; u < QPL; ++u) {
        const float ex = cx[u] - wx, ey = cy[u] - wy, ez = cz[u] - wz;
        spread = fmaxf(spread, sqrtf(fmaf(ez, ez, fmaf(ey, ey, ex * ex))));
    }
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) spread = fmaxf(spread, __shfl_xor(spread, off));
    spread = wave_uniform(spread);
}

// Squared distance of a chunk centre from a point, and the culling test
// d <= (reach + extra) with the relative margin kCullMargin.
__device__ __forceinline__ bool within(const ChunkMeta &m, float x, float y, float z, float reach)
{
    const float ex = m.x - x, ey = m.y - y, ez = m.z - z;
    const float d2 = fmaf(ez, ez, fmaf(ey, ey, ex * ex));
    const float thr = reach * kCullMargin;
    return d2 <= thr * thr;
}

// The culling test of a chunk against a box of centre b and half extents h:
// the distance from the chunk centre to the box at most `reach`, with the
// relative margin kCullMargin.  Every query in the box lies at least that far
// from the chunk centre, so a chunk that fails lies beyond `reach` of them all.
__device__ __forceinline__ bool within_box(const ChunkMeta &m, float bx, float by, float bz, const float *h,
                                           float reach)
{
    const float ex = fmaxf(fabsf(m.x - bx) - h[0], 0.f);
    const float ey = fmaxf(fabsf(m.y - by) - h[1], 0.f);
    const float ez = fmaxf(fabsf(m.z - bz) - h[2], 0.f);
    const float d2 = fmaf(ez, ez, fmaf(ey, ey, ex * ex));
    const float thr = reach * kCullMargin;
    return d2 <= thr * thr;
}

// Walk the chunks split, split + S, split + 2S, ... (< n_chunks) in ascending
// order with two culling levels: (1) a batch of 64 chunks at once, one per
// lane, with `coarse(m)` (a test against the wave's bounding sphere); (2)
// each survivor against every query of the wave with `near(m)`.
// visit(i, lanes) for the i-th chunk of the split when some lane is near,
// with the wave mask of the near lanes.
template <class Coarse, class Near, class Visit>
__device__ __forceinline__ void cull_walk(const float *__restrict__ cull, int n_chunks, int split, int S,
                                          Coarse coarse, Near near, Visit visit)
{
    const int lane = (int)(threadIdx.x & 63u);
    for (int ib = 0; split + ib * S < n_chunks; ib += 64) {
        const int ci = split + (ib + lane) * S;
        ChunkMeta m{0.f, 0.f, 0.f, 0.f, 0.f};
        bool ok = false;
        if (ci < n_chunks) {
            m = load_chunk(cull, ci);
            ok = true;
        }
        const bool pass = ok && coarse(m);
        unsigned long long mask = __ballot(pass);
        while (mask) {
            const int bit = __builtin_ctzll(mask);
            mask &= mask - 1;
            const unsigned long long lanes = __ballot(near(lane_chunk(m, bit)));
            if (!lanes) continue;
            visit(ib + bit, lanes);
        }
    }
}

// ---------------------------------------------------------------------------
// Full outputs over the neighbourhood ball, one query per lane, as tasks.
//
// The 64 queries of a wave spread over a region comparable to the ball, so a
// chunk that some lane needs lies in the ball of only part of the wave: a
// walk that steps every lane through every such chunk leaves most lanes
// masked in the per-pair work.  Here the wave's work is cut into tasks
// (query, sub-chunk of kFine Gaussians), one for each sub-chunk whose
// bounding sphere reaches the query's ball, queued in curve order and run 64
// at a time, one per lane: lane i takes the i-th task, fetches that query's
// state from the lane that owns it and the sub-chunk's records with vector
// loads, and reduces the task's pairs into a partial (the first level of the
// two-level softmin and cost sums).  Each query then folds its tasks'
// partials into its totals in queue order.  Without culling every lane
// queues every sub-chunk of the split for itself: the sub-chunks outside a
// query's ball give empty partials, whose fold changes no bit, so culled and
// dense walks give the same bits.
constexpr int kFine = 16;                // Gaussians per task
constexpr int kFinePer = kCull / kFine;  // sub-chunks per culling chunk
constexpr int kGroup = 16;               // culling chunks per group (the task walk's coarsest level)
constexpr int kGroupDealChunks = 1024;   // chunks per split above which label walks deal whole groups

// The task walk's culling: visit(c, lanes) for each chunk c of split `split`
// (of S) whose bounding sphere reaches some query of the wave, with the mask
// of its near lanes, in ascending order.
//  * Split s takes the chunks s, s + S, ... (< n_chunks) as in cull_walk: 64
//    of them at a time against the wave (`coarse`), then each survivor
//    against every query of the wave (`near`).
//  * Labels with more than kGroupDealChunks chunks per split: split s takes
//    the groups of 16 chunks s, s + S, ..., each with all of its chunks: 64
//    groups at a time against the wave (`coarse`), then the 16 chunks of a
//    surviving group (`coarse` again), then each surviving chunk against
//    every query (`near`).  A walk with a short reach culls nearly every
//    batch, so over a large scene its time goes into the batches: dealt
//    whole groups, the splits of a query tile together scan each group and
//    open each near group once (precision workload: labels 1.39 -> 1.08 ms).
//    Over a small scene the splits are many and short, a query tile's near
//    groups would fall on a few of them, and strided chunks spread its work
//    more evenly (a 200k-Gaussian scene over 64 splits: 0.52 ms with strided
//    chunks, 0.61 with dealt groups).
// With AHEAD the next batch is requested before the current one is tested
// (it holds five more registers).  The group level and AHEAD are compiled in
// with LABELS only (full outputs over a 1 m ball rarely cull a group, and the
// registers they hold would spill the full-output kernel).
template <bool LABELS, class Coarse, class Near, class Visit>
__device__ __forceinline__ void split_walk(const float *__restrict__ groups, const float *__restrict__ chunks,
                                           int n_groups, int n_chunks, int split, int S, Coarse coarse, Near near,
                                           Visit visit)
{
    const int lane = (int)(threadIdx.x & 63u), wv = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    constexpr bool AHEAD = LABELS;
    __shared__ unsigned long long s_near[LABELS ? 1 : kFullTaskBlock / 64][LABELS ? 1 : 64];
    __shared__ int s_near_at[LABELS ? 1 : kFullTaskBlock / 64][LABELS ? 1 : 64];
    const bool by_group = LABELS && n_chunks > kGroupDealChunks * S;
    const int n_units = by_group ? n_groups : n_chunks;
    const int stride = S, first = split;
    const float *meta = by_group ? groups : chunks;
    auto fetch = [&](int ib, ChunkMeta &m) {
        const int u = first + (ib + lane) * stride;
        m = u < n_units ? load_chunk(meta, u) : ChunkMeta{0.f, 0.f, 0.f, 0.f, 0.f};
        return u < n_units;
    };
    ChunkMeta next{0.f, 0.f, 0.f, 0.f, 0.f};
    bool next_ok = false;
    if constexpr (AHEAD) next_ok = fetch(0, next);
    for (int ib = 0; first + ib * stride < n_units; ib += 64) {
        ChunkMeta m;
        bool ok;
        if constexpr (AHEAD) {
            m = next;
            ok = next_ok;
            next_ok = fetch(ib + 64, next);
        } else {
            ok = fetch(ib, m);
        }
        const unsigned long long mask = __ballot(ok && coarse(m));
        // the surviving groups to open, or the batch itself as one (one
        // visit site, so the caller's visit is inlined once)
        unsigned long long gmask = by_group ? mask : 1ull;
        while (gmask) {
            ChunkMeta cm = m;
            unsigned long long cmask = mask;
            int c0 = first + ib * stride, cs = stride;
            if (by_group) {
                // the chunks of group gi: gi*16 <= c < gi*16 + 16, one per lane
                const int gi = first + (ib + __builtin_ctzll(gmask)) * stride;
                c0 = gi * kGroup;
                cs = 1;
                const int c = c0 + lane;
                bool cok = false;
                cm = ChunkMeta{0.f, 0.f, 0.f, 0.f, 0.f};
                if (lane < kGroup && c < n_chunks) {
                    cm = load_chunk(chunks, c);
                    cok = coarse(cm);
                }
                cmask = __ballot(cok);
            }
            gmask &= gmask - 1;
            if constexpr (LABELS) {
                while (cmask) {
                    const int cb = __builtin_ctzll(cmask);
                    cmask &= cmask - 1;
                    const unsigned long long lanes = __ballot(near(lane_chunk(cm, cb)));
                    if (lanes) visit(c0 + cb * cs, lanes);
                }
            } else {
                // the near masks of every surviving chunk first, parked in
                // LDS, so the batch's metadata is dead during the visits
                // (whose queue work needs every register)
                int n_near = 0;
                while (cmask) {
                    const int cb = __builtin_ctzll(cmask);
                    cmask &= cmask - 1;
                    const unsigned long long lanes = __ballot(near(lane_chunk(cm, cb)));
                    if (lanes) {
                        if (lane == 0) {
                            s_near[wv][n_near] = lanes;
                            s_near_at[wv][n_near] = c0 + cb * cs;
                        }
                        ++n_near;
                    }
                }
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                __builtin_amdgcn_wave_barrier();
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
                for (int i = 0; i < n_near; ++i) {
                    const unsigned long long lanes = s_near[wv][i];
                    const int c = __builtin_amdgcn_readfirstlane(s_near_at[wv][i]);
                    visit(c, ((unsigned long long)__builtin_amdgcn_readfirstlane((unsigned)(lanes >> 32)) << 32) |
                                 (unsigned)__builtin_amdgcn_readfirstlane((unsigned)lanes));
                }
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                __builtin_amdgcn_wave_barrier();
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            }
        }
    }
}

// Which evaluations run as tasks: labels, and full outputs over a ball, with
// one query per lane.
template <bool FULL, bool BALL, int QPL, bool ELL>
constexpr bool uses_tasks()
{
    return QPL == 1 && (!FULL || (BALL && (!ELL || CSPLAT_ELL_FULL_TASKS)));
}

template <int M>
struct TaskAcc {
    int cnt[M];
    float mt[M], sm[M], cs[M];
    int nb;
};

template <bool ELL>
struct TaskQuery {
    float cx, cy, cz, r2, kq;
    float L[ELL ? 9 : 1];
};

// Per-task constants of the full-output pair step, in units of t: the
// collision threshold r^2 kq and the variance factors 2 n_v kq (so that
// t = max(0, D kq - 2 n_v kq sqrt(V)) needs no multiply per n_sigma).
template <int M>
struct TaskScale {
    float thr;
    float c[M];
};

template <int M>
__device__ __forceinline__ void task_reset(TaskAcc<M> &T)
{
#pragma unroll
    for (int v = 0; v < M; ++v) {
        T.cnt[v] = 0;
        T.mt[v] = INFINITY;
        T.sm[v] = 0.f;
        T.cs[v] = 0.f;
    }
    T.nb = 0;
}

// One pair: Gaussian record (mean, M row-major) in r0..r2, query Q.
// g0: the cost constant p.g0 held in a VGPR (the cost's fma would otherwise
// name two scalar operands and copy one of them for every pair).
template <int M, bool ELL>
__device__ __forceinline__ void task_pair(const float4 &r0, const float4 &r1, const float4 &r2,
                                          const TaskQuery<ELL> &Q, const TaskScale<M> &K, const EvalParams &p,
                                          float g0, TaskAcc<M> &T)
{
    const float dx = r0.x - Q.cx, dy = r0.y - Q.cy, dz = r0.z - Q.cz;
    const float Db = fmaf(dz, dz, fmaf(dy, dy, dx * dx));
    const float gp[12] = {r0.x, r0.y, r0.z, r0.w, r1.x, r1.y, r1.z, r1.w, r2.x, r2.y, r2.z, r2.w};
    float D, W;
    metric_dw<ELL>(gp, Q.L, dx, dy, dz, Db, D, W);
    // D and W come before the ball test, and W enters it: each lane runs
    // its own task, so the in-ball block runs for the wave whenever one of
    // its 64 pairs is inside (nearly always) and this costs no issue slots,
    // while a test that reads only the mean lets the compiler move the
    // record's other loads behind it, two memory latencies in a row.  W is
    // NaN only for padding records, whose means at +inf fail the test anyway.
    if (Db <= p.rn2 && W >= 0.f) {
        ++T.nb;
        const float sv = fast_sqrt(W);
        const float Dk = D * Q.kq;
#pragma unroll
        for (int v = 0; v < M; ++v) {
            const float x = fmaf(-K.c[v], sv, Dk);  // kt (s^2 - n sqrt(sigma^2))
            T.cnt[v] += x < K.thr;                  // s~^2 < 1
            const float t = fmaxf(x, 0.f);
            // stable log-sum-exp about the task's running minimum (one exp per pair)
            const float e = fast_exp2(-fabsf(t - T.mt[v]));
            const bool lower = t < T.mt[v];
            T.sm[v] = lower ? fmaf(T.sm[v], e, 1.f) : T.sm[v] + e;
            T.mt[v] = lower ? t : T.mt[v];
            // 2^min(y, 0) = min(2^y, 1): the clamp folds into the exp
            T.cs[v] += __builtin_amdgcn_fmed3f(fast_exp2(fmaf(t, -p.g1, g0)), 0.f, 1.f);
        }
    }
}

// One pair for labels only: the sqrt-free test a |a| < 4 n^2 W with
// a = (r^2)(s^2 - 1) (an exact rewrite of s~^2 < 1), inside the ball if any.
template <int M, bool BALL, bool ELL>
__device__ __forceinline__ void task_pair_label(const float4 &r0, const float4 &r1, const float4 &r2,
                                                const TaskQuery<ELL> &Q, const EvalParams &p, TaskAcc<M> &T)
{
    const float dx = r0.x - Q.cx, dy = r0.y - Q.cy, dz = r0.z - Q.cz;
    const float gp[12] = {r0.x, r0.y, r0.z, r0.w, r1.x, r1.y, r1.z, r1.w, r2.x, r2.y, r2.z, r2.w};
    float a, D, W;
    bool in = true;
    if constexpr (ELL) {
        metric_dw<ELL>(gp, Q.L, dx, dy, dz, 0.f, D, W);
        a = D - 1.f;
        if constexpr (BALL) in = fmaf(dz, dz, fmaf(dy, dy, dx * dx)) <= p.rn2;
    } else {
        a = fmaf(dz, dz, fmaf(dy, dy, fmaf(dx, dx, -Q.r2)));
        metric_dw<ELL>(gp, Q.L, dx, dy, dz, 0.f, D, W);
        if constexpr (BALL) in = a + Q.r2 <= p.rn2;
    }
    const float aa = a * fabsf(a);
#pragma unroll
    for (int v = 0; v < M; ++v) T.cnt[v] += in && (aa < p.four_n2[v] * W);
}

// One pair for labels and the minimum (spheres, every kept Gaussian): the
// label test as in task_pair_label, and t = max(0, D - 2 n_v sqrt(V)) =
// r^2 s~^2 (Eq. 8 in r^2 units) folded into the task's minimum.  Padding
// records (mean at +inf, M = 0) give W = NaN and are skipped by the W >= 0
// test, so they never lower the minimum.
template <int M, bool COUNT>
__device__ __forceinline__ void task_pair_label_min(const float4 &r0, const float4 &r1, const float4 &r2,
                                                    const TaskQuery<false> &Q, const EvalParams &p, TaskAcc<M> &T)
{
    const float dx = r0.x - Q.cx, dy = r0.y - Q.cy, dz = r0.z - Q.cz;
    const float gp[12] = {r0.x, r0.y, r0.z, r0.w, r1.x, r1.y, r1.z, r1.w, r2.x, r2.y, r2.z, r2.w};
    const float Db = fmaf(dz, dz, fmaf(dy, dy, dx * dx));
    float D, W;
    metric_dw<false>(gp, Q.L, dx, dy, dz, Db, D, W);
    if constexpr (COUNT) {
        const float a = fmaf(dz, dz, fmaf(dy, dy, fmaf(dx, dx, -Q.r2)));  // as task_pair_label
        const float aa = a * fabsf(a);
#pragma unroll
        for (int v = 0; v < M; ++v) T.cnt[v] += aa < p.four_n2[v] * W;
    }
    const float sv = fast_sqrt(W);
    const bool real = W >= 0.f;
#pragma unroll
    for (int v = 0; v < M; ++v) T.mt[v] = fminf(T.mt[v], real ? fmaxf(fmaf(-p.two_n[v], sv, D), 0.f) : INFINITY);
}

// Fold a task partial X into the totals A (first-level sums into the second).
template <int M>
__device__ __forceinline__ void task_fold(TaskAcc<M> &A, const TaskAcc<M> &X)
{
#pragma unroll
    for (int v = 0; v < M; ++v) {
        A.cnt[v] += X.cnt[v];
        A.cs[v] += X.cs[v];
        // log-sum-exp merge: the sum with the larger minimum is scaled by
        // 2^-(difference); selects instead of branches (a wave's lanes fold
        // partials of different queries).  An empty partial (minimum +inf,
        // sum 0) scales by 0 and leaves the totals' bits unchanged, and an
        // empty total takes the partial as it is (2^-inf = 0).
        const float cm = X.mt[v], tm = A.mt[v];
        const bool lower = cm < tm;
        const float e = lower || cm < INFINITY ? fast_exp2(lower ? cm - tm : tm - cm) : 0.f;
        A.sm[v] = lower ? fmaf(A.sm[v], e, X.sm[v]) : fmaf(X.sm[v], e, A.sm[v]);
        A.mt[v] = lower ? cm : tm;
    }
    A.nb += X.nb;
}

// A task partial as PW words in LDS (cnt | mt | sm | cs | nb), and back.
template <int M, int PW>
__device__ __forceinline__ void task_store(float4 *dst, const TaskAcc<M> &T)
{
    float w[4 * ((4 * M + 4) / 4)];
#pragma unroll
    for (int v = 0; v < M; ++v) {
        w[v] = __int_as_float(T.cnt[v]);
        w[M + v] = T.mt[v];
        w[2 * M + v] = T.sm[v];
        w[3 * M + v] = T.cs[v];
    }
    w[4 * M] = __int_as_float(T.nb);
#pragma unroll
    for (int k = 4 * M + 1; k < 4 * ((4 * M + 4) / 4); ++k) w[k] = w[4 * M];
#pragma unroll
    for (int k = 0; k < (4 * M + 4) / 4; ++k) dst[k] = make_float4(w[4 * k], w[4 * k + 1], w[4 * k + 2], w[4 * k + 3]);
}

template <int M, int PW>
__device__ __forceinline__ TaskAcc<M> task_load(const float4 *src)
{
    float w[4 * ((4 * M + 4) / 4)];
#pragma unroll
    for (int k = 0; k < (4 * M + 4) / 4; ++k) {
        const float4 x = src[k];
        w[4 * k] = x.x, w[4 * k + 1] = x.y, w[4 * k + 2] = x.z, w[4 * k + 3] = x.w;
    }
    TaskAcc<M> X;
#pragma unroll
    for (int v = 0; v < M; ++v) {
        X.cnt[v] = __float_as_int(w[v]);
        X.mt[v] = w[M + v];
        X.sm[v] = w[2 * M + v];
        X.cs[v] = w[3 * M + v];
    }
    X.nb = __float_as_int(w[4 * M]);
    return X;
}

// The end of a full-output work item.  With G = 1 each wave writes its
// queries' totals as partial record `item`.  With G > 1 the G consecutive
// waves of a query group walked splits item G, ..., item G + G - 1 for the
// same queries: their totals meet in LDS (each wave's area of `lds`, free
// after its rounds) and the group's first wave folds them in split order
// (the fold of the combine) and writes one record, so the partials take G
// times fewer words.  Every wave of the block calls this (G is uniform).
template <int M, int PW>
__device__ __forceinline__ void full_item_out(TaskAcc<M> A, int G, int item, int jq, int q, const Part &part,
                                              float4 *lds, int wave_f4, int wv, int lane)
{
    if (G > 1) {
        task_store<M, PW>(lds + (size_t)wv * wave_f4 + lane * (PW / 4), A);
        __syncthreads();
        if (wv % G != 0) return;
        for (int k = 1; k < G; ++k) task_fold(A, task_load<M, PW>(lds + (size_t)(wv + k) * wave_f4 + lane * (PW / 4)));
    }
    if (jq < q) {
#pragma unroll
        for (int v = 0; v < M; ++v) {
            const size_t o = ((size_t)item * M + v) * q + jq;
            part.cnt[o] = A.cnt[v];
            part.mt[o] = A.mt[v];
            part.sm[o] = A.sm[v];
            part.cs[o] = A.cs[v];
        }
        part.nb[(size_t)item * q + jq] = A.nb;
    }
}

// Words of a task partial in LDS (4M + 1 for full outputs, M for labels)
// rounded up to whole float4s, and kept off a multiple of 8 words so that the
// lanes' rows spread over banks.
constexpr int task_words_of(int w) { return ((w + 3) / 4) * 4 % 8 == 0 ? ((w + 3) / 4) * 4 + 4 : ((w + 3) / 4) * 4; }
template <int M, bool FULL>
constexpr int task_words()
{
    return task_words_of(FULL ? 4 * M + 1 : M);
}

__device__ __forceinline__ float lane_shfl(float v, int src) { return __shfl(v, src); }

// Queries per queue entry of the full-output task walk.  With one
// conservatism value a pair costs few operations against its 48-byte record,
// and the walk is bound by the return of vector-memory data (manipulation
// workload: texture units ~72% busy, VALU issue 61%), so an entry holds two
// queries of the same sub-chunk and one lane evaluates both against each
// record it loads.  Each query still has one task per sub-chunk over the
// same records in the same order, folded in queue order: the bits do not
// depend on the entry size.
#ifndef CSPLAT_FULL_QUERIES_PER_TASK
#define CSPLAT_FULL_QUERIES_PER_TASK 2  // 1 or 2
#endif
template <int M, bool ELL>
constexpr int full_entry_queries()
{
    return M == 1 && !ELL ? CSPLAT_FULL_QUERIES_PER_TASK : 1;
}

template <int M, bool FULL, bool BALL, bool CULL, bool ELL>
__device__ __forceinline__ void eval_tile_tasks(const float *__restrict__ gs, int n, int S, int G, int item,
                                                int tile, const float *__restrict__ centers,
                                                const float *__restrict__ radii, int q, const EvalParams &p,
                                                const Part &part, const float *__restrict__ cull, int *tasks_done)
{
    static_assert(FULL && BALL, "labels run in eval_tile_label_tasks");
    constexpr int kRing = 128;  // queued tasks per wave: at most 63 waiting + 64 of one sub-chunk
    constexpr int PW = task_words<M, FULL>();
    constexpr int kWaves = kFullTaskBlock / 64;
    __shared__ int s_task[kWaves][kRing];              // sub-chunk of each queued task
    __shared__ unsigned char s_owner[kWaves][kRing];   // lane of its query
    __shared__ float4 s_part[kWaves][64 * PW / 4];     // partials of a round, PW words per task
    const int lane = (int)(threadIdx.x & 63u), wv = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    // wave wv: the (wv / G)-th 64 queries of the tile, split item G + wv % G
    const int split = item * G + wv % G;
    const int jq = tile * (kFullTaskBlock / G) + (wv / G) * 64 + lane;
    const int jj = jq < q ? jq : q - 1;  // past the end: evaluate a real query, write nothing
    TaskQuery<ELL> own;
    if constexpr (ELL) {
        const float4 *b = reinterpret_cast<const float4 *>(centers + (size_t)kBodyFloats * jj);
        const float4 b0 = b[0], b1 = b[1], b2 = b[2];
        own.cx = b0.x, own.cy = b0.y, own.cz = b0.z;
        own.L[0] = b0.w, own.L[1] = b1.x, own.L[2] = b1.y, own.L[3] = b1.z, own.L[4] = b1.w;
        own.L[5] = b2.x, own.L[6] = b2.y, own.L[7] = b2.z, own.L[8] = b2.w;
        own.r2 = 1.f;
        own.kq = p.kt;
    } else {
        own.cx = centers[3 * jj];
        own.cy = centers[3 * jj + 1];
        own.cz = centers[3 * jj + 2];
        const float r = radii[jj];
        own.r2 = r * r;
        own.kq = p.kt / own.r2;
    }
    TaskAcc<M> A;
    task_reset(A);
    // ring positions of the lane's own queued tasks (bit k of lo: position k,
    // of hi: position 64 + k); head, tail: wave-uniform, counting up
    unsigned long long own_lo = 0, own_hi = 0;
    int head = 0, tail = 0;
    float g0v = p.g0;
    asm volatile("" : "+v"(g0v));

    auto run_round = [&](int n_t) {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        const bool valid = lane < n_t;
        const int pos = (head + lane) & (kRing - 1);
        const int f = valid ? s_task[wv][pos] : 0;
        const int qi = valid ? (int)s_owner[wv][pos] : 0;
        // the lane permutes run with every lane active (a permute reads
        // nothing useful from an inactive source lane), the selects after
        TaskQuery<ELL> tq;
        tq.cx = lane_shfl(own.cx, qi);
        // a lane without a task walks sub-chunk 0 for a query at infinity,
        // which has no Gaussian in its ball (its partial is never folded)
        if (!valid) tq.cx = INFINITY;
        tq.cy = lane_shfl(own.cy, qi);
        tq.cz = lane_shfl(own.cz, qi);
        tq.r2 = lane_shfl(own.r2, qi);
        tq.kq = lane_shfl(own.kq, qi);
        if constexpr (ELL) {
#pragma unroll
            for (int k = 0; k < 9; ++k) tq.L[k] = lane_shfl(own.L[k], qi);
        }
        TaskScale<M> K;
        K.thr = tq.r2 * tq.kq;
#pragma unroll
        for (int v = 0; v < M; ++v) K.c[v] = p.two_n[v] * tq.kq;
        TaskAcc<M> T;
        task_reset(T);
        // the scene's records are padded to whole chunks (pad means at +inf)
        const float4 *rp = reinterpret_cast<const float4 *>(gs) + (size_t)f * (kFine * kGaussFloats / 4);
        constexpr int kTaskUnroll = task_unroll<M>();
#pragma unroll 1
        for (int k = 0; k < kFine; k += kTaskUnroll, rp += kTaskUnroll * (kGaussFloats / 4)) {
            float4 r[kTaskUnroll][3];
#pragma unroll
            for (int u = 0; u < kTaskUnroll; ++u) {
                r[u][0] = rp[u * (kGaussFloats / 4)];
                r[u][1] = rp[u * (kGaussFloats / 4) + 1];
                r[u][2] = rp[u * (kGaussFloats / 4) + 2];
            }
#pragma unroll
            for (int u = 0; u < kTaskUnroll; ++u) task_pair<M, ELL>(r[u][0], r[u][1], r[u][2], tq, K, p, g0v, T);
        }
        // the round's partials to LDS (slot = lane), words: cnt | mt | sm | cs | nb
        {
            float w[PW];
#pragma unroll
            for (int v = 0; v < M; ++v) {
                w[v] = __int_as_float(T.cnt[v]);
                w[M + v] = T.mt[v];
                w[2 * M + v] = T.sm[v];
                w[3 * M + v] = T.cs[v];
            }
            w[4 * M] = __int_as_float(T.nb);
            // the padding words after them are never read: only the float4s
            // that hold data are written (the rest of the last one repeats nb)
            constexpr int kData = (4 * M + 4) / 4;
#pragma unroll
            for (int k = 4 * M + 1; k < 4 * kData; ++k) w[k] = w[4 * M];
            float4 *dst = &s_part[wv][lane * (PW / 4)];
#pragma unroll
            for (int k = 0; k < kData; ++k) dst[k] = make_float4(w[4 * k], w[4 * k + 1], w[4 * k + 2], w[4 * k + 3]);
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        // each query folds its tasks of this round, in queue order; the
        // round's slot i is ring position head + i, head a multiple of 64
        for (unsigned long long mine = (head & 64) ? own_hi : own_lo; mine; mine &= mine - 1) {
            const float4 *src = &s_part[wv][__builtin_ctzll(mine) * (PW / 4)];
            float w[PW];
#pragma unroll
            for (int k = 0; k < (4 * M + 4) / 4; ++k) {
                const float4 x = src[k];
                w[4 * k] = x.x, w[4 * k + 1] = x.y, w[4 * k + 2] = x.z, w[4 * k + 3] = x.w;
            }
            TaskAcc<M> X;
#pragma unroll
            for (int v = 0; v < M; ++v) {
                X.cnt[v] = __float_as_int(w[v]);
                X.mt[v] = w[M + v];
                X.sm[v] = w[2 * M + v];
                X.cs[v] = w[3 * M + v];
            }
            X.nb = __float_as_int(w[4 * M]);
            task_fold(A, X);
        }
        if (head & 64) own_hi = 0;
        else own_lo = 0;
        head += n_t;
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    };
    // queue the tasks of sub-chunk fi for the lanes in `lanes` (every lane is active)
    auto enqueue = [&](int fi, unsigned long long lanes) {
        const int k = (int)__builtin_amdgcn_mbcnt_hi((unsigned)(lanes >> 32),
                                                     __builtin_amdgcn_mbcnt_lo((unsigned)lanes, 0u));
        if ((lanes >> lane) & 1ull) {
            const int pos = (tail + k) & (kRing - 1);
            s_task[wv][pos] = fi;
            s_owner[wv][pos] = (unsigned char)lane;
            if (pos < 64) own_lo |= 1ull << pos;
            else own_hi |= 1ull << (pos - 64);
        }
        const int cnt = __popcll(lanes);
        tail += cnt;
        if (tasks_done) *tasks_done += cnt;
        if (tail - head >= 64) run_round(64);
    };

    const int n_chunks = (n + kCull - 1) / kCull;
    const int n_fine = (n + kFine - 1) / kFine;
    const int n_groups = (n_chunks + kGroup - 1) / kGroup;
    if constexpr (!CULL) {
        for (int c = split; c < n_chunks; c += S)
            for (int k = 0; k < kFinePer; ++k) {
                const int fi = c * kFinePer + k;
                if (fi < n_fine) enqueue(fi, ~0ull);
            }
    } else {
        const float *fine = cull + (size_t)n_chunks * kCullFloats;  // the sub-chunk level
        const float *groups = fine + (size_t)n_fine * kCullFloats;  // the group level
        float cx[1] = {own.cx}, cy[1] = {own.cy}, cz[1] = {own.cz}, r2[1] = {own.r2};
        float wx, wy, wz, spread, r2max;
        wave_sphere<1>(cx, cy, cz, r2, wx, wy, wz, spread, r2max);
        // full outputs reduce over the ball: a chunk farther than r_nbr plus
        // its radius from a body's centre holds no counted pair
        auto reach_of = [&](const ChunkMeta &) { return p.r_nbr; };
        split_walk<false>(
            groups, cull, n_groups, n_chunks, split, S,
            [&](const ChunkMeta &m) { return within(m, wx, wy, wz, spread + m.rad + reach_of(m)); },
            [&](const ChunkMeta &m) { return within(m, own.cx, own.cy, own.cz, m.rad + reach_of(m)); },
            [&](int ci, unsigned long long lanes) {
                // the sub-chunks' records are read together (one latency),
                // tested, and their lanes rotated through one enqueue site
                static_assert(kFinePer == 4, "sub-chunk rotation below assumes four");
                const int f0 = ci * kFinePer;
                ChunkMeta fm[kFinePer];
#pragma unroll
                for (int k = 0; k < kFinePer; ++k) fm[k] = load_chunk(fine, min(f0 + k, n_fine - 1));
                unsigned long long fl[kFinePer];
#pragma unroll
                for (int k = 0; k < kFinePer; ++k) {
                    const unsigned long long exists = f0 + k < n_fine ? ~0ull : 0ull;
                    fl[k] = lanes & exists &
                            __ballot(within(fm[k], own.cx, own.cy, own.cz, fm[k].rad + reach_of(fm[k])));
                }
                unsigned long long l0 = fl[0], l1 = fl[1], l2 = fl[2], l3 = fl[3];
#pragma unroll 1
                for (int k = 0; k < kFinePer; ++k) {
                    if (l0) enqueue(f0 + k, l0);
                    l0 = l1, l1 = l2, l2 = l3, l3 = 0;
                }
            });
    }
    if (tail > head) run_round(tail - head);
    full_item_out<M, PW>(A, G, item, jq, q, part, &s_part[0][0], (int)(sizeof(s_part[0]) / sizeof(float4)), wv, lane);
}

// The same walk with KQ > 1 queries per queue entry (one conservatism value).
template <int M, bool FULL, bool BALL, bool CULL, bool ELL>
__device__ __forceinline__ void eval_tile_tasks_shared(const float *__restrict__ gs, int n, int S, int G, int item,
                                                       int tile, const float *__restrict__ centers,
                                                       const float *__restrict__ radii, int q, const EvalParams &p,
                                                       const Part &part, const float *__restrict__ cull,
                                                       int *tasks_done)
{
    static_assert(FULL && BALL, "labels run in eval_tile_label_tasks");
    constexpr int KQ = full_entry_queries<M, ELL>();  // queries per entry
    static_assert(KQ == 2, "the slot masks hold one bit per entry: two queries per entry");
    constexpr int kRing = 128;  // queued entries per wave: at most 63 waiting + 64 / KQ of one sub-chunk
    constexpr int PW = task_words<M, FULL>();
    constexpr int kWaves = kFullTaskBlock / 64;
    constexpr unsigned char kNone = 0xFF;
    __shared__ int s_task[kWaves][kRing];                  // sub-chunk of each queued entry
    __shared__ unsigned char s_q[kWaves][KQ][kRing];       // lanes of its queries, kNone for an empty slot
    __shared__ float4 s_part[kWaves][KQ * 64 * PW / 4];    // partials of a round, PW words per task
    const int lane = (int)(threadIdx.x & 63u), wv = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    // wave wv: the (wv / G)-th 64 queries of the tile, split item G + wv % G
    const int split = item * G + wv % G;
    const int jq = tile * (kFullTaskBlock / G) + (wv / G) * 64 + lane;
    const int jj = jq < q ? jq : q - 1;  // past the end: evaluate a real query, write nothing
    TaskQuery<ELL> own;
    if constexpr (ELL) {
        const float4 *b = reinterpret_cast<const float4 *>(centers + (size_t)kBodyFloats * jj);
        const float4 b0 = b[0], b1 = b[1], b2 = b[2];
        own.cx = b0.x, own.cy = b0.y, own.cz = b0.z;
        own.L[0] = b0.w, own.L[1] = b1.x, own.L[2] = b1.y, own.L[3] = b1.z, own.L[4] = b1.w;
        own.L[5] = b2.x, own.L[6] = b2.y, own.L[7] = b2.z, own.L[8] = b2.w;
        own.r2 = 1.f;
        own.kq = p.kt;
    } else {
        own.cx = centers[3 * jj];
        own.cy = centers[3 * jj + 1];
        own.cz = centers[3 * jj + 2];
        const float r = radii[jj];
        own.r2 = r * r;
        own.kq = p.kt / own.r2;
    }
    TaskAcc<M> A;
    task_reset(A);
    // ring positions of the lane's own queued tasks (bit k of lo: position k,
    // of hi: position 64 + k) and, with two queries per entry, which slot of
    // the entry is the lane's; head, tail: wave-uniform, counting up
    unsigned long long own_lo = 0, own_hi = 0, slot_lo = 0, slot_hi = 0;
    int head = 0, tail = 0;
    float g0v = p.g0;
    asm volatile("" : "+v"(g0v));

    auto run_round = [&](int n_t) {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        const bool valid = lane < n_t;
        const int pos = (head + lane) & (kRing - 1);
        const int f = valid ? s_task[wv][pos] : 0;
        TaskQuery<ELL> tq[KQ];
        TaskScale<M> K[KQ];
        TaskAcc<M> T[KQ];
#pragma unroll
        for (int j = 0; j < KQ; ++j) {
            const int iq = valid ? (int)s_q[wv][j][pos] : (KQ > 1 ? (int)kNone : 0);
            const bool ok = KQ > 1 ? iq != (int)kNone : valid;
            const int qi = KQ > 1 ? iq & 63 : iq;
            // the lane permutes run with every lane active (a permute reads
            // nothing useful from an inactive source lane), the selects after
            tq[j].cx = lane_shfl(own.cx, qi);
            // a lane without a task walks sub-chunk 0 for a query at
            // infinity, which has no Gaussian in its ball (its partial is
            // never folded); so does an empty slot of an entry
            if (!ok) tq[j].cx = INFINITY;
            tq[j].cy = lane_shfl(own.cy, qi);
            tq[j].cz = lane_shfl(own.cz, qi);
            tq[j].r2 = lane_shfl(own.r2, qi);
            tq[j].kq = lane_shfl(own.kq, qi);
            if constexpr (ELL) {
#pragma unroll
                for (int k = 0; k < 9; ++k) tq[j].L[k] = lane_shfl(own.L[k], qi);
            }
            K[j].thr = tq[j].r2 * tq[j].kq;
#pragma unroll
            for (int v = 0; v < M; ++v) K[j].c[v] = p.two_n[v] * tq[j].kq;
            task_reset(T[j]);
        }
        // the scene's records are padded to whole chunks (pad means at +inf)
        const float4 *rp = reinterpret_cast<const float4 *>(gs) + (size_t)f * (kFine * kGaussFloats / 4);
        constexpr int kTaskUnroll = KQ > 1 ? 2 : task_unroll<M>();
#pragma unroll 1
        for (int k = 0; k < kFine; k += kTaskUnroll, rp += kTaskUnroll * (kGaussFloats / 4)) {
            float4 r[kTaskUnroll][3];
#pragma unroll
            for (int u = 0; u < kTaskUnroll; ++u) {
                r[u][0] = rp[u * (kGaussFloats / 4)];
                r[u][1] = rp[u * (kGaussFloats / 4) + 1];
                r[u][2] = rp[u * (kGaussFloats / 4) + 2];
            }
#pragma unroll
            for (int u = 0; u < kTaskUnroll; ++u)
#pragma unroll
                for (int j = 0; j < KQ; ++j) task_pair<M, ELL>(r[u][0], r[u][1], r[u][2], tq[j], K[j], p, g0v, T[j]);
        }
        // the round's partials to LDS (row = lane KQ + slot), words:
        // cnt | mt | sm | cs | nb
#pragma unroll
        for (int j = 0; j < KQ; ++j) {
            float w[PW];
#pragma unroll
            for (int v = 0; v < M; ++v) {
                w[v] = __int_as_float(T[j].cnt[v]);
                w[M + v] = T[j].mt[v];
                w[2 * M + v] = T[j].sm[v];
                w[3 * M + v] = T[j].cs[v];
            }
            w[4 * M] = __int_as_float(T[j].nb);
            // the padding words after them are never read: only the float4s
            // that hold data are written (the rest of the last one repeats nb)
            constexpr int kData = (4 * M + 4) / 4;
#pragma unroll
            for (int k = 4 * M + 1; k < 4 * kData; ++k) w[k] = w[4 * M];
            float4 *dst = &s_part[wv][(lane * KQ + j) * (PW / 4)];
#pragma unroll
            for (int k = 0; k < kData; ++k) dst[k] = make_float4(w[4 * k], w[4 * k + 1], w[4 * k + 2], w[4 * k + 3]);
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        // each query folds its tasks of this round, in queue order; the
        // round's entry i is ring position head + i, head a multiple of 64
        const unsigned long long slots = (head & 64) ? slot_hi : slot_lo;
        for (unsigned long long mine = (head & 64) ? own_hi : own_lo; mine; mine &= mine - 1) {
            const int e = __builtin_ctzll(mine);
            const int row = KQ > 1 ? e * KQ + (int)((slots >> e) & 1ull) : e;
            const float4 *src = &s_part[wv][row * (PW / 4)];
            float w[PW];
#pragma unroll
            for (int k = 0; k < (4 * M + 4) / 4; ++k) {
                const float4 x = src[k];
                w[4 * k] = x.x, w[4 * k + 1] = x.y, w[4 * k + 2] = x.z, w[4 * k + 3] = x.w;
            }
            TaskAcc<M> X;
#pragma unroll
            for (int v = 0; v < M; ++v) {
                X.cnt[v] = __float_as_int(w[v]);
                X.mt[v] = w[M + v];
                X.sm[v] = w[2 * M + v];
                X.cs[v] = w[3 * M + v];
            }
            X.nb = __float_as_int(w[4 * M]);
            task_fold(A, X);
        }
        if (head & 64) own_hi = 0, slot_hi = 0;
        else own_lo = 0, slot_lo = 0;
        head += n_t;
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    };
    // queue the tasks of sub-chunk fi for the lanes in `lanes`, KQ queries
    // per entry in lane order (every lane is active)
    auto enqueue = [&](int fi, unsigned long long lanes) {
        const int c = __popcll(lanes);
        const int k = (int)__builtin_amdgcn_mbcnt_hi((unsigned)(lanes >> 32),
                                                     __builtin_amdgcn_mbcnt_lo((unsigned)lanes, 0u));
        if ((lanes >> lane) & 1ull) {
            const int pos = (tail + k / KQ) & (kRing - 1);
            const int slot = k % KQ;
            if (slot == 0) s_task[wv][pos] = fi;
            s_q[wv][slot][pos] = (unsigned char)lane;
            if (KQ > 1 && k == c - 1)  // the last entry's empty slots
                for (int j = slot + 1; j < KQ; ++j) s_q[wv][j][pos] = kNone;
            if constexpr (KQ == 1) {
                if (pos < 64) own_lo |= 1ull << pos;
                else own_hi |= 1ull << (pos - 64);
            } else {
                // selects, not branches: the four masks stay in registers
                const unsigned long long bit = 1ull << (pos & 63);
                const bool hi = pos >= 64;
                own_lo |= hi ? 0ull : bit;
                own_hi |= hi ? bit : 0ull;
                slot_lo |= !hi && slot ? bit : 0ull;
                slot_hi |= hi && slot ? bit : 0ull;
            }
        }
        tail += (c + KQ - 1) / KQ;
        if (tasks_done) *tasks_done += c;
        if (tail - head >= 64) run_round(64);
    };

    const int n_chunks = (n + kCull - 1) / kCull;
    const int n_fine = (n + kFine - 1) / kFine;
    const int n_groups = (n_chunks + kGroup - 1) / kGroup;
    if constexpr (!CULL) {
        for (int c = split; c < n_chunks; c += S)
            for (int k = 0; k < kFinePer; ++k) {
                const int fi = c * kFinePer + k;
                if (fi < n_fine) enqueue(fi, ~0ull);
            }
    } else {
        const float *fine = cull + (size_t)n_chunks * kCullFloats;  // the sub-chunk level
        const float *groups = fine + (size_t)n_fine * kCullFloats;  // the group level
        float cx[1] = {own.cx}, cy[1] = {own.cy}, cz[1] = {own.cz}, r2[1] = {own.r2};
        float wx, wy, wz, spread, r2max;
        wave_sphere<1>(cx, cy, cz, r2, wx, wy, wz, spread, r2max);
        // full outputs reduce over the ball: a chunk farther than r_nbr plus
        // its radius from a body's centre holds no counted pair
        auto reach_of = [&](const ChunkMeta &) { return p.r_nbr; };
        split_walk<false>(
            groups, cull, n_groups, n_chunks, split, S,
            [&](const ChunkMeta &m) { return within(m, wx, wy, wz, spread + m.rad + reach_of(m)); },
            [&](const ChunkMeta &m) { return within(m, own.cx, own.cy, own.cz, m.rad + reach_of(m)); },
            [&](int ci, unsigned long long lanes) {
                // the sub-chunks' records are read together (one latency),
                // tested, and their lanes rotated through one enqueue site
                static_assert(kFinePer == 4, "sub-chunk rotation below assumes four");
                const int f0 = ci * kFinePer;
                ChunkMeta fm[kFinePer];
#pragma unroll
                for (int k = 0; k < kFinePer; ++k) fm[k] = load_chunk(fine, min(f0 + k, n_fine - 1));
                unsigned long long fl[kFinePer];
#pragma unroll
                for (int k = 0; k < kFinePer; ++k) {
                    const unsigned long long exists = f0 + k < n_fine ? ~0ull : 0ull;
                    fl[k] = lanes & exists &
                            __ballot(within(fm[k], own.cx, own.cy, own.cz, fm[k].rad + reach_of(fm[k])));
                }
                unsigned long long l0 = fl[0], l1 = fl[1], l2 = fl[2], l3 = fl[3];
#pragma unroll 1
                for (int k = 0; k < kFinePer; ++k) {
                    if (l0) enqueue(f0 + k, l0);
                    l0 = l1, l1 = l2, l2 = l3, l3 = 0;
                }
            });
    }
    if (tail > head) run_round(tail - head);
    full_item_out<M, PW>(A, G, item, jq, q, part, &s_part[0][0], (int)(sizeof(s_part[0]) / sizeof(float4)), wv, lane);
}

// ---------------------------------------------------------------------------
// Labels as tasks.  Labels read a 48-byte record per pair for about 25
// operations, so a lane-per-task walk is bound by the return of vector-memory
// data (counters on the precision workload: texture-data unit busy 88% of
// the kernel, VALU 43%).  Here the queue groups the tasks of a sub-chunk: an
// entry is (sub-chunk, KQ queries), and one lane evaluates all of them
// against each record it loads.  The task partials are counts, whose
// sum does not depend on order, so they are added into per-query counters
// in LDS with integer atomics (no ownership masks, no fold loop).
#ifndef CSPLAT_LABEL_QUERIES_PER_TASK
#define CSPLAT_LABEL_QUERIES_PER_TASK 2
#endif
#ifndef CSPLAT_LABEL_UNROLL
#define CSPLAT_LABEL_UNROLL 2  // records per load group of the label task loop
#endif
constexpr int kLabelUnroll = CSPLAT_LABEL_UNROLL;
// With MINW (spheres, every kept Gaussian) the walk also folds each query's
// minimum of t = r^2 s~^2 over the pairs it evaluates (LDS atomic minimum on
// the bits of non-negative floats: order-free), and query j's reach is that
// of the threshold s~^2 < thr[j] instead of 1 (thr NULL: 1): every pair with
// s~^2 < thr[j] is evaluated.  COUNT = false skips the label counts (the
// later passes of the minimum search).
template <int M, bool BALL, bool CULL, bool ELL, bool COUNT = true, bool MINW = false>
__device__ __forceinline__ void eval_tile_label_tasks(const float *__restrict__ gs, int n, int S, int split,
                                                      int tile, const float *__restrict__ centers,
                                                      const float *__restrict__ radii, int q, const EvalParams &p,
                                                      const Part &part, const float *__restrict__ cull,
                                                      int *tasks_done, const float *__restrict__ thr = nullptr)
{
    static_assert(!MINW || (!ELL && !BALL), "the minimum search runs for spheres over every kept Gaussian");
    static_assert(COUNT || MINW, "nothing to compute");
    constexpr int KQ = CSPLAT_LABEL_QUERIES_PER_TASK;  // queries per entry
    constexpr int kRing = 128;  // queued entries per wave: at most 63 waiting + 64 / KQ of one sub-chunk
    constexpr int kWaves = kBlock / 64;
    constexpr unsigned char kNone = 0xFF;
    __shared__ int s_task[kWaves][kRing];             // sub-chunk of each queued entry
    __shared__ unsigned char s_q[kWaves][KQ][kRing];  // lanes of its queries, kNone for an empty slot
    __shared__ int s_cnt[kWaves][COUNT ? 64 * M : 1]; // the wave's counts, query-major
    __shared__ int s_mt[kWaves][MINW ? 64 * M : 1];   // the wave's minima (float bits), query-major
    const int lane = (int)(threadIdx.x & 63u), wv = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int jq = tile * kBlock + (int)(threadIdx.x & ~63u) + lane;
    // a wave wholly past the last query has nothing to do (the walk has no
    // block-wide barrier); a ragged wave evaluates a real query in its place
    // and writes nothing for it
    if (__builtin_amdgcn_readfirstlane(tile * kBlock + (int)(threadIdx.x & ~63u)) >= q) return;
    const int jj = jq < q ? jq : q - 1;
    TaskQuery<ELL> own;
    float qa, qk;  // reach constants: smallest semi-axis squared, largest / smallest
    if constexpr (ELL) {
        const float4 *b = reinterpret_cast<const float4 *>(centers + (size_t)kBodyFloats * jj);
        const float4 b0 = b[0], b1 = b[1], b2 = b[2], b3 = b[3];
        own.cx = b0.x, own.cy = b0.y, own.cz = b0.z;
        own.L[0] = b0.w, own.L[1] = b1.x, own.L[2] = b1.y, own.L[3] = b1.z, own.L[4] = b1.w;
        own.L[5] = b2.x, own.L[6] = b2.y, own.L[7] = b2.z, own.L[8] = b2.w;
        own.r2 = 1.f;
        qa = b3.x;
        qk = b3.y;
    } else {
        own.cx = centers[3 * jj];
        own.cy = centers[3 * jj + 1];
        own.cz = centers[3 * jj + 2];
        const float r = radii[jj];
        own.r2 = r * r;
        qa = MINW && thr ? own.r2 * thr[jj] : own.r2;  // s~^2 < T  <=>  (r^2 units) t < T r^2
        qk = 1.f;
    }
    own.kq = 0.f;
    if constexpr (COUNT) {
#pragma unroll
        for (int v = 0; v < M; ++v) s_cnt[wv][lane * M + v] = 0;
    }
    if constexpr (MINW) {
#pragma unroll
        for (int v = 0; v < M; ++v) s_mt[wv][lane * M + v] = __float_as_int(INFINITY);
    }
    int head = 0, tail = 0;  // wave-uniform ring positions, counting up

    auto fetch_query = [&](int src, bool ok) {
        // every lane runs the permutes (a permute reads nothing useful from
        // an inactive source lane); a query at infinity has no pair
        TaskQuery<ELL> t;
        t.cx = lane_shfl(own.cx, src);
        if (!ok) t.cx = INFINITY;
        t.cy = lane_shfl(own.cy, src);
        t.cz = lane_shfl(own.cz, src);
        t.r2 = lane_shfl(own.r2, src);
        t.kq = 0.f;
        if constexpr (ELL) {
#pragma unroll
            for (int k = 0; k < 9; ++k) t.L[k] = lane_shfl(own.L[k], src);
        }
        return t;
    };
    auto run_round = [&](int n_t) {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        const bool valid = lane < n_t;
        const int pos = (head + lane) & (kRing - 1);
        const int f = valid ? s_task[wv][pos] : 0;
        int iq[KQ];
        TaskQuery<ELL> tq[KQ];
        TaskAcc<M> T[KQ];
#pragma unroll
        for (int j = 0; j < KQ; ++j) {
            iq[j] = valid ? (int)s_q[wv][j][pos] : (int)kNone;
            tq[j] = fetch_query(iq[j] & 63, iq[j] != (int)kNone);
            task_reset(T[j]);
        }
        // the scene's records are padded to whole chunks (pad means at +inf)
        const float4 *rp = reinterpret_cast<const float4 *>(gs) + (size_t)f * (kFine * kGaussFloats / 4);
#pragma unroll 1
        for (int k = 0; k < kFine; k += kLabelUnroll, rp += kLabelUnroll * (kGaussFloats / 4)) {
            float4 r[kLabelUnroll][3];
#pragma unroll
            for (int u = 0; u < kLabelUnroll; ++u) {
                r[u][0] = rp[u * (kGaussFloats / 4)];
                r[u][1] = rp[u * (kGaussFloats / 4) + 1];
                r[u][2] = rp[u * (kGaussFloats / 4) + 2];
            }
#pragma unroll
            for (int u = 0; u < kLabelUnroll; ++u)
#pragma unroll
                for (int j = 0; j < KQ; ++j) {
                    if constexpr (MINW)
                        task_pair_label_min<M, COUNT>(r[u][0], r[u][1], r[u][2], tq[j], p, T[j]);
                    else
                        task_pair_label<M, BALL, ELL>(r[u][0], r[u][1], r[u][2], tq[j], p, T[j]);
                }
        }
#pragma unroll
        for (int j = 0; j < KQ; ++j)
#pragma unroll
            for (int v = 0; v < M; ++v) {
                if constexpr (COUNT)
                    if (iq[j] != (int)kNone && T[j].cnt[v]) atomicAdd(&s_cnt[wv][iq[j] * M + v], T[j].cnt[v]);
                if constexpr (MINW)
                    if (iq[j] != (int)kNone && T[j].mt[v] < INFINITY)
                        atomicMin(&s_mt[wv][iq[j] * M + v], __float_as_int(T[j].mt[v]));
            }
        head += n_t;
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    };
    // queue sub-chunk fi for the lanes in `lanes`, KQ queries per entry
    // (every lane is active)
    auto enqueue = [&](int fi, unsigned long long lanes) {
        const int c = __popcll(lanes);
        const int k = (int)__builtin_amdgcn_mbcnt_hi((unsigned)(lanes >> 32),
                                                     __builtin_amdgcn_mbcnt_lo((unsigned)lanes, 0u));
        if ((lanes >> lane) & 1ull) {
            const int pos = (tail + k / KQ) & (kRing - 1);
            const int slot = k % KQ;
            if (slot == 0) s_task[wv][pos] = fi;
            s_q[wv][slot][pos] = (unsigned char)lane;
            if (k == c - 1)  // the last entry's empty slots
                for (int j = slot + 1; j < KQ; ++j) s_q[wv][j][pos] = kNone;
        }
        tail += (c + KQ - 1) / KQ;
        if (tasks_done) *tasks_done += c;
        if (tail - head >= 64) run_round(64);
    };

    const int n_chunks = (n + kCull - 1) / kCull;
    const int n_fine = (n + kFine - 1) / kFine;
    const int n_groups = (n_chunks + kGroup - 1) / kGroup;
    if constexpr (!CULL) {
        for (int c = split; c < n_chunks; c += S)
            for (int k = 0; k < kFinePer; ++k) {
                const int fi = c * kFinePer + k;
                if (fi < n_fine) enqueue(fi, ~0ull);
            }
    } else {
        const float *fine = cull + (size_t)n_chunks * kCullFloats;  // the sub-chunk level
        const float *groups = fine + (size_t)n_fine * kCullFloats;  // the group level
        float cx[1] = {own.cx}, cy[1] = {own.cy}, cz[1] = {own.cz}, qv[1] = {qa};
        float wx, wy, wz, spread, qamax, half[3];
        wave_sphere<1>(cx, cy, cz, qv, wx, wy, wz, spread, qamax, half);
        float qkmax = qk;
        if constexpr (ELL) {
#pragma unroll
            for (int off = 32; off >= 1; off >>= 1) qkmax = fmaxf(qkmax, __shfl_xor(qkmax, off));
        }
        // the collision bound qk (n s + sqrt(n^2 s^2 + qa)) (s: the chunk's
        // largest scale), capped by the ball when one is given
        auto reach_of = [&](const ChunkMeta &m, float a2, float kk) {
            const float ns = p.n_max * m.smax;
            float reach = ns + fast_sqrt(fmaf(ns, ns, a2));  // v_sqrt: ~1 ulp, far inside kCullMargin
            if constexpr (ELL) reach *= kk;
            if constexpr (BALL) reach = fminf(reach, p.r_nbr);
            return reach;
        };
        split_walk<true>(
            groups, cull, n_groups, n_chunks, split, S,
            [&](const ChunkMeta &m) {
                // the wave's bounding sphere and box (the box is the tighter
                // bound for the flat blocks a wave of grid points forms)
                const float reach = m.rad + reach_of(m, qamax, qkmax);
                return within(m, wx, wy, wz, spread + reach) && within_box(m, wx, wy, wz, half, reach);
            },
            [&](const ChunkMeta &m) { return within(m, own.cx, own.cy, own.cz, m.rad + reach_of(m, qa, qk)); },
            [&](int ci, unsigned long long lanes) {
                static_assert(kFinePer == 4, "sub-chunk rotation below assumes four");
                const int f0 = ci * kFinePer;
                ChunkMeta fm[kFinePer];
#pragma unroll
                for (int k = 0; k < kFinePer; ++k) fm[k] = load_chunk(fine, min(f0 + k, n_fine - 1));
                unsigned long long fl[kFinePer];
#pragma unroll
                for (int k = 0; k < kFinePer; ++k) {
                    const unsigned long long exists = f0 + k < n_fine ? ~0ull : 0ull;
                    fl[k] = lanes & exists &
                            __ballot(within(fm[k], own.cx, own.cy, own.cz, fm[k].rad + reach_of(fm[k], qa, qk)));
                }
                unsigned long long l0 = fl[0], l1 = fl[1], l2 = fl[2], l3 = fl[3];
#pragma unroll 1
                for (int k = 0; k < kFinePer; ++k) {
                    if (l0) enqueue(f0 + k, l0);
                    l0 = l1, l1 = l2, l2 = l3, l3 = 0;
                }
            });
    }
    if (tail > head) run_round(tail - head);
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    if (jq < q) {
#pragma unroll
        for (int v = 0; v < M; ++v) {
            if constexpr (COUNT) part.cnt[((size_t)split * M + v) * q + jq] = s_cnt[wv][lane * M + v];
            if constexpr (MINW) part.mt[((size_t)split * M + v) * q + jq] = __int_as_float(s_mt[wv][lane * M + v]);
        }
    }
}

// One work item: the queries of `tile` (kBlock x QPL of them) against the
// Gaussian range of `split`, written to the split's partial records.  Shared
// by the evaluation kernel and the serving step kernel, so a request gives
// the same bits in either.
// With CULL, Gaussians are visited in chunks of kCull (consecutive on the curve,
// with a bounding sphere and largest scale per chunk); a wave skips a chunk
// when it provably lies outside the neighbourhood ball of every query the
// wave holds (FULL), or beyond the reach bound n s + sqrt(n^2 s^2 + r^2) of
// every query (labels: no pair of it can have s~^2 < 1).  Skipped pairs
// contribute nothing, and the order of every sum is unchanged: the results
// are the same bits.
template <int M, bool FULL, bool BALL, int QPL, bool CULL = false, bool ELL = false>
__device__ __forceinline__ void eval_tile(const float *__restrict__ gs, int n, int S, int G, int split,
                                          int tile, const float *__restrict__ centers,
                                          const float *__restrict__ radii, int q, const EvalParams &p,
                                          const Part &part, const float *__restrict__ cull = nullptr,
                                          int *chunks_done = nullptr)
{
    if constexpr (uses_tasks<FULL, BALL, QPL, ELL>()) {
        if constexpr (FULL && full_entry_queries<M, ELL>() > 1)
            eval_tile_tasks_shared<M, FULL, BALL, CULL, ELL>(gs, n, S, G, split, tile, centers, radii, q, p, part,
                                                             cull, chunks_done);
        else if constexpr (FULL)
            eval_tile_tasks<M, FULL, BALL, CULL, ELL>(gs, n, S, G, split, tile, centers, radii, q, p, part, cull,
                                                      chunks_done);
        else
            eval_tile_label_tasks<M, BALL, CULL, ELL>(gs, n, S, split, tile, centers, radii, q, p, part, cull,
                                                      chunks_done);
        return;
    }
    // Spheres: centers (q x 3) and radii (q).  Ellipsoids (ELL): `centers`
    // holds the prepared records of kBodyFloats floats, `radii` is unused.
    QState<QPL, ELL> Q;
    int jq[QPL];
#pragma unroll
    for (int u = 0; u < QPL; ++u) {
        jq[u] = (tile * kBlock + (int)(threadIdx.x & ~63u)) * QPL + u * 64 + (int)(threadIdx.x & 63u);
        const int jj = jq[u] < q ? jq[u] : q - 1;  // past the end: evaluate a real query, write nothing
        if constexpr (ELL) {
            const float4 *b = reinterpret_cast<const float4 *>(centers + (size_t)kBodyFloats * jj);
            const float4 b0 = b[0], b1 = b[1], b2 = b[2], b3 = b[3];
            Q.cx[u] = b0.x, Q.cy[u] = b0.y, Q.cz[u] = b0.z;
            Q.L[u][0] = b0.w, Q.L[u][1] = b1.x, Q.L[u][2] = b1.y, Q.L[u][3] = b1.z, Q.L[u][4] = b1.w;
            Q.L[u][5] = b2.x, Q.L[u][6] = b2.y, Q.L[u][7] = b2.z, Q.L[u][8] = b2.w;
            Q.qa[u] = b3.x, Q.qk[u] = b3.y;
            Q.r2[u] = 1.f;
            Q.kq[u] = p.kt;
        } else {
            Q.cx[u] = centers[3 * jj];
            Q.cy[u] = centers[3 * jj + 1];
            Q.cz[u] = centers[3 * jj + 2];
            const float r = radii[jj];
            Q.r2[u] = r * r;
            Q.kq[u] = p.kt / Q.r2[u];  // t = max(0, r^2 s~^2) * kq = s~^2 * kt
            Q.qa[u] = Q.r2[u];
            Q.qk[u] = 1.f;
        }
    }
    Acc<M, QPL> A;
#pragma unroll
    for (int u = 0; u < QPL; ++u) {
        A.nb[u] = 0;
#pragma unroll
        for (int v = 0; v < M; ++v) {
            A.cnt[u][v] = 0;
            A.mt[u][v] = INFINITY;
            A.sm[u][v] = 0.f;
            A.cs[u][v] = 0.f;
        }
    }

    // The Gaussians are visited in chunks of kCull (consecutive on the curve); split
    // `split` of S takes chunks split, split + S, split + 2S, ... so that every
    // split samples the whole scene and the work of a query tile is spread
    // evenly over its S work items.  The softmin and cost sums are accumulated
    // per piece of kPiece consecutive chunks of the split and folded into the
    // lane totals at the end of each piece (two-level summation keeps the
    // float32 rounding of long sums near sqrt(kChunk) ulps).  Folding a piece
    // that received no pair changes nothing.
    const int n_chunks = (n + kCull - 1) / kCull;
    auto reset_chunk = [&]() {
        if constexpr (FULL) {
#pragma unroll
            for (int u = 0; u < QPL; ++u)
#pragma unroll
                for (int v = 0; v < M; ++v) {
                    A.cmt[u][v] = INFINITY;
                    A.csm[u][v] = 0.f;
                    A.ccs[u][v] = 0.f;
                }
        }
    };
    auto fold_chunk = [&]() {
        if constexpr (FULL) {
#pragma unroll
            for (int u = 0; u < QPL; ++u)
#pragma unroll
                for (int v = 0; v < M; ++v) {
                    A.cs[u][v] += A.ccs[u][v];
                    const float cm = A.cmt[u][v], tm = A.mt[u][v];
                    if (cm < tm) {
                        A.sm[u][v] = fmaf(A.sm[u][v], fast_exp2(tm == INFINITY ? -INFINITY : cm - tm), A.csm[u][v]);
                        A.mt[u][v] = cm;
                    } else if (cm < INFINITY) {
                        A.sm[u][v] = fmaf(A.csm[u][v], fast_exp2(tm - cm), A.sm[u][v]);
                    }
                }
        }
    };
    // Gaussians [b0, b1): groups of kUnroll records in wave-uniform (scalar)
    // loads; with kPipeline the next group's records are requested before the
    // current group is evaluated, so their latency overlaps the arithmetic
    auto run = [&](int b0, int b1) {
        // the scene records are read-only during every kernel that calls this:
        // reading them through the constant address space makes the
        // wave-uniform loads scalar whatever else the kernel writes
        using CFloat = const __attribute__((address_space(4))) float;
        const CFloat *gp = reinterpret_cast<const CFloat *>(reinterpret_cast<uintptr_t>(gs)) +
                           (size_t)kGaussFloats * b0;
        int g = b0;
        if constexpr (kPipeline) {
            if (g + kUnroll <= b1) {
                float rec[kGaussFloats * kUnroll];
#pragma unroll
                for (int i = 0; i < kGaussFloats * kUnroll; ++i) rec[i] = gp[i];
                for (; g + kUnroll <= b1; g += kUnroll, gp += kGaussFloats * kUnroll) {
                    // the last group re-reads itself: always an in-range address
                    const CFloat *np = g + 2 * kUnroll <= b1 ? gp + kGaussFloats * kUnroll : gp;
                    float nxt[kGaussFloats * kUnroll];
#pragma unroll
                    for (int i = 0; i < kGaussFloats * kUnroll; ++i) nxt[i] = np[i];
#pragma unroll
                    for (int k = 0; k < kUnroll; ++k)
                        pair_step<M, FULL, BALL, QPL, ELL>(rec + kGaussFloats * k, Q, p, A);
#pragma unroll
                    for (int i = 0; i < kGaussFloats * kUnroll; ++i) rec[i] = nxt[i];
                }
            }
        } else {
            for (; g + kUnroll <= b1; g += kUnroll, gp += kGaussFloats * kUnroll) {
                float rec[kGaussFloats * kUnroll];
#pragma unroll
                for (int i = 0; i < kGaussFloats * kUnroll; ++i) rec[i] = gp[i];
#pragma unroll
                for (int k = 0; k < kUnroll; ++k)
                    pair_step<M, FULL, BALL, QPL, ELL>(rec + kGaussFloats * k, Q, p, A);
            }
        }
        for (; g < b1; ++g, gp += kGaussFloats) {
            float rec[kGaussFloats];
#pragma unroll
            for (int i = 0; i < kGaussFloats; ++i) rec[i] = gp[i];
            pair_step<M, FULL, BALL, QPL, ELL>(rec, Q, p, A);
        }
    };
    int open = -1;  // piece holding the pending sums (wave-uniform)
    auto visit = [&](int i) {  // i-th chunk of the split
        const int piece = i / kPiece;
        if (piece != open) {
            if (open >= 0) fold_chunk();
            reset_chunk();
            open = piece;
        }
        const int b0 = (split + i * S) * kCull;
        run(b0, min(n, b0 + kCull));
    };
    if constexpr (!CULL) {
        for (int i = 0; split + i * S < n_chunks; ++i) visit(i);
    } else {
        // Chunks are visited in the same order as without culling, so every
        // sum keeps its order: skipping changes no bit.
        float wx, wy, wz, spread, qamax;
        wave_sphere<QPL>(Q.cx, Q.cy, Q.cz, Q.qa, wx, wy, wz, spread, qamax);
        float qkmax = 1.f;
        if constexpr (ELL) {
            qkmax = Q.qk[0];
#pragma unroll
            for (int u = 1; u < QPL; ++u) qkmax = fmaxf(qkmax, Q.qk[u]);
#pragma unroll
            for (int off = 32; off >= 1; off >>= 1) qkmax = fmaxf(qkmax, __shfl_xor(qkmax, off));
        }
        // reach of a chunk for a body with constants (qa, qk): no pair farther
        // than qk (n s + sqrt(n^2 s^2 + qa)) from the body's centre can collide
        // (s: the chunk's largest scale); full outputs reduce over the ball
        auto reach_of = [&](const ChunkMeta &m, float qa, float qk) {
            if constexpr (FULL) {
                return p.r_nbr;
            } else {
                const float ns = p.n_max * m.smax;
                float reach = ns + fast_sqrt(fmaf(ns, ns, qa));  // v_sqrt: ~1 ulp, far inside kCullMargin
                if constexpr (ELL) reach *= qk;
                if constexpr (BALL) reach = fminf(reach, p.r_nbr);
                return reach;
            }
        };
        cull_walk(
            cull, n_chunks, split, S,
            [&](const ChunkMeta &m) { return within(m, wx, wy, wz, spread + m.rad + reach_of(m, qamax, qkmax)); },
            [&](const ChunkMeta &m) {
                bool near = false;
#pragma unroll
                for (int u = 0; u < QPL; ++u)
                    near |= within(m, Q.cx[u], Q.cy[u], Q.cz[u], m.rad + reach_of(m, Q.qa[u], Q.qk[u]));
                return near;
            },
            [&](int i, unsigned long long) {
                // lanes outside every reach evaluate the chunk with the
                // wave; their own exact tests reject each of its pairs
                if (chunks_done) ++*chunks_done;
                visit(i);
            });
    }
    if (open >= 0) fold_chunk();
#pragma unroll
    for (int u = 0; u < QPL; ++u) {
        const int j = jq[u];
        if (j >= q) continue;
#pragma unroll
        for (int v = 0; v < M; ++v) {
            const size_t o = ((size_t)split * M + v) * q + j;
            part.cnt[o] = A.cnt[u][v];
            if constexpr (FULL) {
                part.mt[o] = A.mt[u][v];
                part.sm[o] = A.sm[u][v];
                part.cs[o] = A.cs[u][v];
            }
        }
        if constexpr (FULL) part.nb[(size_t)split * q + j] = A.nb[u];
    }
}

template <int M, bool FULL, bool BALL, int QPL, bool CULL, bool ELL>
__global__ void __launch_bounds__(kBlock) CSPLAT_OCCUPANCY
pair_kernel(const float *__restrict__ gs, int n, int S, int G, int n_tiles,
            const float *__restrict__ centers, const float *__restrict__ radii, int q,
            const EvalParams p, Part part, const float *__restrict__ cull,
            unsigned long long *__restrict__ chunk_count)
{
    int b = blockIdx.x;
    const int B = gridDim.x;
    if ((B & 7) == 0) b = (b & 7) * (B >> 3) + (b >> 3);  // XCD-major: one XCD, few ranges
    const int split = b / n_tiles;
    const int tile = b - split * n_tiles;
    int done = 0;
    eval_tile<M, FULL, BALL, QPL, CULL, ELL>(gs, n, S, G, split, tile, centers, radii, q, p, part, cull,
                                             &done);
    if (CULL && chunk_count && (threadIdx.x & 63) == 0) atomicAdd(chunk_count, (unsigned long long)done);
}

// The task walk as its own kernel (labels, or full outputs over a ball; one
// query per lane), with its occupancy target.
// Instances whose state outgrows the cap (ellipsoids with several
// conservatism values) keep 3 waves per SIMD rather than spill.
#ifndef CSPLAT_LABEL_WAVES_PER_EU
#define CSPLAT_LABEL_WAVES_PER_EU 4
#endif
template <int M, bool FULL, bool ELL>
constexpr int task_waves_per_eu()
{
    if constexpr (!FULL && !ELL) return CSPLAT_LABEL_WAVES_PER_EU;
    return (ELL && !(FULL && M == 1)) || (FULL && M > 3) ? 3 : CSPLAT_TASK_WAVES_PER_EU;
}

template <int M, bool FULL, bool BALL, bool CULL, bool ELL>
__global__ void __launch_bounds__(task_block<FULL>())
__attribute__((amdgpu_waves_per_eu(task_waves_per_eu<M, FULL, ELL>())))
pair_task_kernel(const float *__restrict__ gs, int n, int S, int G, int n_tiles, const float *__restrict__ centers,
                 const float *__restrict__ radii, int q, const EvalParams p, Part part,
                 const float *__restrict__ cull, unsigned long long *__restrict__ task_count)
{
    int b = blockIdx.x;
    const int B = gridDim.x;
    if ((B & 7) == 0) b = (b & 7) * (B >> 3) + (b >> 3);  // XCD-major: one XCD, few ranges
    const int split = b / n_tiles;
    const int tile = b - split * n_tiles;
    int done = 0;
    if constexpr (FULL && full_entry_queries<M, ELL>() > 1)
        eval_tile_tasks_shared<M, FULL, BALL, CULL, ELL>(gs, n, S, G, split, tile, centers, radii, q, p, part,
                                                         cull, &done);
    else if constexpr (FULL)
        eval_tile_tasks<M, FULL, BALL, CULL, ELL>(gs, n, S, G, split, tile, centers, radii, q, p, part, cull,
                                                  &done);
    else
        eval_tile_label_tasks<M, BALL, CULL, ELL>(gs, n, S, split, tile, centers, radii, q, p, part, cull, &done);
    if (CULL && task_count && (threadIdx.x & 63) == 0) atomicAdd(task_count, (unsigned long long)done);
}

// ---------------------------------------------------------------------------
// The minimum of s~^2 over every kept Gaussian (Eq. 8; labels optional), by
// passes of the label task walk with a rising threshold.  Pass 1 runs at
// threshold 1 (the labels' own reach) and also folds each query's minimum of
// t = r^2 s~^2 over the pairs it evaluates.  A query is resolved when that
// minimum lies below its threshold: every pair with s~^2 < T was evaluated,
// so no skipped pair can be lower.  An unresolved query is walked again with
// a threshold just above its minimum so far (an upper bound of the true
// minimum: the next pass resolves it), or four times the last one when it had
// no pair at all.  Skipped pairs never lower a minimum and the per-pair
// arithmetic does not depend on the pass, so the result is the same bits as
// the minimum over every pair.  Thresholds carry a relative margin of 2^-10
// (resolution) and 2^-8 (next threshold), far above float32 rounding.
constexpr float kMinResolve = 0.9990234375f;  // 1 - 2^-10
constexpr float kMinNext = 1.00390625f;       // 1 + 2^-8

template <int M, bool COUNT, bool CULL>
__global__ void __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(CSPLAT_LABEL_WAVES_PER_EU)))
pair_min_kernel(const float *__restrict__ gs, int n, int S, int n_tiles, const float *__restrict__ centers,
                const float *__restrict__ radii, const float *__restrict__ thr, int q, const EvalParams p, Part part,
                const float *__restrict__ cull, unsigned long long *__restrict__ task_count)
{
    int b = blockIdx.x;
    const int B = gridDim.x;
    if ((B & 7) == 0) b = (b & 7) * (B >> 3) + (b >> 3);  // XCD-major: one XCD, few ranges
    const int split = b / n_tiles;
    const int tile = b - split * n_tiles;
    int done = 0;
    eval_tile_label_tasks<M, false, CULL, false, COUNT, true>(gs, n, S, split, tile, centers, radii, q, p, part,
                                                              cull, &done, thr);
    if (CULL && task_count && (threadIdx.x & 63) == 0) atomicAdd(task_count, (unsigned long long)done);
}

// Pass 1: counts (summed over splits) to the outputs at row perm[j], minima
// (over splits) to the search state st_mt[j][v], threshold 1, and the flag of
// queries whose minimum is not yet certain.
template <int M, bool COUNT>
__global__ void __launch_bounds__(256)
min_first_combine_kernel(int q, int S, const EvalParams p, Part part, const float *__restrict__ radii,
                         const int32_t *__restrict__ perm, uint8_t *label, int32_t *count,
                         float *__restrict__ st_mt, float *__restrict__ st_thr, uint8_t *__restrict__ flag)
{
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= q) return;
    const int oj = perm ? perm[j] : j;
    const float r = radii[j], r2 = r * r;
    bool unresolved = false;
#pragma unroll
    for (int v = 0; v < M; ++v) {
        int cnt = 0;
        float mt = INFINITY;
        for (int s = 0; s < S; ++s) {
            const size_t o = ((size_t)s * M + v) * q + j;
            if constexpr (COUNT) cnt += part.cnt[o];
            mt = fminf(mt, part.mt[o]);
        }
        if constexpr (COUNT) {
            if (count) count[(size_t)oj * p.m + v] = cnt;
            if (label) label[(size_t)oj * p.m + v] = cnt > p.k ? 1 : 0;
        }
        st_mt[(size_t)j * M + v] = mt;
        unresolved |= !(mt < r2 * kMinResolve);
    }
    st_thr[j] = 1.f;
    flag[j] = unresolved ? 1 : 0;
}

// Before pass k > 1: the listed (unresolved) queries' centres, radii and new
// thresholds, gathered in list order (sorted order: waves stay compact).
template <int M>
__global__ void __launch_bounds__(256)
min_gather_kernel(int nl, const int32_t *__restrict__ list, const float *__restrict__ centers,
                  const float *__restrict__ radii, const float *__restrict__ st_mt, float *__restrict__ st_thr,
                  float *__restrict__ cc, float *__restrict__ rr, float *__restrict__ tt, bool dense)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nl) return;
    const int j = list[i];
    const float r = radii[j], r2 = r * r;
    float mx = 0.f;
#pragma unroll
    for (int v = 0; v < M; ++v) mx = fmaxf(mx, st_mt[(size_t)j * M + v]);
    // just above the minimum so far (an upper bound of the true minimum), or
    // four times the last threshold when no pair was in reach; a dense pass
    // (every pair) has no threshold
    const float t = dense ? INFINITY : mx < INFINITY ? mx / r2 * kMinNext : 4.f * st_thr[j];
    st_thr[j] = t;
    tt[i] = t;
    cc[3 * i] = centers[3 * j];
    cc[3 * i + 1] = centers[3 * j + 1];
    cc[3 * i + 2] = centers[3 * j + 2];
    rr[i] = r;
}

// After pass k > 1: the listed queries' minima and flags.  A later pass has
// few queries and many splits: one wave per listed query, its lanes striding
// over the splits (a minimum: any order).
template <int M>
__global__ void __launch_bounds__(256)
min_next_combine_kernel(int nl, int S, Part part, const int32_t *__restrict__ list, const float *__restrict__ radii,
                        const float *__restrict__ st_thr, float *__restrict__ st_mt, uint8_t *__restrict__ flag)
{
    const int i = (int)(((size_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6);
    const int lane = (int)(threadIdx.x & 63u);
    if (i >= nl) return;  // wave-uniform
    const int j = list[i];
    const float r = radii[j], lim = r * r * st_thr[j] * kMinResolve;
    bool unresolved = false;
#pragma unroll
    for (int v = 0; v < M; ++v) {
        float mt = INFINITY;
        for (int s = lane; s < S; s += 64) mt = fminf(mt, part.mt[((size_t)s * M + v) * nl + i]);
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) mt = fminf(mt, __shfl_xor(mt, off));
        mt = fminf(mt, st_mt[(size_t)j * M + v]);
        if (lane == 0) st_mt[(size_t)j * M + v] = mt;
        unresolved |= !(mt < lim);
    }
    if (lane == 0) flag[j] = unresolved ? 1 : 0;
}

// The minima in s~^2 units at row perm[j].
template <int M>
__global__ void __launch_bounds__(256)
min_output_kernel(int q, int m, const float *__restrict__ radii, const int32_t *__restrict__ perm,
                  const float *__restrict__ st_mt, float *__restrict__ out_min)
{
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= q) return;
    const int oj = perm ? perm[j] : j;
    const float r = radii[j], r2 = r * r;
#pragma unroll
    for (int v = 0; v < M; ++v) out_min[(size_t)oj * m + v] = st_mt[(size_t)j * M + v] / r2;
}

// Merge the split partials of query j, conservatism value v, in split order
// and finalise its outputs.  Output row of query j: perm[j] when the queries
// were evaluated in a permuted (spatially sorted) order, j otherwise.  The
// partials are read eight splits at a time ahead of the (sequential) merge.
template <int M, bool FULL>
__device__ __forceinline__ void combine_one(int j, int v, int q, int S, const EvalParams &p, const Part &part,
                                            const EvalOut &out, const int32_t *perm)
{
    // the splits' words are read kAhead splits at a time (the loads of a
    // batch are in flight together), the ball sizes with them
    constexpr int kAhead = 16;
    const int oj = perm ? perm[j] : j;
    const bool want_nb = FULL && (out.cost || (v == 0 && out.nbr));
    int nb = 0;
    int cnt = 0;
    float mt = INFINITY, sm = 0.f, cs = 0.f;
    for (int s0 = 0; s0 < S; s0 += kAhead) {
        int c[kAhead], bn[kAhead];
        float bm[kAhead], bs[kAhead], bc[kAhead];
#pragma unroll
        for (int k = 0; k < kAhead; ++k) {
            const int s = min(s0 + k, S - 1);
            const size_t o = ((size_t)s * M + v) * q + j;
            c[k] = part.cnt[o];
            if constexpr (FULL) {
                bm[k] = part.mt[o];
                bs[k] = part.sm[o];
                bc[k] = part.cs[o];
                bn[k] = want_nb ? part.nb[(size_t)s * q + j] : 0;
            }
        }
#pragma unroll
        for (int k = 0; k < kAhead; ++k) {
            if (s0 + k >= S) break;
            cnt += c[k];
            if constexpr (FULL) {
                nb += bn[k];
                cs += bc[k];
                if (bm[k] < INFINITY) {
                    if (bm[k] < mt) {
                        sm = fmaf(sm, fast_exp2(mt == INFINITY ? -INFINITY : bm[k] - mt), bs[k]);
                        mt = bm[k];
                    } else {
                        sm = fmaf(bs[k], fast_exp2(mt - bm[k]), sm);
                    }
                }
            }
        }
    }
    if (v == 0 && out.nbr) out.nbr[oj] = nb;
    const size_t o = (size_t)oj * p.m + v;
    if (out.count) out.count[o] = cnt;
    if (out.label) out.label[o] = cnt > p.k ? 1 : 0;
    if constexpr (FULL) {
        const float mn = mt * p.inv_kt;
        if (out.min) out.min[o] = mn;
        if (out.softmin) out.softmin[o] = (!p.soft || mt == INFINITY) ? mn : (mt - fast_log2(sm)) * p.inv_kt;
        if (out.cost) out.cost[o] = nb > 0 ? p.d_max * (cs / (float)nb) : 0.f;
    }
}

template <int M, bool FULL>
__device__ __forceinline__ void combine_query(int j, int q, int S, const EvalParams &p, const Part &part,
                                              const EvalOut &out, const int32_t *perm = nullptr)
{
#pragma unroll
    for (int v = 0; v < M; ++v) combine_one<M, FULL>(j, v, q, S, p, part, out, perm);
}

// One thread per (query, conservatism value), queries fastest.
template <int M, bool FULL>
__global__ void __launch_bounds__(256)
combine_kernel(int q, int S, const EvalParams p, Part part, EvalOut out, const int32_t *__restrict__ perm)
{
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (int64_t)q * M) return;
    const int v = (int)(idx / q), j = (int)(idx - (int64_t)v * q);
    combine_one<M, FULL>(j, v, q, S, p, part, out, perm);
}

#ifndef CSPLAT_FULL_GROUP
#define CSPLAT_FULL_GROUP (CSPLAT_FULL_TASK_BLOCK / 64)
#endif
constexpr int kFullGroup = CSPLAT_FULL_GROUP;  // splits merged per full-output work item, at most
constexpr int kMaxSplitChunks = 2048;          // culling chunks per split of a full-output plan, at most
constexpr int kMinSplitChunksFull = 128;       // ... and at least, for full outputs as tasks (when there are that many)
constexpr int kMinSplitChunksLabels = 64;      // culling chunks per split of a label plan, at least (idem)
constexpr int kMinSplitChunksWave = 4;         // ... of a full-output plan on the wave walk, at least (idem)
constexpr int kMinFullSplits = 32;             // splits of a full-output task plan, at least (see split_plan)
constexpr int kGroupMinSplits = 16;            // splits from which full-output work items fold several
static_assert(kFullGroup >= 1 && kFullGroup <= kFullTaskBlock / 64 && (kFullTaskBlock / 64) % kFullGroup == 0,
              "the groups of a work item divide its waves");

// How an evaluation of q queries against n Gaussians is cut into work items.
// The Gaussian chunks form S splits (split s takes every S-th chunk from s),
// enough to fill the device several times over with at least 16 chunks per
// split.  A work item is a block: with G = 1, kBlock x QPL queries against
// one split; for full outputs as tasks over at least kGroupMinSplits splits,
// groups of G waves that take 64 queries against G consecutive splits,
// merged in LDS into one partial record, so the partials hold S / G records
// per query.  Depends only on (q, n, mode,
// device), so a request gives the same partial reductions wherever it runs.
// per_split: Gaussians of the largest split.
struct SplitPlan {
    int n_tiles, S, per_split, qpl;
    int G;      // splits per work item (full outputs as tasks: up to kFullGroup when S allows, else 1)
    int parts;  // partial records per query: S / G
    int block;  // threads of a work item
};

// dense: a label walk without culling (every pair), which has no walk to
// amortise and keeps splits of 16 chunks.
inline SplitPlan split_plan(int target_blocks, int q, int n, bool full, bool ball, bool ell = false,
                            bool dense = false)
{
    SplitPlan sp;
    sp.qpl = full ? kQplFull : kQplLabels;
    const bool tasks = sp.qpl == 1 && (!full || (ball && (!ell || CSPLAT_ELL_FULL_TASKS)));
    if (tasks)
        target_blocks = (int)((int64_t)target_blocks * CSPLAT_TASK_BLOCKS_PER_CU / CSPLAT_BLOCKS_PER_CU);
    const int n_chunks = (n + kCull - 1) / kCull;
    const int tiles256 = (q + kBlock * sp.qpl - 1) / (kBlock * sp.qpl);
    int S = 0;
    if (n > 0) {
        S = tiles256 > 0 ? (target_blocks + tiles256 - 1) / tiles256 : 1;
        // full outputs: at most kMaxSplitChunks chunks per split, so that one
        // work item (up to 256 queries over a 1 m ball) stays a few
        // milliseconds of one block even when the queries alone fill the
        // device (a serving step lasts as long as its slowest item)
        if (full) S = std::max(S, (n_chunks + kMaxSplitChunks - 1) / kMaxSplitChunks);
        // full outputs as tasks: at least kMinFullSplits splits while their
        // partial records stay within 256 MiB (S / 4 records of up to 52 B
        // per query): a large batch would otherwise get a few long splits,
        // whose items balance badly (the manipulation batch, 393,216 spheres
        // on 500k Gaussians: 6 splits 16.5 ms, 16 splits 15.3 ms, 32 splits
        // 11.7 ms, 64 splits 12.4 ms)
        if (full && tasks) {
            const int64_t mem_cap = (int64_t(256) << 20) / (13 * (int64_t)std::max(q, 1));
            S = std::max(S, (int)std::min<int64_t>(kMinFullSplits, mem_cap));
        }
        // at least 128 chunks per split for full outputs as tasks and 64 for
        // labels: a task work item carries a fixed cost (query state, the
        // walk's first metadata loads, the partial record) that short splits
        // repeat.  Full outputs: a batch of 8,192 spheres took 0.40 ms on a
        // 250k-Gaussian scene with 244 splits of 16 chunks, 0.14 ms with 32
        // of 122 (256 chunks: 0.18).  Labels: 4,096 spheres on a
        // 200k-Gaussian scene 0.24 ms with 16 chunks per split, 0.15 with 64,
        // 0.20 with 128.  The wave walk (full outputs over every Gaussian)
        // has no task set-up and wants many splits over a small scene (10k
        // Gaussians x 4,096 spheres: kernel 0.124 ms with 16 chunks per
        // split, 0.060 with 4); dense label walks keep 16.
        const int min_chunks = full ? (tasks ? kMinSplitChunksFull : kMinSplitChunksWave)
                                    : dense ? 16 : kMinSplitChunksLabels;
        S = std::max(1, std::min(S, n_chunks / min_chunks));
    }
    // full outputs as tasks over many splits merge the splits of a block's
    // waves in LDS (a work item: 64 queries x G splits); S rounds up to a
    // multiple of G.  Over few splits (much work per split) a block keeps
    // four query tiles on one split: its waves share the split's records,
    // and none waits for the others' splits before the block retires (the
    // manipulation batch, S = 6: 15.7 ms with one split per item, 21.2 with
    // four).
    sp.block = full && tasks ? kFullTaskBlock : kBlock;
    sp.G = 1;
    if (full && tasks && S >= kGroupMinSplits)
        for (int g = kFullGroup; g > 1; g >>= 1)
            if (S >= g) {
                sp.G = g;
                break;
            }
    if (sp.G > 1) S = (S + sp.G - 1) / sp.G * sp.G;
    sp.S = S;
    sp.parts = S / sp.G;
    sp.n_tiles = (q + sp.block / sp.G * sp.qpl - 1) / (sp.block / sp.G * sp.qpl);
    sp.per_split = S > 0 ? (n_chunks + S - 1) / S * kCull : 0;
    return sp;
}

// Words of partial reductions per (split, query) for m conservatism values.
inline size_t part_words(int m, bool full) { return (size_t)m * (full ? 4 : 1) + (full ? 1 : 0); }

// Partial-record views over one buffer of S * q * part_words(m, full) words.
inline Part part_views(void *base, int S, int q, int m, bool full)
{
    char *b = static_cast<char *>(base);
    const size_t per = (size_t)(S > 0 ? S : 1) * q;
    Part part{};
    part.cnt = reinterpret_cast<int32_t *>(b);
    if (full) {
        part.mt = reinterpret_cast<float *>(b + per * m * 4);
        part.sm = reinterpret_cast<float *>(b + per * m * 8);
        part.cs = reinterpret_cast<float *>(b + per * m * 12);
        part.nb = reinterpret_cast<int32_t *>(b + per * m * 16);
    }
    return part;
}

}  // namespace pair
}  // namespace csplat
