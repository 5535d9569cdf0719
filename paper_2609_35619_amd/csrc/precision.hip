// The MFMA precision form of the label path (labels and counts).
//
// For a sphere the two quantities that decide a pair are quadratic forms in
// the query centre (Eq. 5, 7 with A = I / r^2):
//   a = |mu - c|^2 - r^2                       (r^2 (s^2 - 1))
//   w = 4 n^2 (mu - c)^T Sigma (mu - c)        (r^4 n^2 sigma^2)
// and s~^2 < 1  <=>  a |a| < w (Eq. 8 without the square root).  About a
// tile-local origin o (mu' = mu - o, c' = c - o) both are dot products of
// query features with per-Gaussian coefficients:
//   a = [1, c'x, c'y, c'z, |c'|^2 - r^2] . [|mu'|^2, -2mu', 1]
//   w = 4n^2 [1, c', c'x^2, c'y^2, c'z^2, c'x c'y, c'x c'z, c'y c'z]
//          . [mu'^T Sigma mu', -2 Sigma mu', Sxx, Syy, Szz, 2Sxy, 2Sxz, 2Syz]
// so a tile of 32 Gaussians x 32 queries is a dense [32 x K] x [K x 32]
// contraction on the matrix cores.  Each feature x is split into x_hi + x_lo
// in bf16 (or fp16) and the contraction sums hi*hi + hi*lo + lo*hi in fp32
// (three products per feature: K = 15 for a, 30 for w), which brings the
// representation error to ~3u^2 of each product.  A certified per-pair
// bound B decides every pair whose |w - a|a|| exceeds it; the counts of
// certain and of possible collisions bracket the exact count, and only
// queries whose label the bracket cannot decide are re-evaluated in fp64.
#include <hipcub/hipcub.hpp>

#include <cmath>

#include "internal.h"
#include "pair_core.h"

namespace csplat {

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

constexpr int kPT = 512;             // Gaussians per tile (one origin)
constexpr int kRB = kPT / 32;        // row blocks (MFMA rows) per tile
constexpr int kOps = 3;              // operands per row block: a, w0, w1
constexpr int kMeta = 24;  // floats per tile: o(3), 1/scale, M1[5], M2[10], radius, largest scale, 0 0 0
constexpr int kChunksPerTile = kPT / pair::kCull;  // culling chunks per tile (two row blocks each)
constexpr int kLanes = 64;
constexpr float kU32 = 5.9604645e-08f;  // 2^-24

template <int P>
struct Prec;

template <>
struct Prec<CSPLAT_PRECISION_BF16_RECHECK> {
    using vec = bf16x8;
    using elem = __bf16;
    static constexpr float u = 0.00390625f;      // 2^-8: bf16 rounding error bound
    static constexpr float eta = 0.f;            // no subnormal loss in the bf16 range used
    static constexpr float far = 1099511627776.f;  // 2^40: padding rows, a = far
    __device__ static f32x16 mfma(vec a, vec b, f32x16 c)
    {
        return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0);
    }
};

template <>
struct Prec<CSPLAT_PRECISION_FP16_RECHECK> {
    using vec = f16x8;
    using elem = _Float16;
    static constexpr float u = 0.00048828125f;   // 2^-11
    static constexpr float eta = 5.9604645e-08f; // 2^-24: absolute loss of subnormal halves
    static constexpr float far = 32768.f;
    __device__ static f32x16 mfma(vec a, vec b, f32x16 c)
    {
        return __builtin_amdgcn_mfma_f32_32x32x16_f16(a, b, c, 0, 0, 0);
    }
};

// Slot order of the three products inside the K dimension.
//   a  (16 slots): hi.hi (5) | hi.lo (5) | lo.hi (5) | 0
//   w  (32 slots): hi.hi (10) | hi.lo (10) | lo.hi (10) | 0 0
// Gaussian side (A operand) value of slot s, query side (B operand) value:
__host__ __device__ inline int slot_feat_a(int s) { return s < 15 ? s % 5 : -1; }
__host__ __device__ inline int slot_part_g_a(int s) { return s < 5 ? 0 : (s < 10 ? 1 : 0); }  // 0 hi, 1 lo
__host__ __device__ inline int slot_part_q_a(int s) { return s < 10 ? 0 : 1; }
__host__ __device__ inline int slot_feat_w(int s) { return s < 30 ? s % 10 : -1; }
__host__ __device__ inline int slot_part_g_w(int s) { return (s >= 10 && s < 20) ? 1 : 0; }
__host__ __device__ inline int slot_part_q_w(int s) { return s >= 20 ? 1 : 0; }

// ---------------------------------------------------------------------------
// Load time: one block per tile; thread i holds Gaussian i of the tile.
template <int P>
__global__ void __launch_bounds__(kPT)
build_tiles_kernel(const float *__restrict__ gauss, int64_t n, float *__restrict__ meta,
                   typename Prec<P>::vec *__restrict__ feat)
{
    using T = Prec<P>;
    using elem = typename T::elem;
    using vec = typename T::vec;
    __shared__ float red[15][kPT];
    __shared__ float box[6];
    __shared__ double s_scale;
    const int64_t t = blockIdx.x;
    const int i = threadIdx.x;
    const int64_t gi = t * kPT + i;
    const bool valid = gi < n;
    const float *r = gauss + (size_t)kGaussFloats * (valid ? gi : 0);
    float mu[3] = {r[0], r[1], r[2]};
    // tile origin: centre of the bounding box of the tile's means (float32)
    for (int k = 0; k < 3; ++k) {
        red[k][i] = valid ? mu[k] : INFINITY;
        red[3 + k][i] = valid ? mu[k] : -INFINITY;
    }
    __syncthreads();
    if (i < 6) {
        float v = red[i][0];
        for (int j = 1; j < kPT; ++j) v = i < 3 ? fminf(v, red[i][j]) : fmaxf(v, red[i][j]);
        box[i] = v;
    }
    __syncthreads();
    const float o[3] = {0.5f * box[0] + 0.5f * box[3], 0.5f * box[1] + 0.5f * box[4],
                        0.5f * box[2] + 0.5f * box[5]};
    double p1[5] = {0, 0, 0, 0, 0}, p2[10] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
    if (valid) {
        double mp[3], S[9];
        for (int k = 0; k < 3; ++k) mp[k] = (double)mu[k] - (double)o[k];  // exact
        for (int a = 0; a < 3; ++a)  // Sigma = M^T M, M = diag(s) R^T
            for (int b = 0; b < 3; ++b) {
                double acc = 0.0;
                for (int k = 0; k < 3; ++k) acc += (double)r[3 + 3 * k + a] * (double)r[3 + 3 * k + b];
                S[3 * a + b] = acc;
            }
        double Sm[3];
        for (int a = 0; a < 3; ++a) Sm[a] = S[3 * a] * mp[0] + S[3 * a + 1] * mp[1] + S[3 * a + 2] * mp[2];
        p1[0] = mp[0] * mp[0] + mp[1] * mp[1] + mp[2] * mp[2];
        p1[1] = -2.0 * mp[0];
        p1[2] = -2.0 * mp[1];
        p1[3] = -2.0 * mp[2];
        p1[4] = 1.0;
        p2[0] = mp[0] * Sm[0] + mp[1] * Sm[1] + mp[2] * Sm[2];
        p2[1] = -2.0 * Sm[0];
        p2[2] = -2.0 * Sm[1];
        p2[3] = -2.0 * Sm[2];
        p2[4] = S[0];
        p2[5] = S[4];
        p2[6] = S[8];
        p2[7] = 2.0 * S[1];
        p2[8] = 2.0 * S[2];
        p2[9] = 2.0 * S[5];
    } else {
        p1[0] = T::far;  // padding row: a = far, w = 0, certainly free
    }
    // per-tile power-of-two scale of the w coefficients (keeps fp16 away from
    // its subnormal range; exact, undone on the query side)
    double mx2 = 0.0;
    for (int k = 0; k < 10; ++k) mx2 = fmax(mx2, fabs(p2[k]));
    red[0][i] = (float)mx2;
    __syncthreads();
    if (i == 0) {
        float v = 0.f;
        for (int j = 0; j < kPT; ++j) v = fmaxf(v, red[0][j]);
        s_scale = v > 0.f ? ldexp(1.0, 4 - ilogb((double)v)) : 1.0;
    }
    __syncthreads();
    const double scale = s_scale;
    for (int k = 0; k < 10; ++k) p2[k] *= scale;
    // hi/lo split
    float h1[5], l1[5], h2[10], l2[10];
    for (int k = 0; k < 5; ++k) {
        float x = (float)p1[k];
        h1[k] = (float)(elem)x;
        l1[k] = (float)(elem)(float)(p1[k] - (double)h1[k]);
    }
    for (int k = 0; k < 10; ++k) {
        float x = (float)p2[k];
        h2[k] = (float)(elem)x;
        l2[k] = (float)(elem)(float)(p2[k] - (double)h2[k]);
    }
    // packed operand layout: row block rb = i / 32, row m = i % 32; lane m + 32 h
    // holds K slots 8h .. 8h+7 of each operand
    const int rb = i >> 5, m = i & 31;
    for (int h = 0; h < 2; ++h) {
        const int lane = m + 32 * h;
        vec va, vw0, vw1;
        for (int j = 0; j < 8; ++j) {
            const int sa = 8 * h + j;
            const int fa = slot_feat_a(sa);
            va[j] = (elem)(fa < 0 ? 0.f : (slot_part_g_a(sa) ? l1[fa] : h1[fa]));
            const int s0 = 8 * h + j, s1 = 16 + 8 * h + j;
            const int f0 = slot_feat_w(s0), f1 = slot_feat_w(s1);
            vw0[j] = (elem)(f0 < 0 ? 0.f : (slot_part_g_w(s0) ? l2[f0] : h2[f0]));
            vw1[j] = (elem)(f1 < 0 ? 0.f : (slot_part_g_w(s1) ? l2[f1] : h2[f1]));
        }
        const size_t base = ((size_t)(t * kRB + rb) * kOps) * kLanes + lane;
        feat[base] = va;
        feat[base + kLanes] = vw0;
        feat[base + 2 * kLanes] = vw1;
    }
    // tile maxima of |hi| over the real rows, for the error bounds; the tile's
    // radius about the origin and its largest scale, for the reach test
    double rad = 0.0, smax = 0.0;
    if (valid) {
        double d2 = 0.0;
        for (int k = 0; k < 3; ++k) {
            const double dk = (double)mu[k] - (double)o[k];
            d2 += dk * dk;
            const double a = r[3 + 3 * k], b = r[4 + 3 * k], c = r[5 + 3 * k];
            smax = fmax(smax, sqrt(a * a + b * b + c * c));
        }
        rad = sqrt(d2);
    }
    __syncthreads();
    for (int k = 0; k < 5; ++k) red[k][i] = valid ? fabsf(h1[k]) : 0.f;
    for (int k = 0; k < 10; ++k) red[5 + k][i] = valid ? fabsf(h2[k]) : 0.f;
    __syncthreads();
    if (i < 15) {
        float v = 0.f;
        for (int j = 0; j < kPT; ++j) v = fmaxf(v, red[i][j]);
        meta[t * kMeta + 4 + i] = v;
    }
    __syncthreads();
    red[0][i] = (float)(rad * (1.0 + 1e-6));
    red[1][i] = (float)(smax * (1.0 + 1e-6));
    __syncthreads();
    if (i < 2) {
        float v = 0.f;
        for (int j = 0; j < kPT; ++j) v = fmaxf(v, red[i][j]);
        meta[t * kMeta + 19 + i] = v;
    }
    if (i == 0) {
        meta[t * kMeta + 0] = o[0];
        meta[t * kMeta + 1] = o[1];
        meta[t * kMeta + 2] = o[2];
        meta[t * kMeta + 3] = (float)(1.0 / scale);
        meta[t * kMeta + 21] = meta[t * kMeta + 22] = meta[t * kMeta + 23] = 0.f;
    }
}

// ---------------------------------------------------------------------------
// Query features relative to a tile.  A wave holds two 32-query column
// blocks; the B operand of column block cb at lane col + 32 h is K half h of
// query (cb, col).  Lane col + 32 h builds both K halves of query (h, col)
// once, and one exchange of the upper 32 lanes of the first half with the
// lower 32 lanes of the second (v_permlane32_swap) hands every lane the two
// operands it needs: the first register then holds column block 0, the
// second column block 1.
template <int P>
struct QFeat {
    typename Prec<P>::vec a, w0, w1;
    float two_ea, c0;
    // the minimum's epilogue: bounds of |a - a~| and of |w - w~| (inflated for
    // their own rounding) and sqrt of the latter
    float ea, ew, sew;
};

typedef unsigned u32x4 __attribute__((ext_vector_type(4)));

template <class V>
__device__ __forceinline__ void swap_halves(V &x, V &y)
{
    u32x4 bx = __builtin_bit_cast(u32x4, x), by = __builtin_bit_cast(u32x4, y);
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const auto r = __builtin_amdgcn_permlane32_swap(bx[i], by[i], false, false);
        bx[i] = r[0];
        by[i] = r[1];
    }
    x = __builtin_bit_cast(V, bx);
    y = __builtin_bit_cast(V, by);
}

__device__ __forceinline__ void swap_halves(float &x, float &y)
{
    const auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(x), __float_as_uint(y), false, false);
    x = __uint_as_float(r[0]);
    y = __uint_as_float(r[1]);
}

// Features of the lane's own query (cx, cy, cz, r2) about tile origin mt,
// exchanged into Q[0], Q[1]; returns false when a bound is not finite.
template <int P>
__device__ __forceinline__ bool build_query(float cx, float cy, float cz, float r2, float four_n2,
                                            const float *__restrict__ mt, QFeat<P> (&Q)[2])
{
    using T = Prec<P>;
    using elem = typename T::elem;
    const float xp = cx - mt[0], yp = cy - mt[1], zp = cz - mt[2];
    const float c2 = fmaf(zp, zp, fmaf(yp, yp, xp * xp));
    const float ph[5] = {1.f, xp, yp, zp, c2 - r2};
    const float g = four_n2 * mt[3];
    const float gx = g * xp, gy = g * yp, gz = g * zp;
    const float ch[10] = {g, gx, gy, gz, gx * xp, gy * yp, gz * zp, gx * yp, gx * zp, gy * zp};
    float h1[5], l1[5], h2[10], l2[10];
#pragma unroll
    for (int k = 0; k < 5; ++k) {
        h1[k] = (float)(elem)ph[k];
        l1[k] = (float)(elem)(ph[k] - h1[k]);
    }
#pragma unroll
    for (int k = 0; k < 10; ++k) {
        h2[k] = (float)(elem)ch[k];
        l2[k] = (float)(elem)(ch[k] - h2[k]);
    }
    // K halves 0 (slots 0-7) and 1 (slots 8-15) of a, of w's first and second
    // operand (slots 0-15, 16-31)
#pragma unroll
    for (int j = 0; j < 8; ++j) {
        const int sa0 = j, sa1 = 8 + j;
        const int fa0 = slot_feat_a(sa0), fa1 = slot_feat_a(sa1);
        Q[0].a[j] = (elem)(fa0 < 0 ? 0.f : (slot_part_q_a(sa0) ? l1[fa0] : h1[fa0]));
        Q[1].a[j] = (elem)(fa1 < 0 ? 0.f : (slot_part_q_a(sa1) ? l1[fa1] : h1[fa1]));
        const int s00 = j, s01 = 8 + j, s10 = 16 + j, s11 = 24 + j;
        const int f00 = slot_feat_w(s00), f01 = slot_feat_w(s01), f10 = slot_feat_w(s10), f11 = slot_feat_w(s11);
        Q[0].w0[j] = (elem)(f00 < 0 ? 0.f : (slot_part_q_w(s00) ? l2[f00] : h2[f00]));
        Q[1].w0[j] = (elem)(f01 < 0 ? 0.f : (slot_part_q_w(s01) ? l2[f01] : h2[f01]));
        Q[0].w1[j] = (elem)(f10 < 0 ? 0.f : (slot_part_q_w(s10) ? l2[f10] : h2[f10]));
        Q[1].w1[j] = (elem)(f11 < 0 ? 0.f : (slot_part_q_w(s11) ? l2[f11] : h2[f11]));
    }
    // certified error bounds of the computed a and w for this (query, tile):
    // per feature 3.1 u^2 |phi||psi| (split residuals and the dropped lo*lo),
    // an absolute eta per value (fp16 subnormal halves), 48 u32 for the float32
    // query features and the fp32 accumulation of up to 31 products, and the
    // rounding of |c'|^2 - r^2
    const float ue = 3.1f * T::u * T::u + 48.f * kU32;
    float sa = 0.f, sa_abs = 0.f, sw = 0.f, sw_abs = 0.f;
#pragma unroll
    for (int k = 0; k < 5; ++k) {
        sa = fmaf(fabsf(h1[k]), mt[4 + k], sa);
        sa_abs += fabsf(h1[k]) + mt[4 + k];
    }
#pragma unroll
    for (int k = 0; k < 10; ++k) {
        sw = fmaf(fabsf(h2[k]), mt[9 + k], sw);
        sw_abs += fabsf(h2[k]) + mt[9 + k];
    }
    const float ea = 1.1f * (ue * sa + T::eta * sa_abs + 4.f * kU32 * (c2 + r2));
    const float ew = 1.1f * (ue * sw + T::eta * sw_abs);
    const float two_ea = 2.f * ea, c0 = fmaf(ea, ea, ew) * 1.0001f;

    swap_halves(Q[0].a, Q[1].a);
    swap_halves(Q[0].w0, Q[1].w0);
    swap_halves(Q[0].w1, Q[1].w1);
    // the query's own scalars, then the same exchange of a register with
    // itself, which broadcasts column block 0's value to the first and
    // column block 1's to the second
    Q[0].two_ea = Q[1].two_ea = two_ea;
    Q[0].c0 = Q[1].c0 = c0;
    Q[0].ea = Q[1].ea = ea * 1.0001f;
    Q[0].ew = Q[1].ew = ew * 1.0001f;
    Q[0].sew = Q[1].sew = sqrtf(ew);
    swap_halves(Q[0].two_ea, Q[1].two_ea);
    swap_halves(Q[0].c0, Q[1].c0);
    swap_halves(Q[0].ea, Q[1].ea);
    swap_halves(Q[0].ew, Q[1].ew);
    swap_halves(Q[0].sew, Q[1].sew);
    return isfinite(two_ea) && isfinite(c0) && isfinite(sa) && isfinite(sw);
}

// ---------------------------------------------------------------------------
// Certification kernel: block = 4 waves x 32 kCB queries (kCB 32-query
// column blocks per wave); grid = query blocks x S splits, split s taking the tiles
// s, s + S, s + 2S, ... (every split samples the whole scene, so the work of
// a query block is spread evenly over its S items).
// With CULL, a column block skips row blocks in pairs (one culling chunk of
// 64 Gaussians) when each of its 32 queries is beyond the chunk's reach
// bound n s_c + sqrt(n^2 s_c^2 + r^2) plus its radius: no pair of them can
// collide.  Chunks are tested 64 at a time (8 tiles x 8 chunks, one per lane;
// over a large scene the 16 chunks of each group that survived a test of 64
// groups) against the wave's bounding sphere and box, then each survivor
// against every query.
// Column blocks of 32 queries per wave: the A operands of a row block are
// loaded once and multiplied against every column block that needs them.
#ifndef CSPLAT_MFMA_COLUMN_BLOCKS
#define CSPLAT_MFMA_COLUMN_BLOCKS 2
#endif
constexpr int kCB = CSPLAT_MFMA_COLUMN_BLOCKS;
static_assert(kCB == 2 || kCB == 4, "column blocks per wave: 2 or 4");
constexpr int kQueriesPerBlock = 4 * 32 * kCB;
// the ellipsoid MFMA kernel keeps two column blocks per wave (one body per lane
// builds its features) whatever kCB is
constexpr int kEllCB = 2;
constexpr int kEllQueriesPerBlock = 4 * 32 * kEllCB;

// The minimum (MINW): per pair v~ = a~ - sqrt(max(w~, 0)), the computed value
// of v = a - sqrt(w) = r^2 (s~^2 - 1) before the clamp, and a certified bound
// e >= |v~ - v|: the contraction's bound E_a on a, E_w / max(sqrt(w~),
// sqrt(E_w)) on the square root (for w~ >= E_w, |sqrt(w) - sqrt(w~)| <=
// E_w / sqrt(w~); below, <= sqrt(E_w)), and the float32 rounding of the
// square root and the difference (8 u (|a~| + sqrt(w~)), generous).  The lane
// keeps the computed minimum m = min v~, lo = min(v~ - e) and
// up = min(v~ + e): the exact minimum over the evaluated pairs lies in
// [lo, up], and so does m.  With `thr` (per query; NULL: 1) the
// reach is that of s~^2 < thr[j]: every pair below the threshold is
// evaluated (the passes of the minimum search).  COUNT = false skips the
// label counts.
template <int P, bool CULL, bool COUNT = true, bool MINW = false>
__global__ void __launch_bounds__(256)
mfma_label_kernel(const typename Prec<P>::vec *__restrict__ feat, const float *__restrict__ meta,
                  int n_tiles, int S, int n_qblocks, const float *__restrict__ cull, int n_chunks,
                  const float *__restrict__ centers, const float *__restrict__ radii, int q, float four_n2,
                  float n_sigma, int32_t *__restrict__ lo_out, int32_t *__restrict__ hi_out,
                  const float *__restrict__ groups, const float *__restrict__ thr = nullptr,
                  float *__restrict__ mlo_out = nullptr,
                  float *__restrict__ mup_out = nullptr, unsigned long long *__restrict__ blocks_done = nullptr)
{
    static_assert(COUNT || MINW, "nothing to compute");
    using T = Prec<P>;
    using vec = typename T::vec;
    constexpr int kG = kCB / 2;  // queries each lane builds features for
    int b = blockIdx.x;
    const int B = gridDim.x;
    if ((B & 7) == 0) b = (b & 7) * (B >> 3) + (b >> 3);  // XCD-major: one XCD, few splits
    const int split = b / n_qblocks;
    const int qb = b - split * n_qblocks;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, col = lane & 31, h = lane >> 5;
    float cx[kCB], cy[kCB], cz[kCB], r2[kCB], qa[kCB];  // qa: the reach's r^2 (times the threshold)
    int jq[kCB];
#pragma unroll
    for (int cb = 0; cb < kCB; ++cb) {
        jq[cb] = qb * kQueriesPerBlock + wave * (32 * kCB) + cb * 32 + col;
        const int jj = jq[cb] < q ? jq[cb] : q - 1;
        cx[cb] = centers[3 * jj];
        cy[cb] = centers[3 * jj + 1];
        cz[cb] = centers[3 * jj + 2];
        const float r = radii[jj];
        r2[cb] = r * r;
        qa[cb] = MINW && thr ? r2[cb] * thr[jj] : r2[cb];
    }
    float mlo[kCB], mup[kCB], mmv[kCB];
#pragma unroll
    for (int cb = 0; cb < kCB; ++cb) mlo[cb] = mup[cb] = mmv[cb] = INFINITY;
    unsigned long long n_blocks = 0;
    int lo[kCB], hi[kCB];
    bool bad[kG];  // a non-finite bound for the lane's own query of column block pair g
#pragma unroll
    for (int cb = 0; cb < kCB; ++cb) lo[cb] = hi[cb] = 0;
#pragma unroll
    for (int g = 0; g < kG; ++g) bad[g] = false;
    // the lane builds the features of query (2 g + h, col) for each pair g
    float ox[kG], oy[kG], oz[kG], or2[kG];
#pragma unroll
    for (int g = 0; g < kG; ++g) {
        ox[g] = h ? cx[2 * g + 1] : cx[2 * g];
        oy[g] = h ? cy[2 * g + 1] : cy[2 * g];
        oz[g] = h ? cz[2 * g + 1] : cz[2 * g];
        or2[g] = h ? r2[2 * g + 1] : r2[2 * g];
    }
    const f32x16 zero = {};
    // tile t: row block rb against column block cb where bit rb of rbm[cb]
    // is set (wave-uniform masks)
    auto do_tile = [&](int t, const unsigned (&rbm_cb)[kCB]) {
        const float *mt = meta + (size_t)t * kMeta;  // wave-uniform: scalar loads
        QFeat<P> Q[kCB];
#pragma unroll
        for (int g = 0; g < kG; ++g) {
            QFeat<P> Qg[2];
            bad[g] |= !build_query<P>(ox[g], oy[g], oz[g], or2[g], four_n2, mt, Qg);
            Q[2 * g] = Qg[0];
            Q[2 * g + 1] = Qg[1];
        }
        const vec *ft = feat + (size_t)t * kRB * kOps * kLanes + lane;
        unsigned rbm = 0;
#pragma unroll
        for (int cb = 0; cb < kCB; ++cb) rbm |= rbm_cb[cb];
        if (!rbm) return;
        // the next row block's operands are requested before the current
        // one is evaluated, so their loads overlap its MFMAs and epilogue
        // (loaded just before use, every row block waited a memory round trip)
        int nrb = __builtin_ctz(rbm);
        rbm &= rbm - 1;
        vec nAa, nAw0, nAw1;
        {
            const vec *fp = ft + (size_t)nrb * kOps * kLanes;
            nAa = fp[0], nAw0 = fp[kLanes], nAw1 = fp[2 * kLanes];
        }
        for (;;) {
            const int rb = nrb;
            const vec Aa = nAa, Aw0 = nAw0, Aw1 = nAw1;
            const bool more = rbm != 0;
            if (more) {
                nrb = __builtin_ctz(rbm);
                rbm &= rbm - 1;
                const vec *fp = ft + (size_t)nrb * kOps * kLanes;
                nAa = fp[0], nAw0 = fp[kLanes], nAw1 = fp[2 * kLanes];
            }
#pragma unroll
            for (int cb = 0; cb < kCB; ++cb) {
                if (!((rbm_cb[cb] >> rb) & 1u)) continue;  // no query of cb near the row block
                ++n_blocks;
                const f32x16 A = T::mfma(Aa, Q[cb].a, zero);
                f32x16 W = T::mfma(Aw0, Q[cb].w0, zero);
                W = T::mfma(Aw1, Q[cb].w1, W);
                if constexpr (COUNT) {
                    const float te = Q[cb].two_ea, c0 = Q[cb].c0;
                    float f[16], bnd[16];
                    bool poss = false;
#pragma unroll
                    for (int i = 0; i < 16; ++i) {
                        const float a = A[i], aa = fabsf(a);
                        f[i] = fmaf(-a, aa, W[i]);      // w - a|a|: > 0 iff collision
                        bnd[i] = fmaf(aa, te, c0);      // certified |f - f_exact| bound
                        poss |= f[i] > -bnd[i];
                    }
                    // most blocks hold no possible collision (and so no certain
                    // one): count only where some lane has one
                    if (__any(poss)) {
#pragma unroll
                        for (int i = 0; i < 16; ++i) {
                            lo[cb] += f[i] > bnd[i];    // certainly in collision
                            hi[cb] += f[i] > -bnd[i];   // possibly in collision
                        }
                    }
                }
                if constexpr (MINW) {
                    const float ea = Q[cb].ea, ew = Q[cb].ew, sew = Q[cb].sew;
#pragma unroll
                    for (int i = 0; i < 16; ++i) {
                        const float a = A[i];
                        const float sq = pair::fast_sqrt(fmaxf(W[i], 0.f));
                        const float v = a - sq;
                        // v_rcp: ~1 ulp, covered by the 1.0001 of ew; the floor keeps
                        // es = 0 (not 0 x inf) when E_w = 0 (n_sigma = 0)
                        const float es = ew * __builtin_amdgcn_rcpf(fmaxf(fmaxf(sq, sew), 1e-30f));
                        const float e = fmaf(fabsf(a) + sq, 8.f * kU32, ea + es);
                        mmv[cb] = fminf(mmv[cb], v);
                        mlo[cb] = fminf(mlo[cb], v - e);
                        mup[cb] = fminf(mup[cb], v + e);
                    }
                }
            }
            if (!more) break;
        }
    };
    if constexpr (!CULL) {
        unsigned all[kCB];
#pragma unroll
        for (int cb = 0; cb < kCB; ++cb) all[cb] = 0xffffu;
        for (int t = split; t < n_tiles; t += S) do_tile(t, all);
    } else {
        float wx, wy, wz, spread, r2max, half[3];
        pair::wave_sphere<kCB>(cx, cy, cz, qa, wx, wy, wz, spread, r2max, half);
        auto reach_of = [&](const pair::ChunkMeta &m, float rr2) {
            const float ns = n_sigma * m.smax;
            return ns + pair::fast_sqrt(fmaf(ns, ns, rr2));  // ~1 ulp, far inside the culling margin
        };
        // against the wave's bounding sphere and box
        auto coarse = [&](const pair::ChunkMeta &m) {
            const float reach = m.rad + reach_of(m, r2max);
            return pair::within(m, wx, wy, wz, spread + reach) && pair::within_box(m, wx, wy, wz, half, reach);
        };
        // Over a large scene (more than kGroupDealChunks chunks per split)
        // split s takes the groups of 16 chunks (two tiles) s, s + S, ...: 64
        // groups at a time against the wave, then the 16 chunks of a
        // surviving group; otherwise it takes the tiles s, s + S, ...: the
        // chunks of 8 tiles at a time against the wave (the choice and its
        // reason as in the float32 label walk).  Then per tile each surviving
        // chunk against the queries of every column block.
        const int n_groups = (n_chunks + pair::kGroup - 1) / pair::kGroup;
        static_assert(pair::kGroup == 2 * kChunksPerTile, "a group holds two tiles");
        const bool by_group = n_chunks > pair::kGroupDealChunks * S;
        const int n_units = by_group ? n_groups : n_tiles;
        const int per_batch = by_group ? 64 : 64 / kChunksPerTile;
        for (int ib = 0; split + ib * S < n_units; ib += per_batch) {
            // one group per lane, or one chunk per lane (8 per tile)
            pair::ChunkMeta bm{0.f, 0.f, 0.f, 0.f, 0.f};
            bool bpass = false;
            if (by_group) {
                const int gl = split + (ib + lane) * S;
                if (gl < n_groups) {
                    bm = pair::load_chunk(groups, gl);
                    bpass = coarse(bm);
                }
            } else {
                const int t = split + (ib + lane / kChunksPerTile) * S;
                const int ci = t * kChunksPerTile + lane % kChunksPerTile;
                if (t < n_tiles && ci < n_chunks) {
                    bm = pair::load_chunk(cull, ci);
                    bpass = coarse(bm);
                }
            }
            const unsigned long long bmask = __ballot(bpass);
            // the surviving groups to open, or the batch itself as one set of chunks
            unsigned long long gmask = by_group ? bmask : 1ull;
            while (gmask) {
                pair::ChunkMeta m = bm;
                unsigned long long mask = bmask;
                int gi = 0;
                if (by_group) {
                    gi = split + (ib + __builtin_ctzll(gmask)) * S;
                    const int ci = gi * pair::kGroup + lane;  // the group's chunks, one per lane
                    bool pass = false;
                    m = pair::ChunkMeta{0.f, 0.f, 0.f, 0.f, 0.f};
                    if (lane < pair::kGroup && ci < n_chunks) {
                        m = pair::load_chunk(cull, ci);
                        pass = coarse(m);
                    }
                    mask = __ballot(pass);
                }
                gmask &= gmask - 1;
                while (mask) {
                    const int g = __builtin_ctzll(mask) / kChunksPerTile;  // tile of the set
                    unsigned tm = (unsigned)(mask >> (kChunksPerTile * g)) & ((1u << kChunksPerTile) - 1u);
                    mask &= ~((((unsigned long long)1 << kChunksPerTile) - 1ull) << (kChunksPerTile * g));
                    // per column block: the chunk's two row blocks where some
                    // query of the block is within reach (testing each row block
                    // through its two 16-Gaussian sub-chunks cost more than the
                    // blocks it skipped: 1.19 -> 1.30 ms on the precision workload)
                    const int t = by_group ? gi * (pair::kGroup / kChunksPerTile) + g : split + (ib + g) * S;
                    unsigned rbm[kCB];
#pragma unroll
                    for (int cb = 0; cb < kCB; ++cb) rbm[cb] = 0;
                    unsigned any = 0;
                    while (tm) {
                        const int k = __builtin_ctz(tm);
                        tm &= tm - 1;
                        const pair::ChunkMeta c = pair::lane_chunk(m, kChunksPerTile * g + k);
#pragma unroll
                        for (int cb = 0; cb < kCB; ++cb)
                            if (__any(pair::within(c, cx[cb], cy[cb], cz[cb], c.rad + reach_of(c, qa[cb]))))
                                rbm[cb] |= 3u << (2 * k);
                    }
#pragma unroll
                    for (int cb = 0; cb < kCB; ++cb) any |= rbm[cb];
                    if (any) do_tile(t, rbm);
                }
            }
        }
    }
#pragma unroll
    for (int cb = 0; cb < kCB; ++cb) {
        lo[cb] += __shfl_xor(lo[cb], 32);
        hi[cb] += __shfl_xor(hi[cb], 32);
        mlo[cb] = fminf(mlo[cb], __shfl_xor(mlo[cb], 32));
        mup[cb] = fminf(mup[cb], __shfl_xor(mup[cb], 32));
        mmv[cb] = fminf(mmv[cb], __shfl_xor(mmv[cb], 32));
        // the query of column block cb was built by the lanes of half cb & 1
        const int g = cb >> 1;
        const bool other = __shfl_xor((int)bad[g], 32) != 0;
        const bool anybad = (h == (cb & 1)) ? bad[g] : other;
        if (h == 0 && jq[cb] < q) {
            if constexpr (COUNT) {
                lo_out[(size_t)split * q + jq[cb]] = lo[cb];
                hi_out[(size_t)split * q + jq[cb]] = anybad ? (1 << 29) : hi[cb];
            }
            if constexpr (MINW) {
                // a bound that is not finite leaves the interval open: (-inf, up]
                mlo_out[(size_t)split * q + jq[cb]] = anybad ? -INFINITY : mlo[cb];
                mup_out[(size_t)split * q + jq[cb]] = anybad ? INFINITY : mup[cb];
                mlo_out[((size_t)S + split) * q + jq[cb]] = mmv[cb];  // the computed minimum after the bounds
            }
        }
    }
    if (blocks_done && lane == 0) atomicAdd(blocks_done, n_blocks);
}

// Merge the splits, decide certified labels (written to the caller's row
// perm[j]) and flag the rest for the recheck.
__global__ void __launch_bounds__(256)
decide_kernel(int q, int S, int m, int v, int k, bool want_count, const int32_t *__restrict__ lo_in,
              const int32_t *__restrict__ hi_in, const int32_t *__restrict__ perm, uint8_t *label, int32_t *count,
              uint8_t *__restrict__ flag)
{
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= q) return;
    int lo = 0, hi = 0;
    for (int s = 0; s < S; ++s) {
        lo += lo_in[(size_t)s * q + j];
        hi = min(hi + hi_in[(size_t)s * q + j], 1 << 29);
    }
    const bool certain = (lo > k || hi <= k) && (!want_count || lo == hi);
    const int oj = perm ? perm[j] : j;
    if (certain) {
        if (label) label[(size_t)oj * m + v] = lo > k ? 1 : 0;
        if (count) count[(size_t)oj * m + v] = lo;
    }
    flag[j] = certain ? 0 : 1;
}

// fp64 recheck of the listed queries.  One wave per work item: a tile of 64
// listed queries (one per lane) x split s of kRecheckSplits (the culling
// chunks s, s + kRecheckSplits, ...).  Chunks are tested 64 at a time
// against the bounding sphere of the tile's queries, then each survivor
// against every query (ballot); a surviving chunk is evaluated with one
// Gaussian per lane (coalesced record loads) for each query that needs it,
// the per-query hit count taken with a ballot.  Exact counts are summed in
// integers (order-free).  Without culling metadata every chunk is evaluated
// for every query.
constexpr int kRecheckSplits = 256;
constexpr int kRecheckWaves = 4;      // waves per block
constexpr int kRecheckGrid = 2048;    // blocks (persistent)

__global__ void __launch_bounds__(64 * kRecheckWaves)
recheck_fp64_kernel(const float *__restrict__ gauss, int n, const float *__restrict__ cull,
                    const float *__restrict__ centers, const float *__restrict__ radii, float n_sigma,
                    const int32_t *__restrict__ list, const int32_t *__restrict__ n_list, int32_t *__restrict__ exact)
{
    const int nl = *n_list;
    const int tiles = (nl + 63) / 64;
    const long items = (long)tiles * kRecheckSplits;
    const int n_chunks = (n + pair::kCull - 1) / pair::kCull;
    const int lane = (int)(threadIdx.x & 63u);
    const double four_n2 = 4.0 * (double)n_sigma * (double)n_sigma;
    const long wave0 = (long)blockIdx.x * kRecheckWaves + (long)(threadIdx.x >> 6);
    const long waves = (long)gridDim.x * kRecheckWaves;
    for (long item = wave0; item < items; item += waves) {
        const int tile = (int)(item / kRecheckSplits), split = (int)(item - (long)tile * kRecheckSplits);
        const int li = tile * 64 + lane;
        const bool valid = li < nl;
        const int j = list[valid ? li : nl - 1];
        float fc[3][1] = {{centers[3 * j]}, {centers[3 * j + 1]}, {centers[3 * j + 2]}};
        const float fr = radii[j];
        float fr2[1] = {fr * fr};
        int cnt = 0;  // exact count of this lane's query
        // chunk ci against the queries of qmask: lanes hold the chunk's Gaussians
        auto chunk = [&](int ci, unsigned long long qmask) {
            const int g = ci * pair::kCull + lane;
            const bool real = g < n;
            const float *p = gauss + (size_t)kGaussFloats * (real ? g : n - 1);
            double mu[3], M[9];
            for (int k = 0; k < 3; ++k) mu[k] = p[k];
            for (int k = 0; k < 9; ++k) M[k] = p[3 + k];
            while (qmask) {
                const int b = __builtin_ctzll(qmask);
                qmask &= qmask - 1;
                const double cx = pair::lane_value(fc[0][0], b), cy = pair::lane_value(fc[1][0], b),
                             cz = pair::lane_value(fc[2][0], b);
                const double rb = pair::lane_value(fr, b);
                const double dx = mu[0] - cx, dy = mu[1] - cy, dz = mu[2] - cz;
                const double a = dx * dx + dy * dy + dz * dz - rb * rb;
                const double e0 = M[0] * dx + M[1] * dy + M[2] * dz;
                const double e1 = M[3] * dx + M[4] * dy + M[5] * dz;
                const double e2 = M[6] * dx + M[7] * dy + M[8] * dz;
                const bool hit = real && a * fabs(a) < four_n2 * (e0 * e0 + e1 * e1 + e2 * e2);
                const int h = __popcll(__ballot(hit));
                if (lane == b) cnt += h;
            }
        };
        const unsigned long long vmask = __ballot(valid);
        if (cull) {
            float wx, wy, wz, spread, r2max;
            pair::wave_sphere<1>(fc[0], fc[1], fc[2], fr2, wx, wy, wz, spread, r2max);
            auto reach_of = [&](const pair::ChunkMeta &m, float rr2) {
                const float ns = n_sigma * m.smax;
                return ns + pair::fast_sqrt(fmaf(ns, ns, rr2));  // ~1 ulp, far inside the culling margin
            };
            for (int ib = 0; split + ib * kRecheckSplits < n_chunks; ib += 64) {
                const int ci = split + (ib + lane) * kRecheckSplits;
                pair::ChunkMeta m{0.f, 0.f, 0.f, 0.f, 0.f};
                bool pass = false;
                if (ci < n_chunks) {
                    m = pair::load_chunk(cull, ci);
                    pass = pair::within(m, wx, wy, wz, spread + m.rad + reach_of(m, r2max));
                }
                unsigned long long mask = __ballot(pass);
                while (mask) {
                    const int bit = __builtin_ctzll(mask);
                    mask &= mask - 1;
                    const pair::ChunkMeta k = pair::lane_chunk(m, bit);
                    const bool near = pair::within(k, fc[0][0], fc[1][0], fc[2][0], k.rad + reach_of(k, fr2[0]));
                    const unsigned long long qmask = __ballot(near) & vmask;
                    if (qmask) chunk(split + (ib + bit) * kRecheckSplits, qmask);
                }
            }
        } else {
            for (int ci = split; ci < n_chunks; ci += kRecheckSplits) chunk(ci, vmask);
        }
        if (valid && cnt) atomicAdd(exact + li, cnt);
    }
}

__global__ void finish_kernel(int m, int v, int k, const int32_t *__restrict__ list,
                              const int32_t *__restrict__ n_list, const int32_t *__restrict__ exact,
                              const int32_t *__restrict__ perm, uint8_t *label, int32_t *count)
{
    const int li = blockIdx.x * blockDim.x + threadIdx.x;
    if (li >= *n_list) return;
    const int j = list[li];
    const int oj = perm ? perm[j] : j;
    if (label) label[(size_t)oj * m + v] = exact[li] > k ? 1 : 0;
    if (count) count[(size_t)oj * m + v] = exact[li];
}

// ---------------------------------------------------------------------------
// The minimum of s~^2 over every kept Gaussian in the precision forms: passes
// of mfma_label_kernel with the minimum's epilogue and a rising threshold
// (as the float32 search: every pair with s~^2 < T is evaluated; a query is
// resolved once its certified upper bound lies below T; otherwise the next
// threshold lies just above that bound, or four times the last one when no
// pair was in reach).  State per query (sorted order): the interval
// [lo, up] of v = r^2 (s~^2 - 1), the threshold, and a flag (0 resolved,
// 1 searching, 2 fp64 fallback: a low-precision bound was not finite).
constexpr float kMinResolveP = 0.9990234375f;  // 1 - 2^-10
constexpr float kMinNextP = 1.00390625f;       // 1 + 2^-8

__global__ void __launch_bounds__(256)
pmin_combine_kernel(int nq, int S, const int32_t *__restrict__ list, const float *__restrict__ radii,
                    const float *__restrict__ mlo, const float *__restrict__ mup, float *__restrict__ st_lo,
                    float *__restrict__ st_up, float *__restrict__ st_mv, float *__restrict__ st_thr,
                    uint8_t *__restrict__ flag, bool first)
{
    // one wave per query, its lanes striding over the splits (minima: any order)
    const int i = (int)(((size_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6);
    const int lane = (int)(threadIdx.x & 63u);
    if (i >= nq) return;  // wave-uniform
    const int j = list ? list[i] : i;
    float lo = INFINITY, up = INFINITY, mv = INFINITY;
    for (int s = lane; s < S; s += 64) {
        lo = fminf(lo, mlo[(size_t)s * nq + i]);
        up = fminf(up, mup[(size_t)s * nq + i]);
        mv = fminf(mv, mlo[((size_t)S + s) * nq + i]);
    }
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        lo = fminf(lo, __shfl_xor(lo, off));
        up = fminf(up, __shfl_xor(up, off));
        mv = fminf(mv, __shfl_xor(mv, off));
    }
    if (lane != 0) return;
    if (first) st_thr[j] = 1.f;
    const float r = radii[j], r2 = r * r;
    st_lo[j] = lo;
    st_up[j] = up;
    st_mv[j] = mv;
    // resolved: the exact minimum over the evaluated pairs (<= up + r^2) lies
    // below the threshold, so no skipped pair is lower
    flag[j] = lo == -INFINITY ? 2 : (up + r2 < r2 * st_thr[j] * kMinResolveP ? 0 : 1);
}

__global__ void __launch_bounds__(256)
pmin_gather_kernel(int nl, const int32_t *__restrict__ list, const float *__restrict__ centers,
                   const float *__restrict__ radii, const float *__restrict__ st_up, float *__restrict__ st_thr,
                   float *__restrict__ cc, float *__restrict__ rr, float *__restrict__ tt)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nl) return;
    const int j = list[i];
    const float r = radii[j], r2 = r * r;
    const float up = st_up[j];
    // just above the certified upper bound of the minimum, or four times the
    // last threshold when no pair was in reach
    const float t = up < INFINITY ? fmaxf(up + r2, 0.f) / r2 * kMinNextP : 4.f * st_thr[j];
    st_thr[j] = fmaxf(t, st_thr[j] * kMinNextP);
    tt[i] = st_thr[j];
    cc[3 * i] = centers[3 * j];
    cc[3 * i + 1] = centers[3 * j + 1];
    cc[3 * i + 2] = centers[3 * j + 2];
    rr[i] = r;
}

// fp64 minimum of t = |d|^2 - 2 n sqrt(d^T Sigma d) (clamped at 0; r^2
// s~^2) over every kept Gaussian for the listed queries: one wave per (listed
// query, split of kRecheckSplits), strided Gaussians, a wave minimum, and an
// atomic minimum on the bits of the non-negative double.
__global__ void __launch_bounds__(64 * kRecheckWaves)
min_fp64_kernel(const float *__restrict__ gauss, int n, const float *__restrict__ centers, float n_sigma,
                const int32_t *__restrict__ list, const int32_t *__restrict__ n_list,
                unsigned long long *__restrict__ best)
{
    const int nl = *n_list;
    const long items = (long)nl * kRecheckSplits;
    const int lane = (int)(threadIdx.x & 63u);
    const long wave0 = (long)blockIdx.x * kRecheckWaves + (long)(threadIdx.x >> 6);
    const long waves = (long)gridDim.x * kRecheckWaves;
    const double two_n = 2.0 * (double)n_sigma;
    for (long item = wave0; item < items; item += waves) {
        const int li = (int)(item / kRecheckSplits), split = (int)(item - (long)li * kRecheckSplits);
        const int j = list[li];
        const double cx = centers[3 * j], cy = centers[3 * j + 1], cz = centers[3 * j + 2];
        double best_t = INFINITY;
        for (long g = (long)split * 64 + lane; g < n; g += 64L * kRecheckSplits) {
            const float *p = gauss + (size_t)kGaussFloats * g;
            const double dx = (double)p[0] - cx, dy = (double)p[1] - cy, dz = (double)p[2] - cz;
            const double e0 = (double)p[3] * dx + (double)p[4] * dy + (double)p[5] * dz;
            const double e1 = (double)p[6] * dx + (double)p[7] * dy + (double)p[8] * dz;
            const double e2 = (double)p[9] * dx + (double)p[10] * dy + (double)p[11] * dz;
            const double t = dx * dx + dy * dy + dz * dz - two_n * sqrt(e0 * e0 + e1 * e1 + e2 * e2);
            best_t = fmin(best_t, t > 0.0 ? t : 0.0);
        }
        for (int off = 32; off >= 1; off >>= 1) best_t = fmin(best_t, __shfl_xor(best_t, off));
        if (lane == 0 && best_t < INFINITY) atomicMin(best + li, (unsigned long long)__double_as_longlong(best_t));
    }
}

// Results at row perm[j]: min = the computed minimum (clamped) over r^2,
// err = its distance to the farther end of the clamped certified interval
// plus the float32 rounding of the additions and the division; fp64 fallback
// queries (flag 2, listed in `list2` with `best`): the fp64 minimum rounded
// to float32 (err: one float32 ulp of it).
__global__ void __launch_bounds__(256)
pmin_output_kernel(int q, int m, int v, const float *__restrict__ radii, const int32_t *__restrict__ perm,
                   const float *__restrict__ st_lo, const float *__restrict__ st_up,
                   const float *__restrict__ st_mv, const uint8_t *__restrict__ flag,
                   const int32_t *__restrict__ slot, const unsigned long long *__restrict__ best, float *out_min,
                   float *out_err)
{
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= q) return;
    const int oj = perm ? perm[j] : j;
    const float r = radii[j], r2 = r * r;
    float mn, err;
    if (flag[j] == 2) {
        const double t = __longlong_as_double((long long)best[slot[j]]);
        mn = (float)(t / ((double)r * (double)r));
        err = 1.1920929e-07f * mn;  // 2^-23 |min|
    } else if (!(st_up[j] < INFINITY)) {  // no Gaussian at all
        mn = INFINITY;
        err = 0.f;
    } else {
        const float tl = fmaxf(st_lo[j] + r2, 0.f), tu = fmaxf(st_up[j] + r2, 0.f);
        const float tm = fminf(fmaxf(st_mv[j] + r2, tl), tu);
        const float dev = fmaxf(tm - tl, tu - tm) + 4.f * kU32 * (fabsf(st_lo[j]) + fabsf(st_up[j]) + 2.f * r2);
        mn = tm / r2;
        err = dev / r2 * 1.000001f + 2.f * kU32 * mn;
    }
    if (out_min) out_min[(size_t)oj * m + v] = mn;
    if (out_err) out_err[(size_t)oj * m + v] = err;
}

// Slot of each fp64 fallback query in the list (filled for the listed ones).
__global__ void pmin_slot_kernel(const int32_t *__restrict__ list, const int32_t *__restrict__ n_list,
                                 int32_t *__restrict__ slot)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < *n_list) slot[list[i]] = i;
}

// ---------------------------------------------------------------------------
// The MFMA form for ellipsoidal bodies (Eq. 5-6 with a general A).
//
// For a body with centre c, its float32 L (A = L^T L) and B = L^T L formed
// once in float32 (the fp64 recheck takes the same L and B), and a Gaussian
// (mu, M), with d = mu - c:
//   a = |L d|^2 - 1 = sum_k f_k^2 - 1,          f_k = L_k . d      (s^2 - 1)
//   w = 4 n^2 |M B d|^2 = sum_k e_k^2,          e_k = 2n M_k . (B d) (n^2 sigma^2)
// and s~^2 < 1  <=>  a |a| < w.  About a tile origin o (mu' = mu - o,
// c' = c - o, beta = B c'), each is a dot product of Gaussian and body
// features:
//   f_k = [mu'x, mu'y, mu'z, 1] . [L_k0, L_k1, L_k2, -(L c')_k]
//   e_k = [M_kp mu'_m (p, m = 0..2), M_k0, M_k1, M_k2]
//       . 2n [B_pm (p, m = 0..2), -beta_0, -beta_1, -beta_2]
// (the Gaussian side of the three f_k and the body side of the three e_k are
// shared): per 32 x 32 block one MFMA for each f_k (K = 16 with the three
// hi/lo products) and three for each e_k (K = 48), and the squares are
// summed per pair.  Linear forms keep the cancellation about the tile origin
// to |o - c| / |d| (the quadratic form of a, or of w with its 60 features
// Sigma x mu mu^T, squares it).
//
// Bounds per (body, tile): E_f >= |f~_k - f_k| and E_e >= |e~_k - e_k| as for
// spheres (3.1 u^2 of sum |g||q| for the split, 64 u32 for the fp32 sums of
// up to 48 exact products, the fp32 errors of the body features, eta per
// value for fp16 subnormals).  Per pair, with F = sum |f~_k| and
// S = sum |e~_k|:
//   |a~ - a| <= E_a = 2 E_f F + 3 E_f^2 + 2 u32 (|a~| + 1)
//   |w~ - w| <= E_w = 2 E_e S + 3 E_e^2 + 6 u32 w~
// and w~ - a~|a~| is within 2 |a~| E_a + E_a^2 + E_w (+ its rounding) of w - a|a|.
constexpr int kEllF = 4, kEllE = 12;   // features of each f_k and of each e_k
constexpr int kEllOps = 1 + 3 * 3;     // Gaussian operand vectors per row block: f (1), e_0, e_1, e_2 (3 each)
constexpr int kEllMeta = 24;  // floats per tile: o(3), 1/scale of e, Gf[4], Ge[12], radius, largest scale, 0 0

// Slot s of an operand with nf features: hi.hi (nf) | hi.lo (nf) | lo.hi (nf) | 0;
// the Gaussian side takes its lo part in the second group, the body side in the third.
__host__ __device__ inline int eslot_feat(int s, int nf) { return s < 3 * nf ? s % nf : -1; }
__host__ __device__ inline bool eslot_glo(int s, int nf) { return s >= nf && s < 2 * nf; }
__host__ __device__ inline bool eslot_qlo(int s, int nf) { return s >= 2 * nf && s < 3 * nf; }

// Load time: one block per tile of kPT Gaussians; thread i holds Gaussian i.
template <int P>
__global__ void __launch_bounds__(kPT)
build_tiles_ell_kernel(const float *__restrict__ gauss, int64_t n, float *__restrict__ meta,
                       typename Prec<P>::vec *__restrict__ feat)
{
    using T = Prec<P>;
    using elem = typename T::elem;
    using vec = typename T::vec;
    __shared__ float red[kEllF + kEllE][kPT];
    __shared__ float box[6];
    __shared__ double s_scale;
    const int64_t t = blockIdx.x;
    const int i = threadIdx.x;
    const int64_t gi = t * kPT + i;
    const bool valid = gi < n;
    const float *r = gauss + (size_t)kGaussFloats * (valid ? gi : 0);
    const float mu[3] = {r[0], r[1], r[2]};
    for (int k = 0; k < 3; ++k) {
        red[k][i] = valid ? mu[k] : INFINITY;
        red[3 + k][i] = valid ? mu[k] : -INFINITY;
    }
    __syncthreads();
    if (i < 6) {
        float v = red[i][0];
        for (int j = 1; j < kPT; ++j) v = i < 3 ? fminf(v, red[i][j]) : fmaxf(v, red[i][j]);
        box[i] = v;
    }
    __syncthreads();
    const float o[3] = {0.5f * box[0] + 0.5f * box[3], 0.5f * box[1] + 0.5f * box[4],
                        0.5f * box[2] + 0.5f * box[5]};
    double gf[kEllF] = {}, ge[3][kEllE] = {};
    if (valid) {
        double mp[3];
        for (int k = 0; k < 3; ++k) mp[k] = (double)mu[k] - (double)o[k];  // exact
        gf[0] = mp[0];
        gf[1] = mp[1];
        gf[2] = mp[2];
        gf[3] = 1.0;
        for (int k = 0; k < 3; ++k)
            for (int p = 0; p < 3; ++p) {
                const double mkp = r[3 + 3 * k + p];  // M = diag(s) R^T, row-major
                for (int m = 0; m < 3; ++m) ge[k][3 * p + m] = mkp * mp[m];
                ge[k][9 + p] = mkp;
            }
    } else {
        // padding row: f_k = far (L_k0 + L_k1 + L_k2), nonzero for some k
        // (the row sums of L are R^T (1, 1, 1) over the semi-axes), w = 0:
        // certainly free
        gf[0] = gf[1] = gf[2] = T::far;
    }
    // per-tile power-of-two scale of the e coefficients (keeps fp16 away from
    // its subnormal range; exact, undone on the body side)
    double mx = 0.0;
    for (int k = 0; k < 3; ++k)
        for (int f = 0; f < kEllE; ++f) mx = fmax(mx, fabs(ge[k][f]));
    red[0][i] = (float)mx;
    __syncthreads();
    if (i == 0) {
        float v = 0.f;
        for (int j = 0; j < kPT; ++j) v = fmaxf(v, red[0][j]);
        s_scale = v > 0.f ? ldexp(1.0, 4 - ilogb((double)v)) : 1.0;
    }
    __syncthreads();
    const double scale = s_scale;
    float hf[kEllF], lf[kEllF], he[3][kEllE], le[3][kEllE];
    for (int f = 0; f < kEllF; ++f) {
        hf[f] = (float)(elem)(float)gf[f];
        lf[f] = (float)(elem)(float)(gf[f] - (double)hf[f]);
    }
    for (int k = 0; k < 3; ++k)
        for (int f = 0; f < kEllE; ++f) {
            const double x = ge[k][f] * scale;
            he[k][f] = (float)(elem)(float)x;
            le[k][f] = (float)(elem)(float)(x - (double)he[k][f]);
        }
    // packed operands: row block rb = i / 32, row m = i % 32; lane m + 32 h
    // holds K slots 16 j + 8 h .. + 7 of operand j
    const int rb = i >> 5, m = i & 31;
    for (int h = 0; h < 2; ++h) {
        const int lane = m + 32 * h;
        const size_t base = ((size_t)(t * kRB + rb) * kEllOps) * kLanes + lane;
        {
            vec v;
            for (int jj = 0; jj < 8; ++jj) {
                const int s = 8 * h + jj, f = eslot_feat(s, kEllF);
                v[jj] = (elem)(f < 0 ? 0.f : (eslot_glo(s, kEllF) ? lf[f] : hf[f]));
            }
            feat[base] = v;
        }
        for (int k = 0; k < 3; ++k)
            for (int j = 0; j < 3; ++j) {
                vec v;
                for (int jj = 0; jj < 8; ++jj) {
                    const int s = 16 * j + 8 * h + jj, f = eslot_feat(s, kEllE);
                    v[jj] = (elem)(f < 0 ? 0.f : (eslot_glo(s, kEllE) ? le[k][f] : he[k][f]));
                }
                feat[base + (size_t)(1 + 3 * k + j) * kLanes] = v;
            }
    }
    // tile maxima of |hi| over the real rows (Ge over the three e_k), the
    // tile's radius about the origin and its largest scale
    double rad = 0.0, smax = 0.0;
    if (valid) {
        double d2 = 0.0;
        for (int k = 0; k < 3; ++k) {
            const double dk = (double)mu[k] - (double)o[k];
            d2 += dk * dk;
            const double a = r[3 + 3 * k], b = r[4 + 3 * k], c = r[5 + 3 * k];
            smax = fmax(smax, sqrt(a * a + b * b + c * c));
        }
        rad = sqrt(d2);
    }
    __syncthreads();
    for (int f = 0; f < kEllF; ++f) red[f][i] = valid ? fabsf(hf[f]) : 0.f;
    for (int f = 0; f < kEllE; ++f)
        red[kEllF + f][i] = valid ? fmaxf(fabsf(he[0][f]), fmaxf(fabsf(he[1][f]), fabsf(he[2][f]))) : 0.f;
    __syncthreads();
    if (i < kEllF + kEllE) {
        float v = 0.f;
        for (int j = 0; j < kPT; ++j) v = fmaxf(v, red[i][j]);
        meta[t * kEllMeta + 4 + i] = v;
    }
    __syncthreads();
    red[0][i] = (float)(rad * (1.0 + 1e-6));
    red[1][i] = (float)(smax * (1.0 + 1e-6));
    __syncthreads();
    if (i < 2) {
        float v = 0.f;
        for (int j = 0; j < kPT; ++j) v = fmaxf(v, red[i][j]);
        meta[t * kEllMeta + 20 + i] = v;
    }
    if (i == 0) {
        meta[t * kEllMeta + 0] = o[0];
        meta[t * kEllMeta + 1] = o[1];
        meta[t * kEllMeta + 2] = o[2];
        meta[t * kEllMeta + 3] = (float)(1.0 / scale);
        meta[t * kEllMeta + 22] = meta[t * kEllMeta + 23] = 0.f;
    }
}

// B = L^T L of each body record (float32, a fixed order of fused products):
// xx, yy, zz, xy, xz, yz.  The MFMA form and its fp64 recheck both read it.
__global__ void ell_bmat_kernel(int q, const float *__restrict__ rec, float *__restrict__ bq)
{
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= q) return;
    const float *L = rec + (size_t)kBodyFloats * j + 3;  // row-major 3 x 3
    auto b = [&](int p, int m) { return fmaf(L[6 + p], L[6 + m], fmaf(L[3 + p], L[3 + m], L[p] * L[m])); };
    float *o = bq + (size_t)6 * j;
    o[0] = b(0, 0);
    o[1] = b(1, 1);
    o[2] = b(2, 2);
    o[3] = b(0, 1);
    o[4] = b(0, 2);
    o[5] = b(1, 2);
}

template <int P>
struct QFeatE {
    typename Prec<P>::vec f[3], e[3];
    float ef, ee;  // E_f, E_e
};

// Features of the lane's own body (centre, L, B) about tile origin mt,
// exchanged into Q[0], Q[1] as build_query does; false when a bound is not
// finite.
template <int P>
__device__ __forceinline__ bool build_query_ell(float cx, float cy, float cz, const float (&L)[9], const float (&B)[6],
                                                float two_n, const float *__restrict__ mt, QFeatE<P> (&Q)[2])
{
    using T = Prec<P>;
    using elem = typename T::elem;
    const float xp = cx - mt[0], yp = cy - mt[1], zp = cz - mt[2];
    const float ax = fabsf(xp), ay = fabsf(yp), az = fabsf(zp);
    const float *Gf = mt + 4, *Ge = mt + 4 + kEllF;
    const float ue = 3.1f * T::u * T::u + 64.f * kU32;
    // f_k: [L_k0, L_k1, L_k2, -(L c')_k]; the fp32 error of (L c')_k is within
    // 4 u32 sum_m |L_km| |c'_m| (its products and the rounding of c')
    float ef = 0.f;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const float lc = fmaf(L[3 * k + 2], zp, fmaf(L[3 * k + 1], yp, L[3 * k] * xp));
        const float la = fmaf(fabsf(L[3 * k + 2]), az, fmaf(fabsf(L[3 * k + 1]), ay, fabsf(L[3 * k]) * ax));
        const float qf[kEllF] = {L[3 * k], L[3 * k + 1], L[3 * k + 2], -lc};
        float h[kEllF], l[kEllF], s = 0.f, sabs = 0.f;
#pragma unroll
        for (int f = 0; f < kEllF; ++f) {
            h[f] = (float)(elem)qf[f];
            l[f] = (float)(elem)(qf[f] - h[f]);
            s = fmaf(fabsf(h[f]), Gf[f], s);
            sabs += fabsf(h[f]) + Gf[f];
        }
#pragma unroll
        for (int jj = 0; jj < 8; ++jj) {
            auto slot = [&](int sl) {
                const int f = eslot_feat(sl, kEllF);
                return (elem)(f < 0 ? 0.f : (eslot_qlo(sl, kEllF) ? l[f] : h[f]));
            };
            Q[0].f[k][jj] = slot(jj);
            Q[1].f[k][jj] = slot(8 + jj);
        }
        ef = fmaxf(ef, ue * s + T::eta * sabs + 4.f * kU32 * Gf[3] * la);
    }
    // e_k: 2n / scale [B_pm, -beta_p]; g B within u32 |g B|, g beta_p within
    // 5 u32 |g| sum_m |B_pm| |c'_m|
    const float bx = fmaf(B[4], zp, fmaf(B[3], yp, B[0] * xp));
    const float by = fmaf(B[5], zp, fmaf(B[1], yp, B[3] * xp));
    const float bz = fmaf(B[2], zp, fmaf(B[5], yp, B[4] * xp));
    const float Bx = fmaf(fabsf(B[4]), az, fmaf(fabsf(B[3]), ay, fabsf(B[0]) * ax));
    const float By = fmaf(fabsf(B[5]), az, fmaf(fabsf(B[1]), ay, fabsf(B[3]) * ax));
    const float Bz = fmaf(fabsf(B[2]), az, fmaf(fabsf(B[5]), ay, fabsf(B[4]) * ax));
    const float g = two_n * mt[3];
    const float qe[kEllE] = {g * B[0], g * B[3], g * B[4], g * B[3], g * B[1], g * B[5],
                             g * B[4], g * B[5], g * B[2], -g * bx, -g * by, -g * bz};
    float he[kEllE], le[kEllE], se = 0.f, se_abs = 0.f, de = 0.f;
#pragma unroll
    for (int f = 0; f < kEllE; ++f) {
        he[f] = (float)(elem)qe[f];
        le[f] = (float)(elem)(qe[f] - he[f]);
        se = fmaf(fabsf(he[f]), Ge[f], se);
        se_abs += fabsf(he[f]) + Ge[f];
        if (f < 9) de = fmaf(Ge[f], fabsf(qe[f]), de);
    }
    de = kU32 * de + fabsf(g) * (5.f * kU32) * (Ge[9] * Bx + Ge[10] * By + Ge[11] * Bz);
#pragma unroll
    for (int jj = 0; jj < 8; ++jj) {
        auto slot = [&](int sl) {
            const int f = eslot_feat(sl, kEllE);
            return (elem)(f < 0 ? 0.f : (eslot_qlo(sl, kEllE) ? le[f] : he[f]));
        };
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            Q[0].e[j][jj] = slot(16 * j + jj);
            Q[1].e[j][jj] = slot(16 * j + 8 + jj);
        }
    }
    const float Ef = 1.1f * ef;
    const float Ee = 1.1f * (ue * se + T::eta * se_abs + de);
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        swap_halves(Q[0].f[k], Q[1].f[k]);
        swap_halves(Q[0].e[k], Q[1].e[k]);
    }
    Q[0].ef = Q[1].ef = Ef;
    Q[0].ee = Q[1].ee = Ee;
    swap_halves(Q[0].ef, Q[1].ef);
    swap_halves(Q[0].ee, Q[1].ee);
    return isfinite(Ef) && isfinite(Ee) && isfinite(Ef * Ef) && isfinite(Ee * Ee);
}

// Certification kernel for ellipsoids: the layout of mfma_label_kernel (block
// = 4 waves x kEllCB 32-body column blocks; grid = query blocks x S tile splits)
// with the operands above; labels and counts.  With CULL a column block skips
// a chunk's two row blocks when each of its bodies is beyond the chunk's
// reach qk (n s_c + sqrt(n^2 s_c^2 + qa)) plus its radius (qa: the smallest
// semi-axis squared, qk: largest over smallest, as in the float32 walk).
template <int P, bool CULL>
__global__ void __launch_bounds__(256)
mfma_ell_label_kernel(const typename Prec<P>::vec *__restrict__ feat, const float *__restrict__ meta, int n_tiles,
                      int S, int n_qblocks, const float *__restrict__ cull, int n_chunks,
                      const float *__restrict__ rec, const float *__restrict__ bq, int q, float n_sigma,
                      int32_t *__restrict__ lo_out, int32_t *__restrict__ hi_out, const float *__restrict__ groups,
                      unsigned long long *__restrict__ blocks_done)
{
    using T = Prec<P>;
    using vec = typename T::vec;
    static_assert(kEllCB == 2, "one body per lane builds its features (two column blocks per wave)");
    int b = blockIdx.x;
    const int Bn = gridDim.x;
    if ((Bn & 7) == 0) b = (b & 7) * (Bn >> 3) + (b >> 3);  // XCD-major: one XCD, few splits
    const int split = b / n_qblocks;
    const int qb = b - split * n_qblocks;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, col = lane & 31, h = lane >> 5;
    float cx[kEllCB], cy[kEllCB], cz[kEllCB], qa[kEllCB], qk[kEllCB];
    int jq[kEllCB];
#pragma unroll
    for (int cb = 0; cb < kEllCB; ++cb) {
        jq[cb] = qb * kEllQueriesPerBlock + wave * (32 * kEllCB) + cb * 32 + col;
        const int jj = jq[cb] < q ? jq[cb] : q - 1;
        const float *rj = rec + (size_t)kBodyFloats * jj;
        cx[cb] = rj[0];
        cy[cb] = rj[1];
        cz[cb] = rj[2];
        qa[cb] = rj[12];
        qk[cb] = rj[13];
    }
    // the lane builds the features of body (h, col)
    const int own = jq[h] < q ? jq[h] : q - 1;
    float Lm[9], Bm[6];
#pragma unroll
    for (int k = 0; k < 9; ++k) Lm[k] = rec[(size_t)kBodyFloats * own + 3 + k];
#pragma unroll
    for (int k = 0; k < 6; ++k) Bm[k] = bq[(size_t)6 * own + k];
    const float ox = h ? cx[1] : cx[0], oy = h ? cy[1] : cy[0], oz = h ? cz[1] : cz[0];
    const float two_n = 2.f * n_sigma;
    unsigned long long n_blocks = 0;
    int lo[kEllCB] = {0, 0}, hi[kEllCB] = {0, 0};
    bool bad = false;
    const f32x16 zero = {};
    auto do_tile = [&](int t, const unsigned (&rbm_cb)[kEllCB]) {
        const float *mt = meta + (size_t)t * kEllMeta;  // wave-uniform: scalar loads
        QFeatE<P> Q[2];
        bad |= !build_query_ell<P>(ox, oy, oz, Lm, Bm, two_n, mt, Q);
        const vec *ft = feat + (size_t)t * kRB * kEllOps * kLanes + lane;
        unsigned rbm = rbm_cb[0] | rbm_cb[1];
        while (rbm) {
            const int rb = __builtin_ctz(rbm);
            rbm &= rbm - 1;
            const vec *fp = ft + (size_t)rb * kEllOps * kLanes;
            vec G[kEllOps];
#pragma unroll
            for (int k = 0; k < kEllOps; ++k) G[k] = fp[(size_t)k * kLanes];
#pragma unroll
            for (int cb = 0; cb < kEllCB; ++cb) {
                if (!((rbm_cb[cb] >> rb) & 1u)) continue;  // no body of cb near the row block
                ++n_blocks;
                // a~ = sum f~_k^2 - 1 and its bound E_a per pair
                f32x16 A2, Fa;
#pragma unroll
                for (int k = 0; k < 3; ++k) {
                    const f32x16 Fk = T::mfma(G[0], Q[cb].f[k], zero);
#pragma unroll
                    for (int i = 0; i < 16; ++i) {
                        A2[i] = k == 0 ? Fk[i] * Fk[i] : fmaf(Fk[i], Fk[i], A2[i]);
                        Fa[i] = k == 0 ? fabsf(Fk[i]) : Fa[i] + fabsf(Fk[i]);
                    }
                }
                const float ef = Q[cb].ef, ee = Q[cb].ee;
                const float ca = fmaf(3.f * ef, ef, 2.f * kU32);
#pragma unroll
                for (int i = 0; i < 16; ++i) {
                    const float a = A2[i] - 1.f;
                    A2[i] = a;
                    Fa[i] = fmaf(2.f * ef, Fa[i], fmaf(fabsf(a), 2.f * kU32, ca));  // E_a
                }
                // w~ = sum e~_k^2 and S = sum |e~_k|
                f32x16 W, Se;
#pragma unroll
                for (int k = 0; k < 3; ++k) {
                    f32x16 E = T::mfma(G[1 + 3 * k], Q[cb].e[0], zero);
                    E = T::mfma(G[2 + 3 * k], Q[cb].e[1], E);
                    E = T::mfma(G[3 + 3 * k], Q[cb].e[2], E);
#pragma unroll
                    for (int i = 0; i < 16; ++i) {
                        W[i] = k == 0 ? E[i] * E[i] : fmaf(E[i], E[i], W[i]);
                        Se[i] = k == 0 ? fabsf(E[i]) : Se[i] + fabsf(E[i]);
                    }
                }
                const float ce = 3.f * ee * ee;
                // w - a|a| (> 0 iff collision) against its certified bound
                auto fb = [&](int i, float &f, float &bnd) {
                    const float a = A2[i], aa = fabsf(a), Ea = Fa[i];
                    const float Ew = fmaf(W[i], 6.f * kU32, fmaf(2.f * ee, Se[i], ce));
                    f = fmaf(-a, aa, W[i]);
                    bnd = fmaf(aa, fmaf(aa, 2.f * kU32, 2.f * Ea), fmaf(Ea, Ea, Ew)) * 1.0001f;
                };
                bool poss = false;
#pragma unroll
                for (int i = 0; i < 16; ++i) {
                    float f, bnd;
                    fb(i, f, bnd);
                    poss |= f > -bnd;
                }
                if (__any(poss)) {
#pragma unroll
                    for (int i = 0; i < 16; ++i) {
                        float f, bnd;
                        fb(i, f, bnd);
                        lo[cb] += f > bnd;   // certainly in collision
                        hi[cb] += f > -bnd;  // possibly in collision
                    }
                }
            }
        }
    };
    if constexpr (!CULL) {
        const unsigned all[kEllCB] = {0xffffu, 0xffffu};
        for (int t = split; t < n_tiles; t += S) do_tile(t, all);
    } else {
        float wx, wy, wz, spread, qamax, half[3];
        pair::wave_sphere<kEllCB>(cx, cy, cz, qa, wx, wy, wz, spread, qamax, half);
        float qkmax = fmaxf(qk[0], qk[1]);
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) qkmax = fmaxf(qkmax, __shfl_xor(qkmax, off));
        qkmax = pair::wave_uniform(qkmax);
        auto reach_of = [&](const pair::ChunkMeta &m, float a2, float kk) {
            const float ns = n_sigma * m.smax;
            return kk * (ns + pair::fast_sqrt(fmaf(ns, ns, a2)));  // ~1 ulp, far inside the culling margin
        };
        auto coarse = [&](const pair::ChunkMeta &m) {
            const float reach = m.rad + reach_of(m, qamax, qkmax);
            return pair::within(m, wx, wy, wz, spread + reach) && pair::within_box(m, wx, wy, wz, half, reach);
        };
        // groups dealt to the splits over a large scene, tiles otherwise, as
        // in mfma_label_kernel
        const int n_groups = (n_chunks + pair::kGroup - 1) / pair::kGroup;
        const bool by_group = n_chunks > pair::kGroupDealChunks * S;
        const int n_units = by_group ? n_groups : n_tiles;
        const int per_batch = by_group ? 64 : 64 / kChunksPerTile;
        for (int ib = 0; split + ib * S < n_units; ib += per_batch) {
            pair::ChunkMeta bm{0.f, 0.f, 0.f, 0.f, 0.f};
            bool bpass = false;
            if (by_group) {
                const int gl = split + (ib + lane) * S;
                if (gl < n_groups) {
                    bm = pair::load_chunk(groups, gl);
                    bpass = coarse(bm);
                }
            } else {
                const int t = split + (ib + lane / kChunksPerTile) * S;
                const int ci = t * kChunksPerTile + lane % kChunksPerTile;
                if (t < n_tiles && ci < n_chunks) {
                    bm = pair::load_chunk(cull, ci);
                    bpass = coarse(bm);
                }
            }
            const unsigned long long bmask = __ballot(bpass);
            unsigned long long gmask = by_group ? bmask : 1ull;
            while (gmask) {
                pair::ChunkMeta m = bm;
                unsigned long long mask = bmask;
                int gi = 0;
                if (by_group) {
                    gi = split + (ib + __builtin_ctzll(gmask)) * S;
                    const int ci = gi * pair::kGroup + lane;
                    bool pass = false;
                    m = pair::ChunkMeta{0.f, 0.f, 0.f, 0.f, 0.f};
                    if (lane < pair::kGroup && ci < n_chunks) {
                        m = pair::load_chunk(cull, ci);
                        pass = coarse(m);
                    }
                    mask = __ballot(pass);
                }
                gmask &= gmask - 1;
                while (mask) {
                    const int g = __builtin_ctzll(mask) / kChunksPerTile;
                    unsigned tm = (unsigned)(mask >> (kChunksPerTile * g)) & ((1u << kChunksPerTile) - 1u);
                    mask &= ~((((unsigned long long)1 << kChunksPerTile) - 1ull) << (kChunksPerTile * g));
                    const int t = by_group ? gi * (pair::kGroup / kChunksPerTile) + g : split + (ib + g) * S;
                    unsigned rbm[kEllCB] = {0u, 0u};
                    while (tm) {
                        const int k = __builtin_ctz(tm);
                        tm &= tm - 1;
                        const pair::ChunkMeta c = pair::lane_chunk(m, kChunksPerTile * g + k);
#pragma unroll
                        for (int cb = 0; cb < kEllCB; ++cb)
                            if (__any(pair::within(c, cx[cb], cy[cb], cz[cb], c.rad + reach_of(c, qa[cb], qk[cb]))))
                                rbm[cb] |= 3u << (2 * k);
                    }
                    if (rbm[0] | rbm[1]) do_tile(t, rbm);
                }
            }
        }
    }
#pragma unroll
    for (int cb = 0; cb < kEllCB; ++cb) {
        lo[cb] += __shfl_xor(lo[cb], 32);
        hi[cb] += __shfl_xor(hi[cb], 32);
        // body cb was built by the lanes of half cb
        const bool other = __shfl_xor((int)bad, 32) != 0;
        const bool anybad = (h == cb) ? bad : other;
        if (h == 0 && jq[cb] < q) {
            lo_out[(size_t)split * q + jq[cb]] = lo[cb];
            hi_out[(size_t)split * q + jq[cb]] = anybad ? (1 << 29) : hi[cb];
        }
    }
    if (blocks_done && lane == 0) atomicAdd(blocks_done, n_blocks);
}

// fp64 recheck of the listed bodies: recheck_fp64_kernel's walk with the
// ellipsoid test (s^2 = |L d|^2, sigma^2 / 4 = |M B d|^2, L and B as the MFMA
// form took them) and the ellipsoid reach.
__global__ void __launch_bounds__(64 * kRecheckWaves)
recheck_ell_fp64_kernel(const float *__restrict__ gauss, int n, const float *__restrict__ cull,
                        const float *__restrict__ rec, const float *__restrict__ bq, float n_sigma,
                        const int32_t *__restrict__ list, const int32_t *__restrict__ n_list,
                        int32_t *__restrict__ exact)
{
    const int nl = *n_list;
    const int tiles = (nl + 63) / 64;
    const long items = (long)tiles * kRecheckSplits;
    const int n_chunks = (n + pair::kCull - 1) / pair::kCull;
    const int lane = (int)(threadIdx.x & 63u);
    const double four_n2 = 4.0 * (double)n_sigma * (double)n_sigma;
    const long wave0 = (long)blockIdx.x * kRecheckWaves + (long)(threadIdx.x >> 6);
    const long waves = (long)gridDim.x * kRecheckWaves;
    for (long item = wave0; item < items; item += waves) {
        const int tile = (int)(item / kRecheckSplits), split = (int)(item - (long)tile * kRecheckSplits);
        const int li = tile * 64 + lane;
        const bool valid = li < nl;
        const int j = list[valid ? li : nl - 1];
        const float *rj = rec + (size_t)kBodyFloats * j;
        float fc[3][1] = {{rj[0]}, {rj[1]}, {rj[2]}};
        float fa[1] = {rj[12]};
        const float fk = rj[13];
        float Bm[6], Lm[9];
        for (int k = 0; k < 6; ++k) Bm[k] = bq[(size_t)6 * j + k];
        for (int k = 0; k < 9; ++k) Lm[k] = rj[3 + k];
        int cnt = 0;
        auto chunk = [&](int ci, unsigned long long qmask) {
            const int g = ci * pair::kCull + lane;
            const bool real = g < n;
            const float *p = gauss + (size_t)kGaussFloats * (real ? g : n - 1);
            double mu[3], M[9];
            for (int k = 0; k < 3; ++k) mu[k] = p[k];
            for (int k = 0; k < 9; ++k) M[k] = p[3 + k];
            while (qmask) {
                const int b = __builtin_ctzll(qmask);
                qmask &= qmask - 1;
                const double cx = pair::lane_value(fc[0][0], b), cy = pair::lane_value(fc[1][0], b),
                             cz = pair::lane_value(fc[2][0], b);
                double B[6], L[9];
                for (int k = 0; k < 6; ++k) B[k] = pair::lane_value(Bm[k], b);
                for (int k = 0; k < 9; ++k) L[k] = pair::lane_value(Lm[k], b);
                const double dx = mu[0] - cx, dy = mu[1] - cy, dz = mu[2] - cz;
                const double f0 = L[0] * dx + L[1] * dy + L[2] * dz;
                const double f1 = L[3] * dx + L[4] * dy + L[5] * dz;
                const double f2 = L[6] * dx + L[7] * dy + L[8] * dz;
                const double a = f0 * f0 + f1 * f1 + f2 * f2 - 1.0;
                const double ux = B[0] * dx + B[3] * dy + B[4] * dz;
                const double uy = B[3] * dx + B[1] * dy + B[5] * dz;
                const double uz = B[4] * dx + B[5] * dy + B[2] * dz;
                const double e0 = M[0] * ux + M[1] * uy + M[2] * uz;
                const double e1 = M[3] * ux + M[4] * uy + M[5] * uz;
                const double e2 = M[6] * ux + M[7] * uy + M[8] * uz;
                const bool hit = real && a * fabs(a) < four_n2 * (e0 * e0 + e1 * e1 + e2 * e2);
                const int hcount = __popcll(__ballot(hit));
                if (lane == b) cnt += hcount;
            }
        };
        const unsigned long long vmask = __ballot(valid);
        if (cull) {
            float wx, wy, wz, spread, amax;
            pair::wave_sphere<1>(fc[0], fc[1], fc[2], fa, wx, wy, wz, spread, amax);
            float kmax = fk;
            for (int off = 32; off >= 1; off >>= 1) kmax = fmaxf(kmax, __shfl_xor(kmax, off));
            kmax = pair::wave_uniform(kmax);
            auto reach_of = [&](const pair::ChunkMeta &m, float a2, float kk) {
                const float ns = n_sigma * m.smax;
                return kk * (ns + pair::fast_sqrt(fmaf(ns, ns, a2)));
            };
            for (int ib = 0; split + ib * kRecheckSplits < n_chunks; ib += 64) {
                const int ci = split + (ib + lane) * kRecheckSplits;
                pair::ChunkMeta m{0.f, 0.f, 0.f, 0.f, 0.f};
                bool pass = false;
                if (ci < n_chunks) {
                    m = pair::load_chunk(cull, ci);
                    pass = pair::within(m, wx, wy, wz, spread + m.rad + reach_of(m, amax, kmax));
                }
                unsigned long long mask = __ballot(pass);
                while (mask) {
                    const int bit = __builtin_ctzll(mask);
                    mask &= mask - 1;
                    const pair::ChunkMeta k = pair::lane_chunk(m, bit);
                    const bool near = pair::within(k, fc[0][0], fc[1][0], fc[2][0], k.rad + reach_of(k, fa[0], fk));
                    const unsigned long long qmask = __ballot(near) & vmask;
                    if (qmask) chunk(split + (ib + bit) * kRecheckSplits, qmask);
                }
            }
        } else {
            for (int ci = split; ci < n_chunks; ci += kRecheckSplits) chunk(ci, vmask);
        }
        if (valid && cnt) atomicAdd(exact + li, cnt);
    }
}

template <int P>
csplat_status build_one(csplat_ctx *ctx, csplat_scene *sc, void **feat_out)
{
    using vec = typename Prec<P>::vec;
    const int64_t nt = (sc->n + kPT - 1) / kPT;
    // the per-tile scale and coefficient maxima are dtype specific: each dtype
    // owns its metadata
    float *meta = nullptr;
    // stream-ordered, like the scene's other buffers (freed with them)
    CSPLAT_HIP(hipMallocAsync(&meta, (size_t)nt * kMeta * sizeof(float), ctx->stream));
    vec *feat = nullptr;
    const size_t fbytes = (size_t)nt * kRB * kOps * kLanes * sizeof(vec);
    hipError_t e = hipMallocAsync(&feat, fbytes, ctx->stream);
    if (e != hipSuccess) {
        (void)hipFreeAsync(meta, ctx->stream);
        return hip_fail(e, "precision features");
    }
    build_tiles_kernel<P><<<(unsigned)nt, kPT, 0, ctx->stream>>>(sc->gauss, sc->n, meta, feat);
    hipError_t le = hipGetLastError();
    if (le == hipSuccess) le = hipStreamSynchronize(ctx->stream);
    if (le != hipSuccess) {
        (void)hipFreeAsync(meta, ctx->stream);
        (void)hipFreeAsync(feat, ctx->stream);
        return hip_fail(le, "build_tiles_kernel");
    }
    feat_out[0] = feat;
    feat_out[1] = meta;
    sc->device_bytes += fbytes + (uint64_t)nt * kMeta * sizeof(float);
    return CSPLAT_OK;
}

}  // namespace

namespace {
template <int P>
csplat_status build_ell_one(csplat_ctx *ctx, csplat_scene *sc, void **feat_out);
}  // namespace

csplat_status precision_build(csplat_ctx *ctx, csplat_scene *sc, uint32_t features)
{
    sc->n_tiles = (sc->n + kPT - 1) / kPT;
    if (features & CSPLAT_FEATURES_BF16) {
        void *out[2];
        csplat_status s = build_one<CSPLAT_PRECISION_BF16_RECHECK>(ctx, sc, out);
        if (s != CSPLAT_OK) return s;
        sc->feat_bf16 = out[0];
        sc->meta_bf16 = static_cast<float *>(out[1]);
    }
    if (features & CSPLAT_FEATURES_FP16) {
        void *out[2];
        csplat_status s = build_one<CSPLAT_PRECISION_FP16_RECHECK>(ctx, sc, out);
        if (s != CSPLAT_OK) return s;
        sc->feat_fp16 = out[0];
        sc->meta_fp16 = static_cast<float *>(out[1]);
    }
    if (features & CSPLAT_FEATURES_ELL_BF16) {
        void *out[2];
        csplat_status s = build_ell_one<CSPLAT_PRECISION_BF16_RECHECK>(ctx, sc, out);
        if (s != CSPLAT_OK) return s;
        sc->feat_ell_bf16 = out[0];
        sc->meta_ell_bf16 = static_cast<float *>(out[1]);
    }
    if (features & CSPLAT_FEATURES_ELL_FP16) {
        void *out[2];
        csplat_status s = build_ell_one<CSPLAT_PRECISION_FP16_RECHECK>(ctx, sc, out);
        if (s != CSPLAT_OK) return s;
        sc->feat_ell_fp16 = out[0];
        sc->meta_ell_fp16 = static_cast<float *>(out[1]);
    }
    return CSPLAT_OK;
}

namespace {
struct IsOne {
    __host__ __device__ uint8_t operator()(uint8_t x) const { return x == 1; }
};
struct IsTwo {
    __host__ __device__ uint8_t operator()(uint8_t x) const { return x == 2; }
};

// One launch of mfma_label_kernel for dtype `precision`.
template <bool COUNT, bool MINW>
void launch_mfma(int precision, bool cull, dim3 grid, hipStream_t st, const csplat_scene *sc, int n_qblocks, int S,
                 int n_chunks, const float *c, const float *r, int q, float four_n2, float nv, int32_t *lo,
                 int32_t *hi, const float *thr, float *mlo, float *mup, unsigned long long *blocks)
{
    const int n_tiles = (int)sc->n_tiles;
    // the group level of the culling metadata: after the chunks and the sub-chunks
    const int64_t n_fine = (sc->n + pair::kFine - 1) / pair::kFine;
    const float *groups = sc->cull ? sc->cull + ((size_t)n_chunks + (size_t)n_fine) * pair::kCullFloats : nullptr;
    if (precision == CSPLAT_PRECISION_BF16_RECHECK) {
        const auto *f = static_cast<const bf16x8 *>(sc->feat_bf16);
        if (cull)
            mfma_label_kernel<CSPLAT_PRECISION_BF16_RECHECK, true, COUNT, MINW><<<grid, 256, 0, st>>>(
                f, sc->meta_bf16, n_tiles, S, n_qblocks, sc->cull, n_chunks, c, r, q, four_n2, nv, lo, hi, groups, thr,
                mlo, mup, blocks);
        else
            mfma_label_kernel<CSPLAT_PRECISION_BF16_RECHECK, false, COUNT, MINW><<<grid, 256, 0, st>>>(
                f, sc->meta_bf16, n_tiles, S, n_qblocks, sc->cull, n_chunks, c, r, q, four_n2, nv, lo, hi, groups, thr,
                mlo, mup, blocks);
    } else {
        const auto *f = static_cast<const f16x8 *>(sc->feat_fp16);
        if (cull)
            mfma_label_kernel<CSPLAT_PRECISION_FP16_RECHECK, true, COUNT, MINW><<<grid, 256, 0, st>>>(
                f, sc->meta_fp16, n_tiles, S, n_qblocks, sc->cull, n_chunks, c, r, q, four_n2, nv, lo, hi, groups, thr,
                mlo, mup, blocks);
        else
            mfma_label_kernel<CSPLAT_PRECISION_FP16_RECHECK, false, COUNT, MINW><<<grid, 256, 0, st>>>(
                f, sc->meta_fp16, n_tiles, S, n_qblocks, sc->cull, n_chunks, c, r, q, four_n2, nv, lo, hi, groups, thr,
                mlo, mup, blocks);
    }
}

__global__ void fill_u64_kernel(unsigned long long *p, int n, unsigned long long v)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

// Splits of a launch over q queries (blocks of `per_block`): enough work
// items to fill the device, each over at least kMinSplitTiles tiles when the
// scene has that many (a work item's fixed cost, its query features and the
// walk's first metadata loads, is otherwise repeated for a tile or two: a
// 4,096-sphere batch on a 200k-Gaussian scene took 0.67 ms in bf16 with one
// tile per split, 0.36 with 16, and a 32,768-sphere one 2.01 and 1.37 ms).
constexpr int kMinSplitTiles = 16;
int mfma_splits(const csplat_ctx *ctx, int q, int n_tiles, int per_block = kQueriesPerBlock)
{
    const int n_qblocks = (q + per_block - 1) / per_block;
    if (n_tiles <= 0) return 1;
    const int S = (ctx_target_blocks(ctx) + n_qblocks - 1) / n_qblocks;
    return std::max(1, std::min(S, n_tiles / kMinSplitTiles));
}
}  // namespace

csplat_status precision_eval(csplat_ctx *ctx, const csplat_scene *sc, int64_t q64, const float *centers,
                             const float *radii, const EvalParams &p, const EvalOut &out, int precision,
                             const std::function<csplat_status()> &gate)
{
    const int q = (int)q64;
    const int n = (int)sc->n;
    const int m = p.m;
    hipStream_t st = ctx->stream;
    const int n_tiles = (int)sc->n_tiles;
    const int n_qblocks = (q + kQueriesPerBlock - 1) / kQueriesPerBlock;
    const int S = mfma_splits(ctx, q, n_tiles);
    const int n_chunks = (n + pair::kCull - 1) / pair::kCull;
    const bool cull = p.cull && n > 0 && sc->cull;
    const bool want_count = out.label || out.count;
    const bool want_min = out.min || out.err;
    const float *c = centers, *r = radii;
    const int32_t *perm = nullptr;
    unsigned long long *blocks = nullptr;
    if (cull) {
        SortedQueries sq;
        csplat_status s = sort_queries(ctx, sc, q, centers, radii, &sq);
        if (s != CSPLAT_OK) return s;
        c = sq.c;
        r = sq.r;
        perm = sq.perm;
        blocks = sq.counter;  // 32 x 32 MFMA blocks evaluated (every pass, every n_sigma)
        ctx->chunk_counter = sq.counter;
        ctx->pairs_per_chunk = 32 * 32;
    }
    // workspace: lo/hi partials, the recheck list, exact counts, flags, compaction scratch
    size_t sel_bytes = 0;
    CSPLAT_HIP(hipcub::DeviceSelect::Flagged(nullptr, sel_bytes, hipcub::CountingInputIterator<int32_t>(0),
                                             (const uint8_t *)nullptr, (int32_t *)nullptr, (int32_t *)nullptr, q,
                                             st));
    const size_t part = (size_t)S * q;
    const size_t off_list = 2 * part * 4, off_exact = off_list + (size_t)q * 4, off_flag = off_exact + (size_t)q * 4,
                 off_sel = (off_flag + (size_t)q + 255) & ~(size_t)255;
    hipError_t e = ctx->partial.reserve(off_sel + sel_bytes + 256);
    if (e != hipSuccess) return hip_fail(e, "precision workspace");
    char *base = ctx->partial.as<char>();
    int32_t *lo = reinterpret_cast<int32_t *>(base);
    int32_t *hi = lo + part;
    int32_t *list = reinterpret_cast<int32_t *>(base + off_list);
    int32_t *exact = reinterpret_cast<int32_t *>(base + off_exact);
    uint8_t *flag = reinterpret_cast<uint8_t *>(base + off_flag);
    void *sel_tmp = base + off_sel;
    // the minimum search's state and partials
    auto al = [](size_t b) { return (b + 255) & ~(size_t)255; };
    const size_t qn = (size_t)q, mpart = (size_t)ctx_target_blocks(ctx) * kQueriesPerBlock + part;
    const size_t o_lo = 0, o_up = o_lo + al(qn * 4), o_thr = o_up + al(qn * 4), o_mflag = o_thr + al(qn * 4),
                 o_mlist = o_mflag + al(qn), o_nl = o_mlist + al(qn * 4), o_cc = o_nl + 256, o_rr = o_cc + al(qn * 12),
                 o_tt = o_rr + al(qn * 4), o_slot = o_tt + al(qn * 4), o_best = o_slot + al(qn * 4),
                 o_mlo = o_best + al(qn * 8), o_mup = o_mlo + al(2 * mpart * 4), o_msel = o_mup + al(mpart * 4),
                 o_mv = o_msel + al(sel_bytes), m_total = o_mv + al(qn * 4);
    char *mb = nullptr;
    if (want_min) {
        e = ctx->minbuf.reserve(m_total);
        if (e != hipSuccess) return hip_fail(e, "minimum-search workspace");
        mb = ctx->minbuf.as<char>();
    }
    float *st_lo = reinterpret_cast<float *>(mb + o_lo), *st_up = reinterpret_cast<float *>(mb + o_up),
          *st_thr = reinterpret_cast<float *>(mb + o_thr), *st_mv = reinterpret_cast<float *>(mb + o_mv);
    uint8_t *mflag = reinterpret_cast<uint8_t *>(mb + o_mflag);
    int32_t *mlist = reinterpret_cast<int32_t *>(mb + o_mlist), *mnl = reinterpret_cast<int32_t *>(mb + o_nl),
            *slot = reinterpret_cast<int32_t *>(mb + o_slot);
    float *cc = reinterpret_cast<float *>(mb + o_cc), *rr = reinterpret_cast<float *>(mb + o_rr),
          *tt = reinterpret_cast<float *>(mb + o_tt), *mlo = reinterpret_cast<float *>(mb + o_mlo),
          *mup = reinterpret_cast<float *>(mb + o_mup);
    auto *best = reinterpret_cast<unsigned long long *>(mb + o_best);
    void *msel = mb + o_msel;
    e = ctx->flags.reserve((size_t)CSPLAT_MAX_M * sizeof(int32_t) + 64);
    if (e != hipSuccess) return hip_fail(e, "flag counters");
    int32_t *n_list = ctx->flags.as<int32_t>();
    CSPLAT_HIP(zero_words(n_list, CSPLAT_MAX_M, st));
    ctx->stats.splits = S;
    ctx->stats.queries_per_lane = 2;
    ctx->stats.kernel_pairs = (int64_t)q * n;
    ctx->flag_counts = want_count ? n_list : nullptr;
    ctx->flag_m = want_count ? m : 0;
    const unsigned qb = (unsigned)((q + 255) / 256);
    float total_ms = 0.f;
    int passes = 0;
    auto time_pass = [&](bool begin) {
        if (!ctx->timing) return;
        (void)hipEventRecord(begin ? ctx->ev0 : ctx->ev1, st);
    };
    auto add_ms = [&]() {
        if (!ctx->timing) return CSPLAT_OK;
        float ms = 0.f;
        CSPLAT_HIP(hipEventSynchronize(ctx->ev1));
        CSPLAT_HIP(hipEventElapsedTime(&ms, ctx->ev0, ctx->ev1));
        total_ms += ms;
        return CSPLAT_OK;
    };
    bool gated = false;
    for (int v = 0; v < m; ++v) {
        const float nv = p.n_sigma[v];
        // pass 1: labels (certified counts) and the minimum's interval
        if (n_tiles > 0) {
            const dim3 grid((unsigned)(n_qblocks * S));
            time_pass(true);
            if (want_count && want_min)
                launch_mfma<true, true>(precision, cull, grid, st, sc, n_qblocks, S, n_chunks, c, r, q, p.four_n2[v],
                                        nv, lo, hi, nullptr, mlo, mup, blocks);
            else if (want_count)
                launch_mfma<true, false>(precision, cull, grid, st, sc, n_qblocks, S, n_chunks, c, r, q,
                                         p.four_n2[v], nv, lo, hi, nullptr, nullptr, nullptr, blocks);
            else
                launch_mfma<false, true>(precision, cull, grid, st, sc, n_qblocks, S, n_chunks, c, r, q,
                                         p.four_n2[v], nv, nullptr, nullptr, nullptr, mlo, mup, blocks);
            time_pass(false);
            CSPLAT_HIP(hipGetLastError());
            csplat_status ts = add_ms();
            if (ts != CSPLAT_OK) return ts;
        }
        if (gate && !gated) {
            // nothing that writes an output is queued before the caller's
            // check of its inputs has passed (the sort and the first MFMA
            // pass write only the workspace and overlap the check)
            gated = true;
            csplat_status gs = gate();
            if (gs != CSPLAT_OK) return gs;
        }
        if (want_count) {
            decide_kernel<<<qb, 256, 0, st>>>(q, n_tiles > 0 ? S : 0, m, v, p.k, out.count != nullptr, lo, hi, perm,
                                              out.label, out.count, flag);
            CSPLAT_HIP(hipGetLastError());
            // the undecided queries, in (sorted) query order
            CSPLAT_HIP(hipcub::DeviceSelect::Flagged(sel_tmp, sel_bytes, hipcub::CountingInputIterator<int32_t>(0),
                                                     flag, list, n_list + v, q, st));
            CSPLAT_HIP(zero_words(exact, (size_t)q, st));
            if (n > 0)
                recheck_fp64_kernel<<<kRecheckGrid, 64 * kRecheckWaves, 0, st>>>(
                    sc->gauss, n, cull ? sc->cull : nullptr, c, r, p.n_sigma[v], list, n_list + v, exact);
            finish_kernel<<<qb, 256, 0, st>>>(m, v, p.k, list, n_list + v, exact, perm, out.label, out.count);
            CSPLAT_HIP(hipGetLastError());
            ctx->rk_list = list;
            ctx->rk_n = n_list + v;
            ctx->rk_perm = perm;
            ctx->rk_q = q;
        }
        if (!want_min) continue;
        // the minimum: later passes for the queries not yet resolved
        pmin_combine_kernel<<<(unsigned)((q + 3) / 4), 256, 0, st>>>(q, n_tiles > 0 ? S : 0, nullptr, r, mlo, mup,
                                                                     st_lo, st_up, st_mv, st_thr, mflag, true);
        CSPLAT_HIP(hipGetLastError());
        int pass = 1;
        for (; n > 0; ++pass) {
            CSPLAT_HIP(hipcub::DeviceSelect::Flagged(msel, sel_bytes, hipcub::CountingInputIterator<int32_t>(0),
                                                     hipcub::TransformInputIterator<uint8_t, IsOne, const uint8_t *>(mflag, IsOne()),
                                                     mlist, mnl, q, st));
            int nl = 0;
            CSPLAT_HIP(hipMemcpyAsync(&nl, mnl, sizeof(int), hipMemcpyDeviceToHost, st));
            CSPLAT_HIP(hipStreamSynchronize(st));
            if (nl == 0) break;
            if (pass >= 64) return fail(CSPLAT_E_DEVICE, "minimum search: thresholds did not converge");
            const unsigned lb = (unsigned)((nl + 255) / 256);
            pmin_gather_kernel<<<lb, 256, 0, st>>>(nl, mlist, c, r, st_up, st_thr, cc, rr, tt);
            const int nqb = (nl + kQueriesPerBlock - 1) / kQueriesPerBlock;
            const int S2 = mfma_splits(ctx, nl, n_tiles);
            time_pass(true);
            launch_mfma<false, true>(precision, cull, dim3((unsigned)(nqb * S2)), st, sc, nqb, S2, n_chunks, cc, rr,
                                     nl, p.four_n2[v], nv, nullptr, nullptr, tt, mlo, mup, blocks);
            time_pass(false);
            CSPLAT_HIP(hipGetLastError());
            csplat_status ts = add_ms();
            if (ts != CSPLAT_OK) return ts;
            pmin_combine_kernel<<<(unsigned)((nl + 3) / 4), 256, 0, st>>>(nl, S2, mlist, r, mlo, mup, st_lo, st_up,
                                                                          st_mv, st_thr, mflag, false);
            CSPLAT_HIP(hipGetLastError());
        }
        passes = std::max(passes, pass);
        // queries whose low-precision bound was not finite: fp64 over every kept Gaussian
        CSPLAT_HIP(hipcub::DeviceSelect::Flagged(msel, sel_bytes, hipcub::CountingInputIterator<int32_t>(0),
                                                 hipcub::TransformInputIterator<uint8_t, IsTwo, const uint8_t *>(mflag, IsTwo()),
                                                 mlist, mnl, q, st));
        fill_u64_kernel<<<qb, 256, 0, st>>>(best, q, 0x7FF0000000000000ull);
        pmin_slot_kernel<<<qb, 256, 0, st>>>(mlist, mnl, slot);
        if (n > 0)
            min_fp64_kernel<<<kRecheckGrid, 64 * kRecheckWaves, 0, st>>>(sc->gauss, n, c, nv, mlist, mnl, best);
        pmin_output_kernel<<<qb, 256, 0, st>>>(q, m, v, r, perm, st_lo, st_up, st_mv, mflag, slot, best, out.min,
                                               out.err);
        CSPLAT_HIP(hipGetLastError());
    }
    ctx->stats.min_passes = want_min ? passes : 0;
    if (ctx->timing) {
        ctx->timed = true;
        ctx->timed_ms = total_ms;
    }
    return CSPLAT_OK;
}

namespace {
template <int P>
csplat_status build_ell_one(csplat_ctx *ctx, csplat_scene *sc, void **feat_out)
{
    using vec = typename Prec<P>::vec;
    const int64_t nt = (sc->n + kPT - 1) / kPT;
    float *meta = nullptr;
    CSPLAT_HIP(hipMallocAsync(&meta, (size_t)nt * kEllMeta * sizeof(float), ctx->stream));
    vec *feat = nullptr;
    const size_t fbytes = (size_t)nt * kRB * kEllOps * kLanes * sizeof(vec);
    hipError_t e = hipMallocAsync(&feat, fbytes, ctx->stream);
    if (e != hipSuccess) {
        (void)hipFreeAsync(meta, ctx->stream);
        return hip_fail(e, "ellipsoid precision features");
    }
    build_tiles_ell_kernel<P><<<(unsigned)nt, kPT, 0, ctx->stream>>>(sc->gauss, sc->n, meta, feat);
    hipError_t le = hipGetLastError();
    if (le == hipSuccess) le = hipStreamSynchronize(ctx->stream);
    if (le != hipSuccess) {
        (void)hipFreeAsync(meta, ctx->stream);
        (void)hipFreeAsync(feat, ctx->stream);
        return hip_fail(le, "build_tiles_ell_kernel");
    }
    feat_out[0] = feat;
    feat_out[1] = meta;
    sc->device_bytes += fbytes + (uint64_t)nt * kEllMeta * sizeof(float);
    return CSPLAT_OK;
}

void launch_mfma_ell(int precision, bool cull, dim3 grid, hipStream_t st, const csplat_scene *sc, int n_qblocks,
                     int S, int n_chunks, const float *rec, const float *bq, int q, float nv, int32_t *lo, int32_t *hi,
                     unsigned long long *blocks)
{
    const int n_tiles = (int)sc->n_tiles;
    const int64_t n_fine = (sc->n + pair::kFine - 1) / pair::kFine;
    const float *groups = sc->cull ? sc->cull + ((size_t)n_chunks + (size_t)n_fine) * pair::kCullFloats : nullptr;
    if (precision == CSPLAT_PRECISION_BF16_RECHECK) {
        const auto *f = static_cast<const bf16x8 *>(sc->feat_ell_bf16);
        if (cull)
            mfma_ell_label_kernel<CSPLAT_PRECISION_BF16_RECHECK, true><<<grid, 256, 0, st>>>(
                f, sc->meta_ell_bf16, n_tiles, S, n_qblocks, sc->cull, n_chunks, rec, bq, q, nv, lo, hi, groups, blocks);
        else
            mfma_ell_label_kernel<CSPLAT_PRECISION_BF16_RECHECK, false><<<grid, 256, 0, st>>>(
                f, sc->meta_ell_bf16, n_tiles, S, n_qblocks, sc->cull, n_chunks, rec, bq, q, nv, lo, hi, groups, blocks);
    } else {
        const auto *f = static_cast<const f16x8 *>(sc->feat_ell_fp16);
        if (cull)
            mfma_ell_label_kernel<CSPLAT_PRECISION_FP16_RECHECK, true><<<grid, 256, 0, st>>>(
                f, sc->meta_ell_fp16, n_tiles, S, n_qblocks, sc->cull, n_chunks, rec, bq, q, nv, lo, hi, groups, blocks);
        else
            mfma_ell_label_kernel<CSPLAT_PRECISION_FP16_RECHECK, false><<<grid, 256, 0, st>>>(
                f, sc->meta_ell_fp16, n_tiles, S, n_qblocks, sc->cull, n_chunks, rec, bq, q, nv, lo, hi, groups, blocks);
    }
}
}  // namespace

csplat_status precision_eval_ell(csplat_ctx *ctx, const csplat_scene *sc, int64_t q64, const float *rec_in,
                                 const EvalParams &p, const EvalOut &out, int precision)
{
    const int q = (int)q64;
    const int n = (int)sc->n;
    const int m = p.m;
    hipStream_t st = ctx->stream;
    const int n_tiles = (int)sc->n_tiles;
    const int n_qblocks = (q + kEllQueriesPerBlock - 1) / kEllQueriesPerBlock;
    const int S = mfma_splits(ctx, q, n_tiles, kEllQueriesPerBlock);
    const int n_chunks = (n + pair::kCull - 1) / pair::kCull;
    const bool cull = p.cull && n > 0 && sc->cull;
    const float *rec = rec_in;
    const int32_t *perm = nullptr;
    unsigned long long *blocks = nullptr;
    if (cull) {
        SortedQueries sq;
        csplat_status s = sort_bodies(ctx, sc, q, rec_in, nullptr, true, &sq);
        if (s != CSPLAT_OK) return s;
        rec = sq.c;
        perm = sq.perm;
        blocks = sq.counter;  // 32 x 32 MFMA blocks evaluated (every n_sigma)
        ctx->chunk_counter = sq.counter;
        ctx->pairs_per_chunk = 32 * 32;
    }
    // workspace: lo/hi partials, the recheck list, exact counts, flags, B of
    // every body, compaction scratch
    size_t sel_bytes = 0;
    CSPLAT_HIP(hipcub::DeviceSelect::Flagged(nullptr, sel_bytes, hipcub::CountingInputIterator<int32_t>(0),
                                             (const uint8_t *)nullptr, (int32_t *)nullptr, (int32_t *)nullptr, q,
                                             st));
    const size_t part = (size_t)S * q;
    const size_t off_list = 2 * part * 4, off_exact = off_list + (size_t)q * 4, off_flag = off_exact + (size_t)q * 4,
                 off_bq = (off_flag + (size_t)q + 255) & ~(size_t)255,
                 off_sel = (off_bq + (size_t)q * 24 + 255) & ~(size_t)255;
    hipError_t e = ctx->partial.reserve(off_sel + sel_bytes + 256);
    if (e != hipSuccess) return hip_fail(e, "precision workspace");
    char *base = ctx->partial.as<char>();
    int32_t *lo = reinterpret_cast<int32_t *>(base);
    int32_t *hi = lo + part;
    int32_t *list = reinterpret_cast<int32_t *>(base + off_list);
    int32_t *exact = reinterpret_cast<int32_t *>(base + off_exact);
    uint8_t *flag = reinterpret_cast<uint8_t *>(base + off_flag);
    float *bq = reinterpret_cast<float *>(base + off_bq);
    void *sel_tmp = base + off_sel;
    e = ctx->flags.reserve((size_t)CSPLAT_MAX_M * sizeof(int32_t) + 64);
    if (e != hipSuccess) return hip_fail(e, "flag counters");
    int32_t *n_list = ctx->flags.as<int32_t>();
    CSPLAT_HIP(zero_words(n_list, CSPLAT_MAX_M, st));
    const unsigned qb = (unsigned)((q + 255) / 256);
    ell_bmat_kernel<<<qb, 256, 0, st>>>(q, rec, bq);
    CSPLAT_HIP(hipGetLastError());
    ctx->stats.splits = S;
    ctx->stats.queries_per_lane = 2;
    ctx->stats.kernel_pairs = (int64_t)q * n;
    ctx->flag_counts = n_list;
    ctx->flag_m = m;
    float total_ms = 0.f;
    for (int v = 0; v < m; ++v) {
        const float nv = p.n_sigma[v];
        if (n_tiles > 0) {
            if (ctx->timing) (void)hipEventRecord(ctx->ev0, st);
            launch_mfma_ell(precision, cull, dim3((unsigned)(n_qblocks * S)), st, sc, n_qblocks, S, n_chunks, rec,
                            bq, q, nv, lo, hi, blocks);
            CSPLAT_HIP(hipGetLastError());
            if (ctx->timing) {
                float ms = 0.f;
                (void)hipEventRecord(ctx->ev1, st);
                CSPLAT_HIP(hipEventSynchronize(ctx->ev1));
                CSPLAT_HIP(hipEventElapsedTime(&ms, ctx->ev0, ctx->ev1));
                total_ms += ms;
            }
        }
        decide_kernel<<<qb, 256, 0, st>>>(q, n_tiles > 0 ? S : 0, m, v, p.k, out.count != nullptr, lo, hi, perm,
                                          out.label, out.count, flag);
        CSPLAT_HIP(hipGetLastError());
        CSPLAT_HIP(hipcub::DeviceSelect::Flagged(sel_tmp, sel_bytes, hipcub::CountingInputIterator<int32_t>(0), flag,
                                                 list, n_list + v, q, st));
        CSPLAT_HIP(zero_words(exact, (size_t)q, st));
        if (n > 0)
            recheck_ell_fp64_kernel<<<kRecheckGrid, 64 * kRecheckWaves, 0, st>>>(
                sc->gauss, n, cull ? sc->cull : nullptr, rec, bq, nv, list, n_list + v, exact);
        finish_kernel<<<qb, 256, 0, st>>>(m, v, p.k, list, n_list + v, exact, perm, out.label, out.count);
        CSPLAT_HIP(hipGetLastError());
        ctx->rk_list = list;
        ctx->rk_n = n_list + v;
        ctx->rk_perm = perm;
        ctx->rk_q = q;
    }
    ctx->stats.min_passes = 0;
    if (ctx->timing) {
        ctx->timed = true;
        ctx->timed_ms = total_ms;
    }
    return CSPLAT_OK;
}

}  // namespace csplat
