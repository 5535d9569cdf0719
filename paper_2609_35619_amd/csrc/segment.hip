// Planner epilogues: reductions of per-query outputs over segments of
// consecutive queries.  An RRT state or edge is in collision when any of its
// link spheres is (Sec. II-E); an MPPI rollout's collision cost sums the
// per-body averaged costs over its links and horizon (Sec. II-D, Eq. 11).
//
// One wave per segment: lanes take the segment's queries with stride 64 in
// order, then a fixed butterfly merges the lanes, so every sum has one order
// for a given segment (bit-reproducible).
#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "internal.h"

namespace csplat {
namespace {

constexpr int kSegWaves = 4;  // waves (segments in flight) per block

__device__ __forceinline__ int64_t seg_begin(const int64_t *offsets, int64_t s, int64_t len)
{
    return offsets ? offsets[s] : s * len;
}

__global__ void __launch_bounds__(64 * kSegWaves)
segment_kernel(int64_t n_seg, int32_t m, const int64_t *__restrict__ offsets, int64_t len,
               const uint8_t *__restrict__ label, const float *__restrict__ cost, uint8_t *__restrict__ seg_any,
               float *__restrict__ seg_cost)
{
    const int lane = threadIdx.x & 63;
    const int64_t wave = (int64_t)blockIdx.x * kSegWaves + (threadIdx.x >> 6);
    const int64_t waves = (int64_t)gridDim.x * kSegWaves;
    for (int64_t s = wave; s < n_seg; s += waves) {
        const int64_t j0 = seg_begin(offsets, s, len), j1 = seg_begin(offsets, s + 1, len);
        for (int v = 0; v < m; ++v) {
            int any = 0;
            float sum = 0.f;
            for (int64_t j = j0 + lane; j < j1; j += 64) {
                if (label) any |= label[j * m + v];
                if (cost) sum += cost[j * m + v];
            }
            if (seg_any) {
                const bool a = __any(any != 0);
                if (lane == 0) seg_any[s * m + v] = a ? 1 : 0;
            }
            if (seg_cost) {
#pragma unroll
                for (int off = 32; off >= 1; off >>= 1) sum += __shfl_xor(sum, off);
                if (lane == 0) seg_cost[s * m + v] = sum;
            }
        }
    }
}

__global__ void check_offsets_kernel(int64_t n_seg, int64_t q, const int64_t *__restrict__ offsets, int *bad)
{
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s > n_seg) return;
    bool ok = offsets[s] >= 0 && offsets[s] <= q;
    if (s == 0) ok = ok && offsets[0] == 0;
    if (s == n_seg) ok = ok && offsets[n_seg] == q;
    if (s < n_seg) ok = ok && offsets[s] <= offsets[s + 1];
    if (!ok) atomicOr(bad, 1);
}

}  // namespace
}  // namespace csplat

using namespace csplat;

extern "C" csplat_status csplat_segment_reduce(csplat_ctx *ctx, int64_t q, int32_t m, int64_t n_seg,
                                                const int64_t *offsets, const uint8_t *label, const float *cost,
                                                uint8_t *seg_any, float *seg_cost)
{
    if (!ctx) return fail(CSPLAT_E_INVALID, "segment_reduce: NULL ctx");
    if (q < 0 || n_seg < 0) return fail(CSPLAT_E_INVALID, "segment_reduce: q and n_seg must be >= 0");
    if (m < 1 || m > CSPLAT_MAX_M) return fail(CSPLAT_E_INVALID, "segment_reduce: m must be in 1..8");
    if (!seg_any && !seg_cost) return fail(CSPLAT_E_INVALID, "segment_reduce: no output requested");
    if ((seg_any && !label) || (seg_cost && !cost))
        return fail(CSPLAT_E_INVALID, "segment_reduce: an output without its input");
    if (n_seg == 0 && q != 0) return fail(CSPLAT_E_INVALID, "segment_reduce: queries but no segments");
    int64_t len = 0;
    if (!offsets) {
        if (n_seg > 0 && q % n_seg != 0)
            return fail(CSPLAT_E_INVALID, "segment_reduce: without offsets q must be a multiple of n_seg");
        len = n_seg > 0 ? q / n_seg : 0;
    }
    if (n_seg == 0) return CSPLAT_OK;
    const void *ptrs[] = {offsets, label, cost, seg_any, seg_cost};
    int kind = -2;
    for (const void *p : ptrs) {
        if (!p) continue;
        const int k = pointer_kind(p);
        if (kind == -2) kind = k;
        else if (kind != k) return fail(CSPLAT_E_INVALID, "segment_reduce: mix of host and device pointers");
    }
    if (kind == 0 && offsets) {
        bool ok = offsets[0] == 0 && offsets[n_seg] == q;
        for (int64_t s = 0; ok && s < n_seg; ++s) ok = offsets[s] <= offsets[s + 1];
        if (!ok) return fail(CSPLAT_E_INVALID, "segment_reduce: offsets must rise from 0 to q");
    }
    DeviceGuard g(ctx->device);
    if (g.err != hipSuccess) return hip_fail(g.err, "hipSetDevice");
    hipStream_t st = ctx->stream;
    const unsigned grid = (unsigned)std::min<int64_t>((n_seg + kSegWaves - 1) / kSegWaves, 65536);
    if (kind == 1) {
        if (offsets) {
            hipError_t e = ctx->flags.reserve(64);
            if (e != hipSuccess) return hip_fail(e, "flag workspace");
            int *bad = ctx->flags.as<int>();
            CSPLAT_HIP(zero_words(bad, 1, st));
            check_offsets_kernel<<<(unsigned)((n_seg + 256) / 256), 256, 0, st>>>(n_seg, q, offsets, bad);
            CSPLAT_HIP(hipGetLastError());
            int hbad = 0;
            CSPLAT_HIP(hipMemcpyAsync(&hbad, bad, sizeof(int), hipMemcpyDeviceToHost, st));
            CSPLAT_HIP(hipStreamSynchronize(st));
            if (hbad) return fail(CSPLAT_E_INVALID, "segment_reduce: offsets must rise from 0 to q");
        }
        segment_kernel<<<grid, 64 * kSegWaves, 0, st>>>(n_seg, m, offsets, len, label, cost, seg_any, seg_cost);
        CSPLAT_HIP(hipGetLastError());
        return CSPLAT_OK;
    }
    // host pointers: stage through the context's staging buffer
    const size_t qm = (size_t)q * m, sm = (size_t)n_seg * m;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t o = off;
        off += (bytes + 255) & ~(size_t)255;
        return o;
    };
    const size_t o_off = offsets ? take((size_t)(n_seg + 1) * 8) : 0, o_lab = label ? take(qm) : 0,
                 o_cost = cost ? take(qm * 4) : 0, o_any = seg_any ? take(sm) : 0,
                 o_sc = seg_cost ? take(sm * 4) : 0;
    hipError_t e = ctx->staging.reserve(off);
    if (e != hipSuccess) return hip_fail(e, "staging workspace");
    char *b = ctx->staging.as<char>();
    if (offsets) CSPLAT_HIP(hipMemcpyAsync(b + o_off, offsets, (size_t)(n_seg + 1) * 8, hipMemcpyHostToDevice, st));
    if (label && seg_any) CSPLAT_HIP(hipMemcpyAsync(b + o_lab, label, qm, hipMemcpyHostToDevice, st));
    if (cost && seg_cost) CSPLAT_HIP(hipMemcpyAsync(b + o_cost, cost, qm * 4, hipMemcpyHostToDevice, st));
    segment_kernel<<<grid, 64 * kSegWaves, 0, st>>>(
        n_seg, m, offsets ? (const int64_t *)(b + o_off) : nullptr, len,
        seg_any ? (const uint8_t *)(b + o_lab) : nullptr, seg_cost ? (const float *)(b + o_cost) : nullptr,
        seg_any ? (uint8_t *)(b + o_any) : nullptr, seg_cost ? (float *)(b + o_sc) : nullptr);
    CSPLAT_HIP(hipGetLastError());
    if (seg_any) CSPLAT_HIP(hipMemcpyAsync(seg_any, b + o_any, sm, hipMemcpyDeviceToHost, st));
    if (seg_cost) CSPLAT_HIP(hipMemcpyAsync(seg_cost, b + o_sc, sm * 4, hipMemcpyDeviceToHost, st));
    CSPLAT_HIP(hipStreamSynchronize(st));
    return CSPLAT_OK;
}
