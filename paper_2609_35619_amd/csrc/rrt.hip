// Batched RRT step on the GPU (Sec. II-E): samples, nearest tree node, steer,
// the edge's collision checks (n_batch x n_strides x n_links spheres through
// the float32 label path) and the append of the collision-free edges, all on
// the context's stream with the tree in device memory.
//
// Every choice is deterministic: the nearest node is the lowest index among
// equal distances, new nodes are appended in batch order, the labels are the
// culled label path's (the same bits as evaluating every pair), and the
// sample generator is a function of (seed, step, sample, axis).
#include <cmath>
#include <cstring>
#include <new>
#include <vector>

#include "internal.h"

struct csplat_rrt {
    csplat_ctx *ctx = nullptr;
    const csplat_scene *scene = nullptr;
    csplat_rrt_opts opts{};
    int32_t max_nodes = 0;
    int32_t n_links = 0;
    float *nodes = nullptr;     // device, max_nodes x 4 (x, y, z, 0)
    int32_t *parent = nullptr;  // device, max_nodes
    int32_t *counts = nullptr;  // device: [0] nodes in the tree, [1] appended by the last step
    float *links = nullptr;     // device, n_links x 4 (offset, radius)
    csplat::DevBuf work;        // the step's samples, edges, spheres and labels
    int32_t last_batch = 0;
    int32_t *last_nearest = nullptr;  // into work
    float *last_end = nullptr;
    uint8_t *last_valid = nullptr;
    uint64_t steps = 0;
};

namespace csplat {
namespace {

// SplitMix64 (Steele, Lea and Flood, "Fast splittable pseudorandom number
// generators", OOPSLA 2014): the finaliser applied to a Weyl sequence; here
// keyed by a counter, so each (seed, step, sample, axis) gets its own draw.
__device__ __forceinline__ uint64_t splitmix64(uint64_t x)
{
    x += 0x9E3779B97F4A7C15ull;
    x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
    x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
    return x ^ (x >> 31);
}

__global__ void rrt_sample_kernel(int n_batch, uint64_t seed, uint64_t step, float3 lo, float3 hi, float *samples)
{
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= n_batch) return;
    const float l[3] = {lo.x, lo.y, lo.z}, h[3] = {hi.x, hi.y, hi.z};
    for (int a = 0; a < 3; ++a) {
        const uint64_t ctr = ((step * 65536ull + (uint64_t)b) << 2) | (uint64_t)a;
        // 24 random bits -> [0, 1)
        const float u = (float)(splitmix64(seed ^ splitmix64(ctr)) >> 40) * 5.9604645e-08f;
        samples[3 * b + a] = fminf(l[a] + u * (h[a] - l[a]), h[a]);
    }
}

// Nearest node of sample b: one block per sample, threads striding over the
// nodes, the (squared distance, index) minimum (lowest index among ties).
__global__ void __launch_bounds__(256) rrt_nearest_kernel(int n_batch, const float *__restrict__ samples,
                                                          const float4 *__restrict__ nodes,
                                                          const int32_t *__restrict__ counts, int32_t *nearest)
{
    const int b = blockIdx.x;
    if (b >= n_batch) return;
    const int n = counts[0];
    const float sx = samples[3 * b], sy = samples[3 * b + 1], sz = samples[3 * b + 2];
    float best = INFINITY;
    int bi = 0x7FFFFFFF;
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
        const float4 p = nodes[i];
        const float dx = p.x - sx, dy = p.y - sy, dz = p.z - sz;
        const float d2 = fmaf(dz, dz, fmaf(dy, dy, dx * dx));
        if (d2 < best) {  // i rises: the first of equal distances is kept
            best = d2;
            bi = i;
        }
    }
    __shared__ float s_d[256];
    __shared__ int s_i[256];
    s_d[threadIdx.x] = best;
    s_i[threadIdx.x] = bi;
    __syncthreads();
    for (int off = 128; off >= 1; off >>= 1) {
        if ((int)threadIdx.x < off) {
            const float d = s_d[threadIdx.x + off];
            const int i = s_i[threadIdx.x + off];
            if (d < s_d[threadIdx.x] || (d == s_d[threadIdx.x] && i < s_i[threadIdx.x])) {
                s_d[threadIdx.x] = d;
                s_i[threadIdx.x] = i;
            }
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) nearest[b] = s_i[0];
}

// Steer and place the edge's spheres: thread (b, t, l) of n_batch x n_strides
// x n_links.  The end is the sample, or the point at distance `step` toward
// it; check point t (1..n_strides) lies at t / n_strides of the edge.
__global__ void rrt_edges_kernel(int n_batch, int n_strides, int n_links, float step,
                                 const float *__restrict__ samples, const float4 *__restrict__ nodes,
                                 const int32_t *__restrict__ nearest, const float4 *__restrict__ links,
                                 float *__restrict__ centers, float *__restrict__ radii, float *__restrict__ end,
                                 float *__restrict__ len)
{
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t total = (int64_t)n_batch * n_strides * n_links;
    if (g >= total) return;
    const int l = (int)(g % n_links);
    const int t = (int)((g / n_links) % n_strides) + 1;
    const int b = (int)(g / ((int64_t)n_links * n_strides));
    const float4 p = nodes[nearest[b]];
    const float dx = samples[3 * b] - p.x, dy = samples[3 * b + 1] - p.y, dz = samples[3 * b + 2] - p.z;
    const float d = sqrtf(fmaf(dz, dz, fmaf(dy, dy, dx * dx)));
    const float f = d > step ? step / d : 1.f;
    const float ex = fmaf(dx, f, p.x), ey = fmaf(dy, f, p.y), ez = fmaf(dz, f, p.z);
    const float w = (float)t / (float)n_strides;
    const float4 o = links[l];
    centers[3 * g] = fmaf(ex - p.x, w, p.x) + o.x;
    centers[3 * g + 1] = fmaf(ey - p.y, w, p.y) + o.y;
    centers[3 * g + 2] = fmaf(ez - p.z, w, p.z) + o.z;
    radii[g] = o.w;
    if (t == n_strides && l == 0) {
        end[3 * b] = ex;
        end[3 * b + 1] = ey;
        end[3 * b + 2] = ez;
        len[b] = d * f;
    }
}

// Edge validity (no state in collision, positive length) and the append in
// batch order: one block; thread i takes a run of consecutive edges, a block
// scan gives each its slot.
__global__ void __launch_bounds__(1024) rrt_append_kernel(int n_batch, int per_edge, int max_nodes,
                                                          const uint8_t *__restrict__ label,
                                                          const int32_t *__restrict__ nearest,
                                                          const float *__restrict__ end,
                                                          const float *__restrict__ len, float4 *nodes,
                                                          int32_t *parent, int32_t *counts, uint8_t *valid)
{
    __shared__ int s_scan[1024];
    const int tid = threadIdx.x;
    const int per = (n_batch + 1023) / 1024;
    const int b0 = tid * per, b1 = min(n_batch, b0 + per);
    int mine = 0;
    for (int b = b0; b < b1; ++b) {
        bool ok = len[b] > 0.f;
        for (int k = 0; k < per_edge && ok; ++k) ok = label[(size_t)b * per_edge + k] == 0;
        valid[b] = ok ? 1 : 0;
        mine += ok;
    }
    s_scan[tid] = mine;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {  // inclusive scan
        const int v = tid >= off ? s_scan[tid - off] : 0;
        __syncthreads();
        s_scan[tid] += v;
        __syncthreads();
    }
    const int n0 = counts[0];
    int at = n0 + s_scan[tid] - mine;
    for (int b = b0; b < b1; ++b) {
        if (!valid[b]) continue;
        if (at < max_nodes) {
            nodes[at] = make_float4(end[3 * b], end[3 * b + 1], end[3 * b + 2], 0.f);
            parent[at] = nearest[b];
        }
        ++at;
    }
    __syncthreads();
    if (tid == 0) {
        const int total = s_scan[1023];
        const int added = min(total, max_nodes - n0);
        counts[0] = n0 + added;
        counts[1] = added;
    }
}

__global__ void rrt_init_kernel(float4 *nodes, int32_t *parent, int32_t *counts, float x, float y, float z)
{
    nodes[0] = make_float4(x, y, z, 0.f);
    parent[0] = -1;
    counts[0] = 1;
    counts[1] = 0;
}

bool finite3(const float *v) { return std::isfinite(v[0]) && std::isfinite(v[1]) && std::isfinite(v[2]); }

}  // namespace
}  // namespace csplat

using namespace csplat;

extern "C" {

csplat_status csplat_rrt_create(csplat_ctx *ctx, const csplat_scene *scene, const csplat_rrt_opts *o,
                                int32_t max_nodes, const float *root, csplat_rrt **out)
{
    if (!ctx || !scene || !o || !root || !out) return fail(CSPLAT_E_INVALID, "rrt_create: NULL argument");
    *out = nullptr;
    if (scene->device != ctx->device) return fail(CSPLAT_E_INVALID, "rrt_create: scene on another device");
    if (max_nodes < 1 || max_nodes > (1 << 26)) return fail(CSPLAT_E_INVALID, "rrt_create: max_nodes out of range");
    if (!finite3(o->lo) || !finite3(o->hi) || !finite3(root))
        return fail(CSPLAT_E_INVALID, "rrt_create: box and root must be finite");
    for (int a = 0; a < 3; ++a)
        if (!(o->lo[a] < o->hi[a])) return fail(CSPLAT_E_INVALID, "rrt_create: the box needs lo < hi");
    if (!(o->step > 0.f) || !std::isfinite(o->step) || !(o->resolution > 0.f) || !std::isfinite(o->resolution))
        return fail(CSPLAT_E_INVALID, "rrt_create: step and resolution must be finite and > 0");
    if (!(o->n_sigma >= 0.f) || !std::isfinite(o->n_sigma) || o->k < 0)
        return fail(CSPLAT_E_INVALID, "rrt_create: n_sigma must be finite and >= 0, k >= 0");
    if (o->n_links < 1 || o->n_links > 64 || !o->link_offsets || !o->link_radii)
        return fail(CSPLAT_E_INVALID, "rrt_create: 1..64 links with offsets and radii");
    if (std::ceil(o->step / o->resolution) > 4096.f)
        return fail(CSPLAT_E_INVALID, "rrt_create: more than 4096 checks per edge");
    std::vector<float> lk((size_t)o->n_links * 4);
    for (int l = 0; l < o->n_links; ++l) {
        if (!finite3(o->link_offsets + 3 * l) || !(o->link_radii[l] > 0.f) || !std::isfinite(o->link_radii[l]))
            return fail(CSPLAT_E_INVALID, "rrt_create: link offsets finite, radii finite and > 0");
        for (int a = 0; a < 3; ++a) lk[(size_t)4 * l + a] = o->link_offsets[3 * l + a];
        lk[(size_t)4 * l + 3] = o->link_radii[l];
    }
    DeviceGuard g(ctx->device);
    if (g.err != hipSuccess) return hip_fail(g.err, "hipSetDevice");
    csplat_rrt *t = new (std::nothrow) csplat_rrt();
    if (!t) return fail(CSPLAT_E_OOM, "rrt_create: host allocation");
    t->ctx = ctx;
    t->work.stream = ctx->stream;
    t->scene = scene;
    t->opts = *o;
    t->opts.link_offsets = nullptr;
    t->opts.link_radii = nullptr;
    t->max_nodes = max_nodes;
    t->n_links = o->n_links;
    hipError_t e = hipMalloc(&t->nodes, (size_t)max_nodes * 16);
    if (e == hipSuccess) e = hipMalloc(&t->parent, (size_t)max_nodes * 4);
    if (e == hipSuccess) e = hipMalloc(&t->counts, 64);
    if (e == hipSuccess) e = hipMalloc(&t->links, lk.size() * 4);
    if (e == hipSuccess) e = hipMemcpyAsync(t->links, lk.data(), lk.size() * 4, hipMemcpyHostToDevice, ctx->stream);
    if (e == hipSuccess) {
        rrt_init_kernel<<<1, 1, 0, ctx->stream>>>(reinterpret_cast<float4 *>(t->nodes), t->parent, t->counts,
                                                  root[0], root[1], root[2]);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
    if (e != hipSuccess) {
        csplat_status st = hip_fail(e, "rrt_create");
        csplat_rrt_destroy(t);
        return st;
    }
    *out = t;
    return CSPLAT_OK;
}

csplat_status csplat_rrt_destroy(csplat_rrt *t)
{
    if (!t) return CSPLAT_OK;
    DeviceGuard g(t->ctx->device);
    (void)hipStreamSynchronize(t->ctx->stream);
    if (t->nodes) (void)hipFree(t->nodes);
    if (t->parent) (void)hipFree(t->parent);
    if (t->counts) (void)hipFree(t->counts);
    if (t->links) (void)hipFree(t->links);
    t->work.release();
    delete t;
    return CSPLAT_OK;
}

csplat_status csplat_rrt_step(csplat_rrt *t, int32_t n_batch, const float *samples, int32_t *n_added)
{
    if (!t) return fail(CSPLAT_E_INVALID, "rrt_step: NULL tree");
    if (n_batch < 1 || n_batch > 65536) return fail(CSPLAT_E_INVALID, "rrt_step: n_batch must be in 1..65536");
    if (samples && pointer_kind(samples) != 1) return fail(CSPLAT_E_INVALID, "rrt_step: samples must be a device pointer");
    csplat_ctx *ctx = t->ctx;
    const int n_strides = std::max(1, (int)std::ceil(t->opts.step / t->opts.resolution));
    const int per_edge = n_strides * t->n_links;
    const int64_t q = (int64_t)n_batch * per_edge;
    if (q > (1 << 24)) return fail(CSPLAT_E_INVALID, "rrt_step: more than 2^24 spheres in one step");
    DeviceGuard g(ctx->device);
    if (g.err != hipSuccess) return hip_fail(g.err, "hipSetDevice");
    hipStream_t st = ctx->stream;
    // workspace: samples, nearest, end, length, valid, sphere centres and radii, labels
    auto al = [](size_t b) { return (b + 255) & ~(size_t)255; };
    const size_t nb = (size_t)n_batch, qn = (size_t)q;
    const size_t o_smp = 0, o_near = o_smp + al(nb * 12), o_end = o_near + al(nb * 4), o_len = o_end + al(nb * 12),
                 o_valid = o_len + al(nb * 4), o_c = o_valid + al(nb), o_r = o_c + al(qn * 12),
                 o_lab = o_r + al(qn * 4), total = o_lab + al(qn);
    hipError_t e = t->work.reserve(total);
    if (e != hipSuccess) return hip_fail(e, "rrt workspace");
    char *w = t->work.as<char>();
    float *smp = samples ? const_cast<float *>(samples) : reinterpret_cast<float *>(w + o_smp);
    int32_t *nearest = reinterpret_cast<int32_t *>(w + o_near);
    float *end = reinterpret_cast<float *>(w + o_end), *len = reinterpret_cast<float *>(w + o_len);
    uint8_t *valid = reinterpret_cast<uint8_t *>(w + o_valid);
    float *centers = reinterpret_cast<float *>(w + o_c), *radii = reinterpret_cast<float *>(w + o_r);
    uint8_t *label = reinterpret_cast<uint8_t *>(w + o_lab);
    if (!samples) {
        rrt_sample_kernel<<<(unsigned)((n_batch + 255) / 256), 256, 0, st>>>(
            n_batch, t->opts.seed, t->steps, make_float3(t->opts.lo[0], t->opts.lo[1], t->opts.lo[2]),
            make_float3(t->opts.hi[0], t->opts.hi[1], t->opts.hi[2]), smp);
        CSPLAT_HIP(hipGetLastError());
    }
    const float4 *nodes4 = reinterpret_cast<const float4 *>(t->nodes);
    rrt_nearest_kernel<<<(unsigned)n_batch, 256, 0, st>>>(n_batch, smp, nodes4, t->counts, nearest);
    rrt_edges_kernel<<<(unsigned)((q + 255) / 256), 256, 0, st>>>(
        n_batch, n_strides, t->n_links, t->opts.step, smp, nodes4, nearest,
        reinterpret_cast<const float4 *>(t->links), centers, radii, end, len);
    CSPLAT_HIP(hipGetLastError());
    // the collision labels of every state's links (the label path of csplat_eval)
    csplat_reduce_opts ro{};
    ro.k = t->opts.k;
    ro.softmin_tau = 0.f;
    ro.neighbor_radius = INFINITY;
    ro.d_max = 1.f;
    ro.gamma = 1.f;
    ro.s_min = 1.f;
    ro.precision = CSPLAT_PRECISION_FP32;
    ro.cull = 1;
    EvalParams p;
    csplat_status s = build_params(&t->opts.n_sigma, 1, ro, p);
    if (s != CSPLAT_OK) return s;
    EvalOut eo{label, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr};
    s = fp32_eval(ctx, t->scene, q, centers, radii, p, eo, true, false);
    scene_note_use(t->scene, st);
    if (s != CSPLAT_OK) return s;
    rrt_append_kernel<<<1, 1024, 0, st>>>(n_batch, per_edge, t->max_nodes, label, nearest, end, len,
                                          reinterpret_cast<float4 *>(t->nodes), t->parent, t->counts, valid);
    CSPLAT_HIP(hipGetLastError());
    t->last_batch = n_batch;
    t->last_nearest = nearest;
    t->last_end = end;
    t->last_valid = valid;
    ++t->steps;
    if (n_added) {
        CSPLAT_HIP(hipMemcpyAsync(n_added, t->counts + 1, sizeof(int32_t), hipMemcpyDeviceToHost, st));
        CSPLAT_HIP(hipStreamSynchronize(st));
    }
    return CSPLAT_OK;
}

csplat_status csplat_rrt_nodes(csplat_rrt *t, float *pos, int32_t *parent, int32_t cap, int32_t *n)
{
    if (!t || !n || cap < 0) return fail(CSPLAT_E_INVALID, "rrt_nodes: bad argument");
    DeviceGuard g(t->ctx->device);
    hipStream_t st = t->ctx->stream;
    int32_t c[2] = {0, 0};
    CSPLAT_HIP(hipMemcpyAsync(c, t->counts, sizeof(c), hipMemcpyDeviceToHost, st));
    CSPLAT_HIP(hipStreamSynchronize(st));
    *n = c[0];
    const int k = std::min(cap, c[0]);
    if (k > 0 && pos) {
        std::vector<float> tmp((size_t)k * 4);
        CSPLAT_HIP(hipMemcpyAsync(tmp.data(), t->nodes, (size_t)k * 16, hipMemcpyDeviceToHost, st));
        CSPLAT_HIP(hipStreamSynchronize(st));
        for (int i = 0; i < k; ++i)
            for (int a = 0; a < 3; ++a) pos[3 * i + a] = tmp[(size_t)4 * i + a];
    }
    if (k > 0 && parent) {
        CSPLAT_HIP(hipMemcpyAsync(parent, t->parent, (size_t)k * 4, hipMemcpyDeviceToHost, st));
        CSPLAT_HIP(hipStreamSynchronize(st));
    }
    return CSPLAT_OK;
}

csplat_status csplat_rrt_last_edges(csplat_rrt *t, int32_t *nearest, float *end, uint8_t *valid)
{
    if (!t) return fail(CSPLAT_E_INVALID, "rrt_last_edges: NULL tree");
    if (t->last_batch == 0) return CSPLAT_OK;
    DeviceGuard g(t->ctx->device);
    hipStream_t st = t->ctx->stream;
    const size_t nb = (size_t)t->last_batch;
    if (nearest) CSPLAT_HIP(hipMemcpyAsync(nearest, t->last_nearest, nb * 4, hipMemcpyDeviceToHost, st));
    if (end) CSPLAT_HIP(hipMemcpyAsync(end, t->last_end, nb * 12, hipMemcpyDeviceToHost, st));
    if (valid) CSPLAT_HIP(hipMemcpyAsync(valid, t->last_valid, nb, hipMemcpyDeviceToHost, st));
    CSPLAT_HIP(hipStreamSynchronize(st));
    return CSPLAT_OK;
}

}  // extern "C"
