// The C ABI of the library: argument validation, ownership and dispatch.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <initializer_list>
#include <new>
#include <string>
#include <vector>

#include <mutex>

#include "internal.h"

// Device workspace of csplat_eval_noalloc: a fixed array in the library's
// code object, one copy per GPU, held until the process ends.  Host code
// never passes this name to a kernel (on the host it is only a handle): the
// device address of each GPU's copy is looked up once per device at context
// creation and used from then on.
constexpr size_t kScratchBytes = (size_t)CSPLAT_NOALLOC_SCRATCH_MB << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace csplat {

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_dev[kMaxDevices] = {};  // device address of each GPU's copy of `scratch`

// With `device` current: the device address of its copy of `scratch`.
csplat_status scratch_setup(int device)
{
    if (device < 0 || device >= kMaxDevices) return fail(CSPLAT_E_INVALID, "scratch: device index out of range");
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (g_scratch_dev[device]) return CSPLAT_OK;
    void *ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr) return hip_fail(e != hipSuccess ? e : hipErrorInvalidSymbol, "hipGetSymbolAddress(scratch)");
    g_scratch_dev[device] = ptr;
    return CSPLAT_OK;
}

void *scratch_of(int device)
{
    if (device < 0 || device >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    return g_scratch_dev[device];
}
}  // namespace

thread_local std::string g_last_error;

void set_error(const std::string &msg) { g_last_error = msg; }

csplat_status fail(csplat_status code, const std::string &msg)
{
    g_last_error = msg;
    return code;
}

csplat_status hip_fail(hipError_t e, const char *what)
{
    g_last_error = std::string(what) + ": " + hipGetErrorString(e);
    return e == hipErrorOutOfMemory ? CSPLAT_E_OOM : CSPLAT_E_DEVICE;
}

// Work items per launch: CSPLAT_BLOCKS_PER_CU blocks per compute unit.
int target_blocks(int dev)
{
    static int cache[64] = {0};
    if (dev < 0 || dev >= 64) return 256 * CSPLAT_BLOCKS_PER_CU;
    if (!cache[dev]) {
        int v = 0;
        if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || v <= 0)
            v = 256;
        cache[dev] = v * CSPLAT_BLOCKS_PER_CU;
    }
    return cache[dev];
}

namespace {
__global__ void zero_kernel(int32_t *p, size_t n)
{
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0;
}
}  // namespace

hipError_t zero_words(int32_t *p, size_t n, hipStream_t st)
{
    if (n == 0) return hipSuccess;
    zero_kernel<<<(unsigned)((n + 255) / 256), 256, 0, st>>>(p, n);
    return hipGetLastError();
}

hipError_t DevBuf::reserve(size_t want)
{
    if (want <= bytes) return hipSuccess;
    // earlier work on the owner's stream may still use the old block: it is
    // released in stream order, after that work
    release();
    size_t grow = want + want / 4;
    hipError_t e = hipMallocAsync(&ptr, grow, stream);
    if (e != hipSuccess) {
        ptr = nullptr;
        bytes = 0;
        return e;
    }
    bytes = grow;
    return hipSuccess;
}

void DevBuf::release()
{
    if (ptr) (void)hipFreeAsync(ptr, stream);
    ptr = nullptr;
    bytes = 0;
}

void scene_note_use(const csplat_scene *sc, hipStream_t st, bool may_create)
{
    if (!sc) return;
    std::lock_guard<std::mutex> lk(sc->use_mu);
    for (auto &u : sc->uses)
        if (u.first == st) {
            if (u.second) (void)hipEventRecord(u.second, st);
            return;
        }
    hipEvent_t ev = nullptr;
    // without an event (not created, or not allowed to be: the allocation-free
    // entry point) freeing the scene waits for the whole stream instead
    if (may_create && hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess) ev = nullptr;
    sc->uses.emplace_back(st, ev);
    if (ev) (void)hipEventRecord(ev, st);
}

// A non-blocking stream per device on which scene memory is released (after
// waiting for the scene's users), created on first use.
hipStream_t release_stream(int device)
{
    static std::mutex mu;
    static hipStream_t streams[64] = {};
    if (device < 0 || device >= 64) return nullptr;
    std::lock_guard<std::mutex> lk(mu);
    if (!streams[device] && hipStreamCreateWithFlags(&streams[device], hipStreamNonBlocking) != hipSuccess)
        streams[device] = nullptr;
    return streams[device];
}

// 0: host, 1: device
int pointer_kind(const void *p)
{
    hipPointerAttribute_t a;
    if (hipPointerGetAttributes(&a, p) != hipSuccess) {
        (void)hipGetLastError();
        return 0;
    }
    if (a.type == hipMemoryTypeDevice || a.type == hipMemoryTypeManaged) return 1;
    return 0;
}

csplat_status build_params(const float *n_sigma, int m, const csplat_reduce_opts &o, EvalParams &p)
{
    if (o.k < 0) return fail(CSPLAT_E_INVALID, "reduce opts: k must be >= 0");
    if (!(o.softmin_tau >= 0.f) || !std::isfinite(o.softmin_tau))
        return fail(CSPLAT_E_INVALID, "reduce opts: softmin_tau must be finite and >= 0");
    if (!(o.neighbor_radius > 0.f))
        return fail(CSPLAT_E_INVALID, "reduce opts: neighbor_radius must be > 0 (or +inf)");
    if (!(o.d_max > 0.f) || !std::isfinite(o.d_max))
        return fail(CSPLAT_E_INVALID, "reduce opts: d_max must be finite and > 0");
    if (!(o.gamma >= 0.f) || !std::isfinite(o.gamma))
        return fail(CSPLAT_E_INVALID, "reduce opts: gamma must be finite and >= 0");
    if (!std::isfinite(o.s_min)) return fail(CSPLAT_E_INVALID, "reduce opts: s_min must be finite");
    if (o.precision < CSPLAT_PRECISION_FP32 || o.precision > CSPLAT_PRECISION_FP16_RECHECK)
        return fail(CSPLAT_E_INVALID, "reduce opts: unknown precision");
    std::memset(&p, 0, sizeof(p));
    p.m = m;
    p.k = o.k;
    for (int v = 0; v < m; ++v) {
        double n = n_sigma[v];
        p.n_sigma[v] = n_sigma[v];
        p.two_n[v] = (float)(2.0 * n);
        p.four_n2[v] = (float)(4.0 * n * n);
    }
    p.soft = o.softmin_tau > 0.f;
    // t = s~^2 * kt; the softmin sum is sum 2^(t_min - t), so kt = log2(e) / tau
    double kt = p.soft ? 1.4426950408889634 / (double)o.softmin_tau : 1.0;
    if (!std::isfinite((float)kt)) return fail(CSPLAT_E_INVALID, "reduce opts: softmin_tau too small");
    p.kt = (float)kt;
    p.inv_kt = (float)(1.0 / kt);
    // cost term d_max exp(-gamma max(s~^2 - s_min, 0)) = d_max 2^min(g0 - g1 t, 0)
    p.g1 = (float)((double)o.gamma * 1.4426950408889634 / kt);
    p.g0 = (float)((double)o.gamma * 1.4426950408889634 * (double)o.s_min);
    p.d_max = o.d_max;
    p.rn2 = std::isinf(o.neighbor_radius) ? INFINITY
                                          : (float)((double)o.neighbor_radius * o.neighbor_radius);
    p.r_nbr = o.neighbor_radius;
    p.n_max = 0.f;
    for (int v = 0; v < m; ++v) p.n_max = std::max(p.n_max, n_sigma[v]);
    if (o.cull != 0 && o.cull != 1) return fail(CSPLAT_E_INVALID, "reduce opts: cull must be 0 or 1");
    p.cull = o.cull;
    return CSPLAT_OK;
}

namespace {

// Query spheres must have finite centres and finite radii > 0.  Host arrays
// are checked here; device arrays by check_queries_kernel before any output
// is written.
bool queries_valid_host(int64_t q, const float *c, const float *r)
{
    for (int64_t j = 0; j < q; ++j) {
        if (!std::isfinite(c[3 * j]) || !std::isfinite(c[3 * j + 1]) || !std::isfinite(c[3 * j + 2]))
            return false;
        if (!(r[j] > 0.f) || !std::isfinite(r[j])) return false;
    }
    return true;
}

__global__ void check_queries_kernel(int64_t q, const float *__restrict__ c, const float *__restrict__ r,
                                     int *bad)
{
    int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= q) return;
    bool ok = isfinite(c[3 * j]) && isfinite(c[3 * j + 1]) && isfinite(c[3 * j + 2]) && r[j] > 0.f &&
              isfinite(r[j]);
    if (!ok) *bad = 1;  // every writer stores the same value
}

}  // namespace

// Ellipsoidal bodies: finite centres, finite nonzero quaternions, finite
// semi-axes > 0.
bool bodies_valid_host(int64_t q, const float *c, const float *quat, const float *ax)
{
    for (int64_t j = 0; j < q; ++j) {
        float qq = 0.f;
        for (int k = 0; k < 3; ++k)
            if (!std::isfinite(c[3 * j + k]) || !(ax[3 * j + k] > 0.f) || !std::isfinite(ax[3 * j + k])) return false;
        for (int k = 0; k < 4; ++k) {
            if (!std::isfinite(quat[4 * j + k])) return false;
            qq += quat[4 * j + k] * quat[4 * j + k];
        }
        if (!(qq > 0.f)) return false;
    }
    return true;
}

namespace {

__global__ void check_bodies_kernel(int64_t q, const float *__restrict__ c, const float *__restrict__ quat,
                                    const float *__restrict__ ax, int *bad)
{
    int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= q) return;
    bool ok = true;
    float qq = 0.f;
    for (int k = 0; k < 3; ++k) ok = ok && isfinite(c[3 * j + k]) && ax[3 * j + k] > 0.f && isfinite(ax[3 * j + k]);
    for (int k = 0; k < 4; ++k) {
        ok = ok && isfinite(quat[4 * j + k]);
        qq += quat[4 * j + k] * quat[4 * j + k];
    }
    if (!(ok && qq > 0.f)) atomicOr(bad, 1);
}

// Checks common to the evaluation calls; fills p.
csplat_status eval_checks(csplat_ctx *ctx, const csplat_scene *sc, int64_t q, const csplat_reduce_opts *opts,
                          const csplat_outputs *out, const char *who, EvalParams &p, bool &want_dist)
{
    if (!ctx || !sc || !opts || !out) return fail(CSPLAT_E_INVALID, std::string(who) + ": NULL argument");
    if (q < 0) return fail(CSPLAT_E_INVALID, std::string(who) + ": q < 0");
    if (q > (int64_t)0x7FFFFFFF / 8) return fail(CSPLAT_E_INVALID, std::string(who) + ": q too large");
    if (sc->device != ctx->device) return fail(CSPLAT_E_INVALID, std::string(who) + ": scene on another device");
    csplat_status s = build_params(ctx->n_sigma, ctx->m, *opts, p);
    if (s != CSPLAT_OK) return s;
    want_dist = out->min || out->softmin || out->cost || out->nbr;
    if (!want_dist && !out->label && !out->count && !out->err)
        return fail(CSPLAT_E_INVALID, std::string(who) + ": no output requested");
    if (out->err && opts->precision == CSPLAT_PRECISION_FP32)
        return fail(CSPLAT_E_INVALID, std::string(who) + ": err is an output of the precision forms");
    return CSPLAT_OK;
}

// One kind (1 device, 0 host) for every non-NULL pointer, or -1 for a mix.
int common_kind(std::initializer_list<const void *> ptrs)
{
    int kind = -2;
    for (const void *ptr : ptrs) {
        if (!ptr) continue;
        int k = pointer_kind(ptr);
        if (kind == -2) kind = k;
        else if (kind != k) return -1;
    }
    return kind == -2 ? 0 : kind;
}

// Device-side validation: `launch(bad)` queues a check kernel that sets *bad.
template <class Launch>
csplat_status device_check(csplat_ctx *ctx, Launch launch, const char *msg)
{
    hipError_t e = ctx->flags.reserve(64);
    if (e != hipSuccess) return hip_fail(e, "flag workspace");
    int *bad = ctx->flags.as<int>();
    CSPLAT_HIP(zero_words(bad, 1, ctx->stream));
    launch(bad);
    CSPLAT_HIP(hipGetLastError());
    int hbad = 0;
    CSPLAT_HIP(hipMemcpyAsync(&hbad, bad, sizeof(int), hipMemcpyDeviceToHost, ctx->stream));
    CSPLAT_HIP(hipStreamSynchronize(ctx->stream));
    if (hbad) return fail(CSPLAT_E_INVALID, msg);
    return CSPLAT_OK;
}

// The same check queued without waiting: the check kernel stores its flag
// straight into pinned host memory (cleared by the host first), an event
// follows it, and wait_device_check() waits for that event only (the work
// queued after it keeps the device busy meanwhile).
template <class Launch>
csplat_status queue_device_check(csplat_ctx *ctx, Launch launch)
{
    // the flag and its event are allocated by csplat_ctx_create
    if (!ctx->check_host || !ctx->ev_check) return fail(CSPLAT_E_DEVICE, "context without check flag");
    // a check of an evaluation that ended early may still be queued: it
    // finishes before its flag is cleared for this one
    if (ctx->check_pending) {
        CSPLAT_HIP(hipEventSynchronize(ctx->ev_check));
        ctx->check_pending = false;
    }
    *ctx->check_host = 0;
    launch(ctx->check_dev);
    CSPLAT_HIP(hipGetLastError());
    CSPLAT_HIP(hipEventRecord(ctx->ev_check, ctx->stream));
    ctx->check_pending = true;
    return CSPLAT_OK;
}

csplat_status wait_device_check(csplat_ctx *ctx, const char *msg)
{
    CSPLAT_HIP(hipEventSynchronize(ctx->ev_check));
    ctx->check_pending = false;
    if (*ctx->check_host) return fail(CSPLAT_E_INVALID, msg);
    return CSPLAT_OK;
}

// Runs run(dev_inputs, eo) with every input and output on the device: device
// pointers as given (asynchronous); host inputs staged through the context's
// staging buffer and host outputs copied back (synchronous).
template <class Run>
csplat_status on_device(csplat_ctx *ctx, int kind, int64_t q, int m, std::initializer_list<const void *> in,
                        std::initializer_list<size_t> in_bytes, const csplat_outputs *out, Run run)
{
    std::vector<const void *> dev_in(in);
    if (kind == 1) {
        EvalOut eo{out->label, out->count, out->min, out->softmin, out->cost, out->nbr, out->err};
        return run(dev_in, eo);
    }
    const size_t qm = (size_t)q * m;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t o = off;
        off += (bytes + 255) & ~(size_t)255;
        return o;
    };
    std::vector<size_t> o_in;
    for (size_t b : in_bytes) o_in.push_back(take(b));
    const size_t o_lab = out->label ? take(qm) : 0, o_cnt = out->count ? take(qm * 4) : 0;
    const size_t o_min = out->min ? take(qm * 4) : 0, o_sm = out->softmin ? take(qm * 4) : 0;
    const size_t o_cs = out->cost ? take(qm * 4) : 0, o_nb = out->nbr ? take((size_t)q * 4) : 0;
    const size_t o_er = out->err ? take(qm * 4) : 0;
    hipError_t e = ctx->staging.reserve(off);
    if (e != hipSuccess) return hip_fail(e, "staging workspace");
    char *b = ctx->staging.as<char>();
    hipStream_t st = ctx->stream;
    size_t i = 0;
    for (size_t bytes : in_bytes) {
        CSPLAT_HIP(hipMemcpyAsync(b + o_in[i], dev_in[i], bytes, hipMemcpyHostToDevice, st));
        dev_in[i] = b + o_in[i];
        ++i;
    }
    EvalOut eo{out->label ? (uint8_t *)(b + o_lab) : nullptr, out->count ? (int32_t *)(b + o_cnt) : nullptr,
               out->min ? (float *)(b + o_min) : nullptr, out->softmin ? (float *)(b + o_sm) : nullptr,
               out->cost ? (float *)(b + o_cs) : nullptr, out->nbr ? (int32_t *)(b + o_nb) : nullptr,
               out->err ? (float *)(b + o_er) : nullptr};
    csplat_status s = run(dev_in, eo);
    if (s != CSPLAT_OK) return s;
    if (out->label) CSPLAT_HIP(hipMemcpyAsync(out->label, eo.label, qm, hipMemcpyDeviceToHost, st));
    if (out->count) CSPLAT_HIP(hipMemcpyAsync(out->count, eo.count, qm * 4, hipMemcpyDeviceToHost, st));
    if (out->min) CSPLAT_HIP(hipMemcpyAsync(out->min, eo.min, qm * 4, hipMemcpyDeviceToHost, st));
    if (out->softmin) CSPLAT_HIP(hipMemcpyAsync(out->softmin, eo.softmin, qm * 4, hipMemcpyDeviceToHost, st));
    if (out->cost) CSPLAT_HIP(hipMemcpyAsync(out->cost, eo.cost, qm * 4, hipMemcpyDeviceToHost, st));
    if (out->nbr) CSPLAT_HIP(hipMemcpyAsync(out->nbr, eo.nbr, (size_t)q * 4, hipMemcpyDeviceToHost, st));
    if (out->err) CSPLAT_HIP(hipMemcpyAsync(out->err, eo.err, qm * 4, hipMemcpyDeviceToHost, st));
    CSPLAT_HIP(hipStreamSynchronize(st));
    return CSPLAT_OK;
}

void reset_stats(csplat_ctx *ctx, int64_t q, const csplat_scene *sc)
{
    std::memset(&ctx->stats, 0, sizeof(ctx->stats));
    ctx->stats.pairs = q * sc->n;
    ctx->timed = false;
    ctx->timed_ms = -1.f;
    ctx->flag_counts = nullptr;
    ctx->flag_m = 0;
    ctx->chunk_counter = nullptr;
    ctx->rk_list = ctx->rk_n = ctx->rk_perm = nullptr;
    ctx->rk_q = 0;
}

}  // namespace
}  // namespace csplat

using namespace csplat;

extern "C" {

const char *csplat_last_error(void) { return g_last_error.c_str(); }

csplat_status csplat_ctx_create(int32_t device, void *hip_stream, csplat_ctx **out)
{
    if (!out) return fail(CSPLAT_E_INVALID, "ctx_create: out is NULL");
    *out = nullptr;
    int ndev = 0;
    hipError_t e = hipGetDeviceCount(&ndev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDeviceCount");
    if (device < 0 || device >= ndev) return fail(CSPLAT_E_INVALID, "ctx_create: no such device");
    DeviceGuard g(device);
    if (g.err != hipSuccess) return hip_fail(g.err, "hipSetDevice");
    csplat_ctx *ctx = new (std::nothrow) csplat_ctx();
    if (!ctx) return fail(CSPLAT_E_OOM, "ctx_create: host allocation");
    ctx->device = device;
    if (hip_stream) {
        ctx->stream = static_cast<hipStream_t>(hip_stream);
    } else {
        e = hipStreamCreateWithFlags(&ctx->stream, hipStreamNonBlocking);
        if (e != hipSuccess) {
            delete ctx;
            return hip_fail(e, "hipStreamCreate");
        }
        ctx->own_stream = true;
    }
    for (DevBuf *b : {&ctx->partial, &ctx->staging, &ctx->flags, &ctx->sortbuf, &ctx->bodies, &ctx->minbuf})
        b->stream = ctx->stream;
    ctx->m = 1;
    ctx->n_sigma[0] = 1.0f;
    // the device-side input check's pinned flag and event, allocated here so
    // that no evaluation allocates them; this device's scratch address
    csplat_status s = CSPLAT_OK;
    e = hipHostMalloc((void **)&ctx->check_host, 64, hipHostMallocDefault);
    if (e == hipSuccess) e = hipHostGetDevicePointer((void **)&ctx->check_dev, ctx->check_host, 0);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&ctx->ev_check, hipEventDisableTiming);
    if (e != hipSuccess) s = hip_fail(e, "ctx_create: check flag");
    if (s == CSPLAT_OK) s = scratch_setup(device);
    if (s != CSPLAT_OK) {
        const std::string msg = g_last_error;
        csplat_ctx_destroy(ctx);
        return fail(s, msg);
    }
    *out = ctx;
    return CSPLAT_OK;
}

csplat_status csplat_ctx_destroy(csplat_ctx *ctx)
{
    if (!ctx) return CSPLAT_OK;
    DeviceGuard g(ctx->device);
    ctx->partial.release();
    ctx->staging.release();
    ctx->flags.release();
    ctx->sortbuf.release();
    ctx->bodies.release();
    ctx->minbuf.release();
    (void)hipStreamSynchronize(ctx->stream);
    if (ctx->ev0) (void)hipEventDestroy(ctx->ev0);
    if (ctx->ev1) (void)hipEventDestroy(ctx->ev1);
    if (ctx->ev_check) (void)hipEventDestroy(ctx->ev_check);
    if (ctx->check_host) (void)hipHostFree(ctx->check_host);
    if (ctx->own_stream) (void)hipStreamDestroy(ctx->stream);
    delete ctx;
    return CSPLAT_OK;
}

csplat_status csplat_scene_load(csplat_ctx *ctx, int64_t n, const float *means, const float *quats,
                                const float *scales, const float *opacity,
                                const csplat_scene_opts *opts, csplat_scene **out)
{
    if (!ctx || !out) return fail(CSPLAT_E_INVALID, "scene_load: NULL ctx or out");
    *out = nullptr;
    if (n < 0) return fail(CSPLAT_E_INVALID, "scene_load: n < 0");
    if (n > 0 && (!means || !quats || !scales || !opacity))
        return fail(CSPLAT_E_INVALID, "scene_load: NULL input array");
    csplat_scene_opts o{};
    o.param_mode = CSPLAT_PARAM_ACTIVATED;
    if (opts) o = *opts;
    if (o.param_mode != CSPLAT_PARAM_ACTIVATED && o.param_mode != CSPLAT_PARAM_RAW_3DGS)
        return fail(CSPLAT_E_INVALID, "scene_load: unknown param_mode");
    if (!std::isfinite(o.floater_opacity_max) || !std::isfinite(o.floater_extent_min))
        return fail(CSPLAT_E_INVALID, "scene_load: non-finite floater thresholds");
    if (o.precision_features &
        ~(CSPLAT_FEATURES_BF16 | CSPLAT_FEATURES_FP16 | CSPLAT_FEATURES_ELL_BF16 | CSPLAT_FEATURES_ELL_FP16))
        return fail(CSPLAT_E_INVALID, "scene_load: unknown precision feature bits");
    if (n > 0) {  // the scene arrays are host arrays: reject device pointers early
        if (pointer_kind(means) || pointer_kind(quats) || pointer_kind(scales) || pointer_kind(opacity))
            return fail(CSPLAT_E_INVALID, "scene_load: inputs must be host pointers");
    }
    DeviceGuard g(ctx->device);
    if (g.err != hipSuccess) return hip_fail(g.err, "hipSetDevice");
    csplat_scene *sc = new (std::nothrow) csplat_scene();
    if (!sc) return fail(CSPLAT_E_OOM, "scene_load: host allocation");
    csplat_status s = scene_build(ctx, n, means, quats, scales, opacity, o, sc);
    if (s == CSPLAT_OK && o.precision_features && sc->n > 0)
        s = precision_build(ctx, sc, o.precision_features);
    if (s != CSPLAT_OK) {
        scene_release(sc, ctx->stream);
        (void)hipStreamSynchronize(ctx->stream);
        delete sc;
        return s;
    }
    *out = sc;
    return CSPLAT_OK;
}

csplat_status csplat_scene_info(const csplat_scene *sc, int64_t *n_kept, uint64_t *device_bytes)
{
    if (!sc) return fail(CSPLAT_E_INVALID, "scene_info: NULL scene");
    if (n_kept) *n_kept = sc->n;
    if (device_bytes) *device_bytes = sc->device_bytes;
    return CSPLAT_OK;
}

csplat_status csplat_scene_free(csplat_scene *sc)
{
    if (!sc) return CSPLAT_OK;
    DeviceGuard g(sc->device);
    hipStream_t rs = release_stream(sc->device);
    {
        std::lock_guard<std::mutex> lk(sc->use_mu);
        for (auto &u : sc->uses) {
            if (u.second && rs) {
                (void)hipStreamWaitEvent(rs, u.second, 0);
                (void)hipEventDestroy(u.second);
            } else {
                (void)hipStreamSynchronize(u.first);
                if (u.second) (void)hipEventDestroy(u.second);
            }
        }
        sc->uses.clear();
    }
    scene_release(sc, rs);
    delete sc;
    return CSPLAT_OK;
}

csplat_status csplat_set_conservatism(csplat_ctx *ctx, const float *n_sigma, int32_t m)
{
    if (!ctx || !n_sigma) return fail(CSPLAT_E_INVALID, "set_conservatism: NULL argument");
    if (m < 1 || m > CSPLAT_MAX_M) return fail(CSPLAT_E_INVALID, "set_conservatism: m must be in 1..8");
    for (int v = 0; v < m; ++v)
        if (!(n_sigma[v] >= 0.f) || !std::isfinite(n_sigma[v]))
            return fail(CSPLAT_E_INVALID, "set_conservatism: n_sigma must be finite and >= 0");
    ctx->m = m;
    for (int v = 0; v < m; ++v) ctx->n_sigma[v] = n_sigma[v];
    return CSPLAT_OK;
}

csplat_status csplat_eval(csplat_ctx *ctx, const csplat_scene *sc, int64_t q, const float *centers,
                          const float *radii, const csplat_reduce_opts *opts,
                          const csplat_outputs *out)
{
    EvalParams p;
    bool want_dist = false;
    csplat_status s = eval_checks(ctx, sc, q, opts, out, "eval", p, want_dist);
    if (s != CSPLAT_OK) return s;
    if (opts->precision != CSPLAT_PRECISION_FP32) {
        if (out->softmin || out->cost || out->nbr)
            return fail(CSPLAT_E_INVALID, "eval: the MFMA precision forms compute labels, counts and min only");
        if (std::isfinite(opts->neighbor_radius))
            return fail(CSPLAT_E_INVALID,
                        "eval: the MFMA precision forms count over every kept Gaussian (neighbor_radius = +inf)");
        uint32_t need = opts->precision == CSPLAT_PRECISION_BF16_RECHECK ? CSPLAT_FEATURES_BF16
                                                                          : CSPLAT_FEATURES_FP16;
        void *f = need == CSPLAT_FEATURES_BF16 ? sc->feat_bf16 : sc->feat_fp16;
        if (sc->n > 0 && !f)
            return fail(CSPLAT_E_INVALID, "eval: scene was loaded without the requested precision features");
    }
    if (q == 0) return CSPLAT_OK;
    if (!centers || !radii) return fail(CSPLAT_E_INVALID, "eval: NULL centers or radii");
    const int kind = common_kind({centers, radii, out->label, out->count, out->min, out->softmin, out->cost,
                                  out->nbr, out->err});
    if (kind < 0) return fail(CSPLAT_E_INVALID, "eval: mix of host and device pointers");
    const char *bad_msg = "eval: query centres must be finite and radii finite and > 0";
    if (kind == 0 && !queries_valid_host(q, centers, radii)) return fail(CSPLAT_E_INVALID, bad_msg);
    DeviceGuard g(ctx->device);
    if (g.err != hipSuccess) return hip_fail(g.err, "hipSetDevice");
    reset_stats(ctx, q, sc);
    std::function<csplat_status()> gate;
    if (kind == 1) {
        // device inputs: checked on the device before any output is touched.
        // Both paths queue their sort and first pair pass (which write only
        // the workspace) before they wait for the check.
        auto check = [&](int *bad) {
            check_queries_kernel<<<(unsigned)((q + 255) / 256), 256, 0, ctx->stream>>>(q, centers, radii, bad);
        };
        s = queue_device_check(ctx, check);
        gate = [&]() { return wait_device_check(ctx, bad_msg); };
        if (s != CSPLAT_OK) return s;
    }
    s = on_device(ctx, kind, q, ctx->m, {centers, radii}, {(size_t)q * 12, (size_t)q * 4}, out,
                  [&](const std::vector<const void *> &in, const EvalOut &eo) {
                      const float *c = static_cast<const float *>(in[0]), *r = static_cast<const float *>(in[1]);
                      if (opts->precision != CSPLAT_PRECISION_FP32)
                          return precision_eval(ctx, sc, q, c, r, p, eo, opts->precision, gate);
                      return fp32_eval(ctx, sc, q, c, r, p, eo, !want_dist, false, gate);
                  });
    scene_note_use(sc, ctx->stream);
    return s;
}

csplat_status csplat_eval_ellipsoids(csplat_ctx *ctx, const csplat_scene *sc, int64_t q, const float *centers,
                                     const float *quats, const float *axes, const csplat_reduce_opts *opts,
                                     const csplat_outputs *out)
{
    EvalParams p;
    bool want_dist = false;
    csplat_status s = eval_checks(ctx, sc, q, opts, out, "eval_ellipsoids", p, want_dist);
    if (s != CSPLAT_OK) return s;
    if (opts->precision != CSPLAT_PRECISION_FP32) {
        if (out->min || out->softmin || out->cost || out->nbr || out->err)
            return fail(CSPLAT_E_INVALID, "eval_ellipsoids: the MFMA precision forms compute labels and counts only");
        if (std::isfinite(opts->neighbor_radius))
            return fail(CSPLAT_E_INVALID,
                        "eval_ellipsoids: the MFMA precision forms count over every kept Gaussian (neighbor_radius = +inf)");
        const void *f = opts->precision == CSPLAT_PRECISION_BF16_RECHECK ? sc->feat_ell_bf16 : sc->feat_ell_fp16;
        if (sc->n > 0 && !f)
            return fail(CSPLAT_E_INVALID,
                        "eval_ellipsoids: scene was loaded without the requested ellipsoid precision features");
    }
    if (q == 0) return CSPLAT_OK;
    if (!centers || !quats || !axes) return fail(CSPLAT_E_INVALID, "eval_ellipsoids: NULL body array");
    const int kind = common_kind({centers, quats, axes, out->label, out->count, out->min, out->softmin,
                                  out->cost, out->nbr});
    if (kind < 0) return fail(CSPLAT_E_INVALID, "eval_ellipsoids: mix of host and device pointers");
    const char *bad_msg =
        "eval_ellipsoids: centres must be finite, quaternions finite and nonzero, semi-axes finite and > 0";
    if (kind == 0 && !bodies_valid_host(q, centers, quats, axes)) return fail(CSPLAT_E_INVALID, bad_msg);
    DeviceGuard g(ctx->device);
    if (g.err != hipSuccess) return hip_fail(g.err, "hipSetDevice");
    reset_stats(ctx, q, sc);
    if (kind == 1) {
        s = device_check(
            ctx,
            [&](int *bad) {
                check_bodies_kernel<<<(unsigned)((q + 255) / 256), 256, 0, ctx->stream>>>(q, centers, quats, axes,
                                                                                       bad);
            },
            bad_msg);
        if (s != CSPLAT_OK) return s;
    }
    hipError_t e = ctx->bodies.reserve((size_t)q * kBodyFloats * 4);
    if (e != hipSuccess) return hip_fail(e, "body workspace");
    s = on_device(ctx, kind, q, ctx->m, {centers, quats, axes}, {(size_t)q * 12, (size_t)q * 16, (size_t)q * 12},
                  out, [&](const std::vector<const void *> &in, const EvalOut &eo) {
                      float *rec = ctx->bodies.as<float>();
                      csplat_status st = prepare_bodies(ctx, (int)q, static_cast<const float *>(in[0]),
                                                        static_cast<const float *>(in[1]),
                                                        static_cast<const float *>(in[2]), rec);
                      if (st != CSPLAT_OK) return st;
                      if (opts->precision != CSPLAT_PRECISION_FP32)
                          return precision_eval_ell(ctx, sc, q, rec, p, eo, opts->precision);
                      return fp32_eval(ctx, sc, q, rec, nullptr, p, eo, !want_dist, true);
                  });
    scene_note_use(sc, ctx->stream);
    return s;
}

csplat_status csplat_eval_labels(csplat_ctx *ctx, const csplat_scene *sc, int64_t q, const float *centers,
                                 const float *radii, const csplat_reduce_opts *opts, uint8_t *label,
                                 int32_t *count)
{
    if (!label) return fail(CSPLAT_E_INVALID, "eval_labels: label is NULL");
    csplat_outputs o{};
    o.label = label;
    o.count = count;
    return csplat_eval(ctx, sc, q, centers, radii, opts, &o);
}

csplat_status csplat_eval_distance(csplat_ctx *ctx, const csplat_scene *sc, int64_t q, const float *centers,
                                   const float *radii, const csplat_reduce_opts *opts, float *min,
                                   float *softmin, float *cost)
{
    if (!min) return fail(CSPLAT_E_INVALID, "eval_distance: min is NULL");
    csplat_outputs o{};
    o.min = min;
    o.softmin = softmin;
    o.cost = cost;
    return csplat_eval(ctx, sc, q, centers, radii, opts, &o);
}

csplat_status csplat_eval_noalloc(csplat_ctx *ctx, const csplat_scene *sc, int64_t q, const float *centers,
                                  const float *radii, const csplat_reduce_opts *opts, const csplat_outputs *out)
{
    EvalParams p;
    bool want_dist = false;
    csplat_status s = eval_checks(ctx, sc, q, opts, out, "eval_noalloc", p, want_dist);
    if (s != CSPLAT_OK) return s;
    if (opts->precision != CSPLAT_PRECISION_FP32)
        return fail(CSPLAT_E_INVALID, "eval_noalloc: the float32 path only");
    if (q > CSPLAT_NOALLOC_MAX_Q) return fail(CSPLAT_E_INVALID, "eval_noalloc: q above CSPLAT_NOALLOC_MAX_Q");
    if (q == 0) return CSPLAT_OK;
    if (!centers || !radii) return fail(CSPLAT_E_INVALID, "eval_noalloc: NULL centers or radii");
    const int kind = common_kind({centers, radii, out->label, out->count, out->min, out->softmin, out->cost,
                                  out->nbr});
    if (kind != 1) return fail(CSPLAT_E_INVALID, "eval_noalloc: every array must be a device pointer");
    if (!ctx->check_host || !ctx->ev_check) return fail(CSPLAT_E_DEVICE, "eval_noalloc: context without check flag");
    char *ws_base = static_cast<char *>(scratch_of(ctx->device));
    if (!ws_base) return fail(CSPLAT_E_DEVICE, "eval_noalloc: no scratch address for this device");
    DeviceGuard g(ctx->device);
    if (g.err != hipSuccess) return hip_fail(g.err, "hipSetDevice");
    reset_stats(ctx, q, sc);
    const char *bad_msg = "eval_noalloc: query centres must be finite and radii finite and > 0";
    s = queue_device_check(ctx, [&](int *bad) {
        check_queries_kernel<<<(unsigned)((q + 255) / 256), 256, 0, ctx->stream>>>(q, centers, radii, bad);
    });
    if (s != CSPLAT_OK) return s;
    const Workspace ws{ws_base, kScratchBytes};
    const EvalOut eo{out->label, out->count, out->min, out->softmin, out->cost, out->nbr, nullptr};
    s = fp32_eval(ctx, sc, q, centers, radii, p, eo, !want_dist, false,
                  [&]() { return wait_device_check(ctx, bad_msg); }, &ws);
    scene_note_use(sc, ctx->stream, false);
    return s;
}

csplat_status csplat_ctx_set_timing(csplat_ctx *ctx, int32_t enable)
{
    if (!ctx) return fail(CSPLAT_E_INVALID, "set_timing: NULL ctx");
    DeviceGuard g(ctx->device);
    if (enable && !ctx->ev0) {
        CSPLAT_HIP(hipEventCreate(&ctx->ev0));
        CSPLAT_HIP(hipEventCreate(&ctx->ev1));
    }
    ctx->timing = enable != 0;
    ctx->timed = false;
    return CSPLAT_OK;
}

csplat_status csplat_last_stats(csplat_ctx *ctx, csplat_eval_stats *stats)
{
    if (!ctx || !stats) return fail(CSPLAT_E_INVALID, "last_stats: NULL argument");
    *stats = ctx->stats;
    stats->kernel_ms = -1.f;
    stats->workspace_bytes = ctx->partial.bytes + ctx->staging.bytes + ctx->flags.bytes + ctx->sortbuf.bytes +
                             ctx->bodies.bytes + ctx->minbuf.bytes;
    if (ctx->chunk_counter) {  // culled evaluation: pairs the kernel actually evaluated
        DeviceGuard g(ctx->device);
        unsigned long long chunks = 0;
        CSPLAT_HIP(hipMemcpyAsync(&chunks, ctx->chunk_counter, sizeof(chunks), hipMemcpyDeviceToHost, ctx->stream));
        CSPLAT_HIP(hipStreamSynchronize(ctx->stream));
        stats->kernel_pairs = (int64_t)chunks * ctx->pairs_per_chunk;
    }
    if (ctx->flag_counts && ctx->flag_m > 0) {  // precision forms: rechecked queries
        DeviceGuard g(ctx->device);
        int32_t h[CSPLAT_MAX_M] = {0};
        CSPLAT_HIP(hipMemcpyAsync(h, ctx->flag_counts, sizeof(int32_t) * ctx->flag_m, hipMemcpyDeviceToHost,
                                  ctx->stream));
        CSPLAT_HIP(hipStreamSynchronize(ctx->stream));
        int64_t tot = 0;
        for (int v = 0; v < ctx->flag_m; ++v) tot += h[v];
        stats->flagged = tot;
        stats->flagged_fp64 = tot;
        ctx->stats.flagged = tot;
        ctx->stats.flagged_fp64 = tot;
    }
    if (ctx->timing && ctx->timed && ctx->timed_ms >= 0.f) {
        stats->kernel_ms = ctx->timed_ms;
    } else if (ctx->timing && ctx->timed) {
        DeviceGuard g(ctx->device);
        CSPLAT_HIP(hipEventSynchronize(ctx->ev1));
        float ms = 0.f;
        CSPLAT_HIP(hipEventElapsedTime(&ms, ctx->ev0, ctx->ev1));
        stats->kernel_ms = ms;
    }
    return CSPLAT_OK;
}

csplat_status csplat_last_rechecked(csplat_ctx *ctx, int32_t *idx, int64_t cap, int64_t *n)
{
    if (!ctx || !n || cap < 0 || (cap > 0 && !idx)) return fail(CSPLAT_E_INVALID, "last_rechecked: bad argument");
    *n = 0;
    if (!ctx->rk_list) return CSPLAT_OK;
    DeviceGuard g(ctx->device);
    int32_t nl = 0;
    CSPLAT_HIP(hipMemcpyAsync(&nl, ctx->rk_n, sizeof(int32_t), hipMemcpyDeviceToHost, ctx->stream));
    CSPLAT_HIP(hipStreamSynchronize(ctx->stream));
    *n = nl;
    const int64_t k = std::min<int64_t>(cap, nl);
    if (k == 0) return CSPLAT_OK;
    std::vector<int32_t> list((size_t)k), perm;
    CSPLAT_HIP(hipMemcpyAsync(list.data(), ctx->rk_list, (size_t)k * 4, hipMemcpyDeviceToHost, ctx->stream));
    if (ctx->rk_perm) {
        perm.resize((size_t)ctx->rk_q);
        CSPLAT_HIP(hipMemcpyAsync(perm.data(), ctx->rk_perm, (size_t)ctx->rk_q * 4, hipMemcpyDeviceToHost,
                                  ctx->stream));
    }
    CSPLAT_HIP(hipStreamSynchronize(ctx->stream));
    for (int64_t i = 0; i < k; ++i) idx[i] = ctx->rk_perm ? perm[(size_t)list[(size_t)i]] : list[(size_t)i];
    return CSPLAT_OK;
}

csplat_status csplat_synchronize(csplat_ctx *ctx)
{
    if (!ctx) return fail(CSPLAT_E_INVALID, "synchronize: NULL ctx");
    DeviceGuard g(ctx->device);
    CSPLAT_HIP(hipStreamSynchronize(ctx->stream));
    return CSPLAT_OK;
}

}  // extern "C"
