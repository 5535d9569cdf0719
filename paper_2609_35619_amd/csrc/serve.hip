// The serving form: resident scenes, admission by memory, continuous batching
// of work items into steps that are replays of a captured HIP graph.
//
// Per step the graph copies a staging area from pinned host memory (the
// descriptors of the active requests, the work items sorted by variant, the
// requests completing in this step), runs four persistent step kernels (one
// per (labels|full) x (ball|no ball) variant) that each walk their item
// range with the same per-tile code as csplat_eval, and a combine kernel
// that finalises the completing requests straight into pinned host memory.
// Two graph instances with their own staging areas alternate, so the worker
// thread prepares step k+1 while step k runs.
#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <thread>
#include <vector>

#include "pair_core.h"
#include "sched.h"

namespace csplat {
namespace {

using namespace pair;
using serve::Item;
using serve::ReqSpec;
using serve::Scheduler;
using serve::State;
using serve::StepPlan;

constexpr int kVariants = 8;        // bit 0: a ball; bit 1: full outputs; bit 2: ellipsoidal bodies
constexpr int kStepBlocks = 2048;   // persistent grid of each step kernel (8 blocks per CU)
constexpr int kMaxItems = 16384;    // work items per step
constexpr int kMaxSlots = 64;
constexpr int64_t kStepPairs = 40000000000LL;  // first step budget (dense pairs)
// The budget is steered toward kStepTargetMs of GPU time per step: culling
// makes a dense pair cost very different amounts of work from one request
// mix to the next, and steps much shorter than that are dominated by their
// fixed costs (staging, launch, host planning); much longer ones delay the
// small requests that share them.
constexpr double kStepTargetMs = 4.0;
constexpr int64_t kStepPairsMin = 1000000000LL, kStepPairsMax = 1000000000000000LL;

struct ReqDesc {
    const float *gs;
    const float *centers;
    const float *radii;
    int32_t n, per_split, S, q;
    int32_t G, parts;  // splits per work item, partial records per query
    int32_t full;
    const float *cull;  // the scene's culling chunks
    EvalParams p;
    Part part;
    EvalOut out;  // device-visible pointers into pinned host memory
};

struct StepHeader {
    int32_t begin[kVariants + 1];  // item range of each variant
    int32_t n_done;
    int32_t done[kMaxSlots];
    int32_t next[kVariants];       // work counters of the step kernels (zero in the staged copy)
};

inline size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

struct StageLayout {
    size_t desc, items, bytes;
    explicit StageLayout(int slots)
    {
        desc = align256(sizeof(StepHeader));
        items = desc + align256(sizeof(ReqDesc) * (size_t)slots);
        bytes = items + align256(sizeof(Item) * (size_t)kMaxItems);
    }
};

template <bool FULL, bool BALL, bool ELL>
__device__ __forceinline__ void step_body(const char *__restrict__ stage, int variant, size_t desc_off,
                                          size_t items_off, int32_t *__restrict__ next)
{
    // the staged step is read-only here (scalar loads); the work counter is
    // the header's next[variant], written only through `next`
    const StepHeader *h = reinterpret_cast<const StepHeader *>(stage);
    const ReqDesc *reqs = reinterpret_cast<const ReqDesc *>(stage + desc_off);
    const Item *items = reinterpret_cast<const Item *>(stage + items_off);
    const int b0 = h->begin[variant], b1 = h->begin[variant + 1];
    constexpr int QPL = FULL ? kQplFull : kQplLabels;
    constexpr bool CULL = !FULL || BALL;  // same bits as without culling
    // blocks take the variant's items in order from a shared counter, so a
    // block that drew cheap items goes on to the next one (items differ
    // widely in cost once culled)
    __shared__ int s_it;
    for (;;) {
        if (threadIdx.x == 0) s_it = b0 + atomicAdd(next, 1);
        __syncthreads();
        const int it = __builtin_amdgcn_readfirstlane(s_it);
        __syncthreads();
        if (it >= b1) break;
        const Item w = items[it];
        const ReqDesc &R = reqs[__builtin_amdgcn_readfirstlane(w.slot)];
        eval_tile<1, FULL, BALL, QPL, CULL, ELL>(R.gs, R.n, R.S, R.G, __builtin_amdgcn_readfirstlane(w.split),
                                            __builtin_amdgcn_readfirstlane(w.tile), R.centers, R.radii, R.q, R.p,
                                            R.part, R.cull, nullptr);
    }
}

template <bool FULL, bool BALL, bool ELL>
__global__ void __launch_bounds__(kBlock) CSPLAT_OCCUPANCY step_kernel(const char *__restrict__ stage, int variant,
                                                                          size_t desc_off, size_t items_off,
                                                                          int32_t *__restrict__ next)
{
    step_body<FULL, BALL, ELL>(stage, variant, desc_off, items_off, next);
}

// Full outputs over a ball (the task walk, eight-wave blocks; ellipsoids
// without it: the wave walk, kBlock), at its own occupancy target.
template <bool ELL>
constexpr int full_ball_block()
{
    return uses_tasks<true, true, 1, ELL>() ? kFullTaskBlock : kBlock;
}
template <bool ELL>
__global__ void __launch_bounds__(full_ball_block<ELL>())
__attribute__((amdgpu_waves_per_eu(task_waves_per_eu<1, true, ELL>())))
step_task_kernel(const char *__restrict__ stage, int variant, size_t desc_off, size_t items_off,
                 int32_t *__restrict__ next)
{
    step_body<true, true, ELL>(stage, variant, desc_off, items_off, next);
}

__global__ void __launch_bounds__(256) serve_combine_kernel(const char *__restrict__ stage, size_t desc_off)
{
    const StepHeader *h = reinterpret_cast<const StepHeader *>(stage);
    const ReqDesc *reqs = reinterpret_cast<const ReqDesc *>(stage + desc_off);
    for (int d = 0; d < h->n_done; ++d) {
        const ReqDesc &R = reqs[h->done[d]];
        for (int j = (int)(blockIdx.x * blockDim.x + threadIdx.x); j < R.q; j += (int)(gridDim.x * blockDim.x)) {
            if (R.full) combine_query<1, true>(j, R.q, R.parts, R.p, R.part, R.out);
            else combine_query<1, false>(j, R.q, R.parts, R.p, R.part, R.out);
        }
    }
}

double now_s()
{
    using namespace std::chrono;
    return duration<double>(steady_clock::now().time_since_epoch()).count();
}

// f(begin, end) over [0, n) on up to 16 host threads (one for small n).
template <class F>
void parallel_rows(size_t n, F f)
{
    const size_t kMinRows = 1 << 17;
    unsigned t = std::thread::hardware_concurrency();
    t = std::max(1u, std::min(t, 16u));
    if (n < 2 * kMinRows || t == 1) {
        f(0, n);
        return;
    }
    t = (unsigned)std::min<size_t>(t, n / kMinRows);
    std::vector<std::thread> pool;
    const size_t per = (n + t - 1) / t;
    for (unsigned k = 1; k < t; ++k) {
        const size_t b = k * per, e = std::min(n, b + per);
        if (b < e) pool.emplace_back([=, &f] { f(b, e); });
    }
    f(0, std::min(n, per));
    for (auto &th : pool) th.join();
}

struct Rec {
    int32_t scene = 0, kind = 0;
    int64_t q = 0;
    std::vector<float> centers, radii;  // until admission, in curve order
    std::vector<float> quats, axes;     // ellipsoidal bodies: orientation and semi-axes, the same order
    std::vector<int32_t> perm;          // curve position -> the caller's query index
    EvalParams p{};
    SplitPlan sp{};
    bool full = false, ball = false, ell = false;
    int64_t pairs = 0;
    // arena layout of the request (ellipsoids: the prepared body records at
    // d_centers, the raw bodies uploaded at d_raw)
    size_t d_centers = 0, d_raw = 0, d_part = 0;
    size_t h_in = 0, h_label = 0, h_count = 0, h_min = 0, h_soft = 0, h_cost = 0, h_nbr = 0;
};

}  // namespace
}  // namespace csplat

using namespace csplat;

struct csplat_server {
    int device = 0;
    int slots = 0;
    uint64_t budget = 0;
    hipStream_t stream = nullptr, copy_stream = nullptr;
    char *dev_arena = nullptr;
    char *host_arena = nullptr;      // pinned, device-mapped
    char *host_arena_dev = nullptr;  // its device address
    StageLayout layout{1};
    char *stage_host[2] = {nullptr, nullptr};
    char *stage_dev[2] = {nullptr, nullptr};
    hipGraphExec_t graph[2] = {nullptr, nullptr};
    hipEvent_t step_ev[2] = {nullptr, nullptr};
    hipEvent_t step_ev0[2] = {nullptr, nullptr};  // step starts (timing)
    hipEvent_t copy_ev = nullptr;
    bool copies_pending = false;
    std::vector<const csplat_scene *> scenes;
    Scheduler *sched = nullptr;
    std::map<int64_t, Rec> recs;
    std::vector<ReqDesc> desc;       // per slot
    std::vector<int64_t> slot_ticket;
    struct Inflight {
        int64_t step;
        int stage;
        bool full;  // the plan stopped at the budget (more work was waiting)
    };
    std::vector<Inflight> inflight;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::thread worker;
    bool stop = false;
    csplat_status fatal = CSPLAT_OK;
    std::string fatal_msg;
    // statistics
    csplat_serving_stats st{};
    std::vector<double> lat_ms;
    double first_admit = -1, last_done = -1;
    int64_t pairs_done = 0;
};

namespace csplat {
namespace {

void set_fatal(csplat_server *s, hipError_t e, const char *what)
{
    if (s->fatal == CSPLAT_OK) {
        s->fatal = e == hipErrorOutOfMemory ? CSPLAT_E_OOM : CSPLAT_E_DEVICE;
        s->fatal_msg = std::string("server: ") + what + ": " + hipGetErrorString(e);
    }
}

// Admitted request: upload its inputs (pinned staging -> device arena, on the
// copy stream) and write its descriptor.
void setup_request(csplat_server *s, int64_t t)
{
    const serve::ReqInfo *ri = s->sched->info(t);
    Rec &r = s->recs[t];
    const size_t qn = (size_t)r.q;
    char *hbase = s->host_arena + ri->host_off;
    char *dbase = s->dev_arena + ri->dev_off;
    if (!r.ell) {
        std::memcpy(hbase + r.h_in, r.centers.data(), qn * 12);
        std::memcpy(hbase + r.h_in + qn * 12, r.radii.data(), qn * 4);
        if (qn) {
            hipError_t e = hipMemcpyAsync(dbase + r.d_centers, hbase + r.h_in, qn * 16, hipMemcpyHostToDevice,
                                          s->copy_stream);
            if (e != hipSuccess) set_fatal(s, e, "input upload");
            s->copies_pending = true;
        }
    } else {
        // the raw bodies, then their records prepared on the device by the
        // kernel csplat_eval_ellipsoids uses (the same bits)
        std::memcpy(hbase + r.h_in, r.centers.data(), qn * 12);
        std::memcpy(hbase + r.h_in + qn * 12, r.quats.data(), qn * 16);
        std::memcpy(hbase + r.h_in + qn * 28, r.axes.data(), qn * 12);
        if (qn) {
            char *raw = dbase + r.d_raw;
            hipError_t e = hipMemcpyAsync(raw, hbase + r.h_in, qn * 40, hipMemcpyHostToDevice, s->copy_stream);
            if (e == hipSuccess)
                e = prepare_bodies_on(s->copy_stream, (int)qn, reinterpret_cast<const float *>(raw),
                                      reinterpret_cast<const float *>(raw + qn * 12),
                                      reinterpret_cast<const float *>(raw + qn * 28),
                                      reinterpret_cast<float *>(dbase + r.d_centers));
            if (e != hipSuccess) set_fatal(s, e, "input upload");
            s->copies_pending = true;
        }
    }
    std::vector<float>().swap(r.centers);
    std::vector<float>().swap(r.radii);
    std::vector<float>().swap(r.quats);
    std::vector<float>().swap(r.axes);
    const csplat_scene *sc = s->scenes[(size_t)r.scene];
    ReqDesc d{};
    d.gs = sc->gauss;
    d.centers = reinterpret_cast<const float *>(dbase + r.d_centers);
    d.radii = r.ell ? nullptr : reinterpret_cast<const float *>(dbase + r.d_centers + qn * 12);
    d.n = (int32_t)sc->n;
    d.per_split = r.sp.per_split;
    d.S = r.sp.S;
    d.G = r.sp.G;
    d.parts = r.sp.parts;  // 0 for an empty scene: the combine then folds nothing
    d.q = (int32_t)r.q;
    d.full = r.full ? 1 : 0;
    d.cull = sc->cull;
    d.p = r.p;
    d.part = part_views(dbase + r.d_part, std::max(d.parts, 1), (int)r.q, 1, r.full);
    char *hd = s->host_arena_dev + ri->host_off;
    d.out.label = reinterpret_cast<uint8_t *>(hd + r.h_label);
    d.out.count = reinterpret_cast<int32_t *>(hd + r.h_count);
    if (r.full) {
        d.out.min = reinterpret_cast<float *>(hd + r.h_min);
        d.out.softmin = reinterpret_cast<float *>(hd + r.h_soft);
        d.out.cost = reinterpret_cast<float *>(hd + r.h_cost);
        d.out.nbr = reinterpret_cast<int32_t *>(hd + r.h_nbr);
    }
    s->desc[(size_t)ri->slot] = d;
    s->slot_ticket[(size_t)ri->slot] = t;
    if (s->first_admit < 0) s->first_admit = now_s();
}

void launch_step(csplat_server *s, const StepPlan &plan)
{
    const int k = (int)(plan.step & 1);
    char *h = s->stage_host[k];
    StepHeader *hd = reinterpret_cast<StepHeader *>(h);
    std::memset(hd, 0, sizeof(StepHeader));
    int n = 0;
    for (int v = 0; v < kVariants; ++v) {
        hd->begin[v] = n;
        for (const Item &it : plan.items)
            if (it.variant == v) reinterpret_cast<Item *>(h + s->layout.items)[n++] = it;
    }
    hd->begin[kVariants] = n;
    hd->n_done = (int32_t)plan.completing.size();
    for (size_t i = 0; i < plan.completing.size(); ++i) hd->done[i] = plan.completing[i];
    std::memcpy(h + s->layout.desc, s->desc.data(), sizeof(ReqDesc) * (size_t)s->slots);
    hipError_t e = hipSuccess;
    if (s->copies_pending) {
        e = hipEventRecord(s->copy_ev, s->copy_stream);
        if (e == hipSuccess) e = hipStreamWaitEvent(s->stream, s->copy_ev, 0);
        s->copies_pending = false;
    }
    if (e == hipSuccess) e = hipEventRecord(s->step_ev0[k], s->stream);
    if (e == hipSuccess) e = hipGraphLaunch(s->graph[k], s->stream);
    if (e == hipSuccess) e = hipEventRecord(s->step_ev[k], s->stream);
    if (e != hipSuccess) {
        set_fatal(s, e, "step launch");
        return;
    }
    s->inflight.push_back({plan.step, k, plan.pairs >= s->sched->step_pairs()});
    ++s->st.steps;
    // how many requests the step serves together (continuous batching)
    int32_t reqs = 0;
    std::vector<int32_t> seen;
    for (const Item &it : plan.items)
        if (std::find(seen.begin(), seen.end(), it.slot) == seen.end()) seen.push_back(it.slot);
    reqs = (int32_t)seen.size();
    if (reqs >= 2) ++s->st.shared_steps;
    s->st.max_requests_per_step = std::max(s->st.max_requests_per_step, reqs);
}

void worker_main(csplat_server *s)
{
    (void)hipSetDevice(s->device);
    std::unique_lock<std::mutex> lk(s->mu);
    for (;;) {
        bool progressed = false;
        // completed steps, oldest first
        while (!s->inflight.empty()) {
            hipError_t q = hipEventQuery(s->step_ev[s->inflight.front().stage]);
            if (q == hipErrorNotReady) break;
            if (q != hipSuccess) {
                set_fatal(s, q, "step execution");
                (void)hipGetLastError();
            }
            const double t = now_s();
            {
                // steer the step budget toward kStepTargetMs (full steps only)
                const auto &f = s->inflight.front();
                float ms = 0.f;
                if (f.full && hipEventElapsedTime(&ms, s->step_ev0[f.stage], s->step_ev[f.stage]) == hipSuccess &&
                    ms > 0.f) {
                    const double scale = std::min(2.0, std::max(0.5, kStepTargetMs / ms));
                    const double b = (double)s->sched->step_pairs() * scale;
                    s->sched->set_step_pairs(
                        (int64_t)std::min((double)kStepPairsMax, std::max((double)kStepPairsMin, b)));
                }
            }
            for (int64_t tk : s->sched->step_done(s->inflight.front().step, t)) {
                const serve::ReqInfo *ri = s->sched->info(tk);
                if (ri && ri->state == State::Done) {
                    s->lat_ms.push_back((ri->t_done - ri->t_submit) * 1e3);
                    s->pairs_done += s->recs[tk].pairs;
                    s->last_done = t;
                    ++s->st.completed;
                } else if (ri && ri->state == State::Cancelled) {
                    ++s->st.cancelled;
                }
            }
            s->inflight.erase(s->inflight.begin());
            s->cv_done.notify_all();
            progressed = true;
        }
        if (s->fatal != CSPLAT_OK) {
            s->cv_done.notify_all();
            if (s->stop && s->inflight.empty()) break;
        }
        if (s->stop && s->inflight.empty()) break;
        if (!s->stop && s->fatal == CSPLAT_OK) {
            for (int64_t tk : s->sched->admit(now_s())) {
                setup_request(s, tk);
                progressed = true;
            }
            if (s->inflight.size() < 2) {
                StepPlan plan;
                if (s->sched->plan(&plan)) {
                    launch_step(s, plan);
                    progressed = true;
                }
            }
        }
        if (!progressed) {
            // nothing to do right now: sleep briefly (woken early by submit/cancel/stop)
            s->cv_work.wait_for(lk, std::chrono::microseconds(s->inflight.empty() ? 2000 : 50));
        }
    }
}

csplat_status capture_graphs(csplat_server *s)
{
    for (int k = 0; k < 2; ++k) {
        hipGraph_t g = nullptr;
        CSPLAT_HIP(hipStreamBeginCapture(s->stream, hipStreamCaptureModeThreadLocal));
        hipError_t e = hipMemcpyAsync(s->stage_dev[k], s->stage_host[k], s->layout.bytes, hipMemcpyHostToDevice,
                                      s->stream);
        const char *st = s->stage_dev[k];
        int32_t *ctr = reinterpret_cast<StepHeader *>(s->stage_dev[k])->next;
        const size_t dof = s->layout.desc, iof = s->layout.items;
        if (e == hipSuccess) {
            step_kernel<false, false, false><<<kStepBlocks, kBlock, 0, s->stream>>>(st, 0, dof, iof, ctr + 0);
            step_kernel<false, true, false><<<kStepBlocks, kBlock, 0, s->stream>>>(st, 1, dof, iof, ctr + 1);
            step_kernel<true, false, false><<<kStepBlocks, kBlock, 0, s->stream>>>(st, 2, dof, iof, ctr + 2);
            step_task_kernel<false><<<kStepBlocks, full_ball_block<false>(), 0, s->stream>>>(st, 3, dof, iof, ctr + 3);
            step_kernel<false, false, true><<<kStepBlocks, kBlock, 0, s->stream>>>(st, 4, dof, iof, ctr + 4);
            step_kernel<false, true, true><<<kStepBlocks, kBlock, 0, s->stream>>>(st, 5, dof, iof, ctr + 5);
            step_kernel<true, false, true><<<kStepBlocks, kBlock, 0, s->stream>>>(st, 6, dof, iof, ctr + 6);
            step_task_kernel<true><<<kStepBlocks, full_ball_block<true>(), 0, s->stream>>>(st, 7, dof, iof, ctr + 7);
            serve_combine_kernel<<<1024, 256, 0, s->stream>>>(st, dof);
            e = hipGetLastError();
        }
        hipError_t e2 = hipStreamEndCapture(s->stream, &g);
        if (e != hipSuccess) return hip_fail(e, "graph capture");
        if (e2 != hipSuccess) return hip_fail(e2, "graph capture end");
        e = hipGraphInstantiate(&s->graph[k], g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (e != hipSuccess) return hip_fail(e, "graph instantiate");
    }
    return CSPLAT_OK;
}

void server_release(csplat_server *s)
{
    for (int k = 0; k < 2; ++k) {
        if (s->graph[k]) (void)hipGraphExecDestroy(s->graph[k]);
        if (s->step_ev[k]) (void)hipEventDestroy(s->step_ev[k]);
        if (s->step_ev0[k]) (void)hipEventDestroy(s->step_ev0[k]);
        if (s->stage_host[k]) (void)hipHostFree(s->stage_host[k]);
        if (s->stage_dev[k]) (void)hipFree(s->stage_dev[k]);
    }
    if (s->copy_ev) (void)hipEventDestroy(s->copy_ev);
    if (s->dev_arena) (void)hipFree(s->dev_arena);
    if (s->host_arena) (void)hipHostFree(s->host_arena);
    if (s->stream) (void)hipStreamDestroy(s->stream);
    if (s->copy_stream) (void)hipStreamDestroy(s->copy_stream);
    delete s->sched;
}

}  // namespace
}  // namespace csplat

extern "C" {

csplat_status csplat_server_create(int32_t device, uint64_t hbm_budget, int32_t slots, csplat_server **out)
{
    if (!out) return fail(CSPLAT_E_INVALID, "server_create: out is NULL");
    *out = nullptr;
    if (slots < 1 || slots > kMaxSlots) return fail(CSPLAT_E_INVALID, "server_create: slots must be in 1..64");
    if (hbm_budget < (1u << 20)) return fail(CSPLAT_E_INVALID, "server_create: budget below 1 MiB");
    int ndev = 0;
    CSPLAT_HIP(hipGetDeviceCount(&ndev));
    if (device < 0 || device >= ndev) return fail(CSPLAT_E_INVALID, "server_create: no such device");
    DeviceGuard g(device);
    if (g.err != hipSuccess) return hip_fail(g.err, "hipSetDevice");
    csplat_server *s = new (std::nothrow) csplat_server();
    if (!s) return fail(CSPLAT_E_OOM, "server_create: host allocation");
    s->device = device;
    s->slots = slots;
    s->budget = hbm_budget;
    s->layout = StageLayout(slots);
    s->desc.assign((size_t)slots, ReqDesc{});
    s->slot_ticket.assign((size_t)slots, 0);
    hipError_t e = hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&s->copy_stream, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void **>(&s->dev_arena), hbm_budget);
    if (e == hipSuccess)
        e = hipHostMalloc(reinterpret_cast<void **>(&s->host_arena), hbm_budget, hipHostMallocMapped);
    if (e == hipSuccess) e = hipHostGetDevicePointer(reinterpret_cast<void **>(&s->host_arena_dev), s->host_arena, 0);
    for (int k = 0; k < 2 && e == hipSuccess; ++k) {
        e = hipHostMalloc(reinterpret_cast<void **>(&s->stage_host[k]), s->layout.bytes, hipHostMallocDefault);
        if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void **>(&s->stage_dev[k]), s->layout.bytes);
        if (e == hipSuccess) {
            std::memset(s->stage_host[k], 0, s->layout.bytes);
            e = hipEventCreate(&s->step_ev[k]);
            if (e == hipSuccess) e = hipEventCreate(&s->step_ev0[k]);
        }
    }
    if (e == hipSuccess) e = hipEventCreateWithFlags(&s->copy_ev, hipEventDisableTiming);
    if (e != hipSuccess) {
        csplat_status st = hip_fail(e, "server_create");
        server_release(s);
        delete s;
        return st;
    }
    csplat_status st = capture_graphs(s);
    if (st != CSPLAT_OK) {
        server_release(s);
        delete s;
        return st;
    }
    s->sched = new Scheduler(hbm_budget, hbm_budget, slots, kStepPairs, kMaxItems);
    s->sched->set_min_items(kStepBlocks);
    s->worker = std::thread(worker_main, s);
    *out = s;
    return CSPLAT_OK;
}

csplat_status csplat_server_destroy(csplat_server *s)
{
    if (!s) return CSPLAT_OK;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
    }
    s->cv_work.notify_all();
    if (s->worker.joinable()) s->worker.join();
    DeviceGuard g(s->device);
    (void)hipStreamSynchronize(s->stream);
    (void)hipStreamSynchronize(s->copy_stream);
    server_release(s);
    delete s;
    return CSPLAT_OK;
}

csplat_status csplat_server_add_scene(csplat_server *s, const csplat_scene *sc, int32_t *scene_id)
{
    if (!s || !sc || !scene_id) return fail(CSPLAT_E_INVALID, "server_add_scene: NULL argument");
    if (sc->device != s->device) return fail(CSPLAT_E_INVALID, "server_add_scene: scene on another device");
    std::lock_guard<std::mutex> lk(s->mu);
    s->scenes.push_back(sc);
    *scene_id = (int32_t)s->scenes.size() - 1;
    return CSPLAT_OK;
}

// Spheres (centres, radii) or, with quats, ellipsoidal bodies (centres,
// quats, axes); host arrays.
static csplat_status submit_impl(csplat_server *s, int32_t scene_id, int32_t kind, int64_t q, const float *centers,
                                 const float *radii, const float *quats, const float *axes,
                                 const csplat_reduce_opts *opts, const float *n_sigma, int32_t m, uint64_t *ticket)
{
    // latency counts from entry: validation, the host-side sort and the copy
    // below are part of what the caller waits for
    const double t_entry = now_s();
    const bool ell = quats != nullptr;
    if (!s || !opts || !n_sigma || !ticket) return fail(CSPLAT_E_INVALID, "server_submit: NULL argument");
    *ticket = 0;
    if (kind != CSPLAT_SERVE_COST && kind != CSPLAT_SERVE_LABELS)
        return fail(CSPLAT_E_INVALID, "server_submit: unknown kind");
    if (m != 1) return fail(CSPLAT_E_INVALID, "server_submit: one conservatism value per request (m = 1)");
    if (!(n_sigma[0] >= 0.f) || !std::isfinite(n_sigma[0]))
        return fail(CSPLAT_E_INVALID, "server_submit: n_sigma must be finite and >= 0");
    if (opts->precision != CSPLAT_PRECISION_FP32)
        return fail(CSPLAT_E_INVALID, "server_submit: the serving form evaluates in float32");
    if (q < 0 || q > (int64_t)0x7FFFFFFF / 8) return fail(CSPLAT_E_INVALID, "server_submit: q out of range");
    if (!ell) {
        if (q > 0 && (!centers || !radii)) return fail(CSPLAT_E_INVALID, "server_submit: NULL centers or radii");
        if (q > 0 && (pointer_kind(centers) || pointer_kind(radii)))
            return fail(CSPLAT_E_INVALID, "server_submit: inputs must be host pointers");
        for (int64_t j = 0; j < q; ++j) {
            if (!std::isfinite(centers[3 * j]) || !std::isfinite(centers[3 * j + 1]) ||
                !std::isfinite(centers[3 * j + 2]) || !(radii[j] > 0.f) || !std::isfinite(radii[j]))
                return fail(CSPLAT_E_INVALID, "server_submit: query centres must be finite and radii finite and > 0");
        }
    } else {
        if (q > 0 && (!centers || !axes)) return fail(CSPLAT_E_INVALID, "server_submit_ellipsoids: NULL body array");
        if (q > 0 && (pointer_kind(centers) || pointer_kind(quats) || pointer_kind(axes)))
            return fail(CSPLAT_E_INVALID, "server_submit_ellipsoids: inputs must be host pointers");
        if (!bodies_valid_host(q, centers, quats, axes))
            return fail(CSPLAT_E_INVALID, "server_submit_ellipsoids: centres must be finite, quaternions finite and "
                                          "nonzero, semi-axes finite and > 0");
    }
    Rec r;
    csplat_status st = build_params(n_sigma, 1, *opts, r.p);
    if (st != CSPLAT_OK) return st;
    const csplat_scene *sc = nullptr;
    {
        // resident scenes stay until the server is destroyed: the pointer
        // and the scene's grid are read without the lock below
        std::lock_guard<std::mutex> g(s->mu);
        if (s->fatal != CSPLAT_OK) return fail(s->fatal, s->fatal_msg);
        if (scene_id < 0 || scene_id >= (int32_t)s->scenes.size())
            return fail(CSPLAT_E_NOT_FOUND, "server_submit: unknown scene id");
        sc = s->scenes[(size_t)scene_id];
    }
    r.scene = scene_id;
    r.kind = kind;
    r.q = q;
    r.full = kind == CSPLAT_SERVE_COST;
    r.ball = std::isfinite(r.p.rn2);
    r.ell = ell;
    r.sp = split_plan(target_blocks(s->device), (int)q, (int)sc->n, r.full, r.ball, ell);
    r.pairs = q * sc->n;
    // the queries in the scene's Hilbert order (as csplat_eval evaluates
    // them): waves hold nearby spheres and the culling skips more; results
    // go back to the caller's order when collected
    // (key << 32 | index) words: keys and the gather on several host threads
    // for large requests, a stable LSD radix sort on the 30 key bits (the
    // same order as sorting (key, index) pairs)
    {
        const size_t qn = (size_t)q;
        std::vector<uint64_t> a(qn), b(qn);
        parallel_rows(qn, [&](size_t j0, size_t j1) {
            for (size_t j = j0; j < j1; ++j) {
                uint32_t ix[3];
                for (int k = 0; k < 3; ++k) {
                    const float f = (centers[3 * j + k] - sc->box_lo[k]) * sc->box_scale[k];
                    ix[k] = (uint32_t)std::min(std::max(f, 0.f), 1023.f);
                }
                a[j] = ((uint64_t)hilbert_key_branchless(ix[0], ix[1], ix[2]) << 32) | (uint64_t)j;
            }
        });
        for (int pass = 0; pass < 3; ++pass) {
            const int sh = 32 + 10 * pass;
            std::vector<size_t> pos(1025, 0);
            for (size_t j = 0; j < qn; ++j) ++pos[((a[j] >> sh) & 1023u) + 1];
            for (int d = 0; d < 1024; ++d) pos[d + 1] += pos[d];
            for (size_t j = 0; j < qn; ++j) b[pos[(a[j] >> sh) & 1023u]++] = a[j];
            a.swap(b);
        }
        r.perm.resize(qn);
        r.centers.resize(qn * 3);
        if (ell) {
            r.quats.resize(qn * 4);
            r.axes.resize(qn * 3);
        } else {
            r.radii.resize(qn);
        }
        parallel_rows(qn, [&](size_t j0, size_t j1) {
            for (size_t j = j0; j < j1; ++j) {
                const int32_t i = (int32_t)(a[j] & 0xffffffffu);
                r.perm[j] = i;
                for (int k = 0; k < 3; ++k) r.centers[3 * j + k] = centers[3 * (size_t)i + k];
                if (ell) {
                    for (int k = 0; k < 4; ++k) r.quats[4 * j + k] = quats[4 * (size_t)i + k];
                    for (int k = 0; k < 3; ++k) r.axes[3 * j + k] = axes[3 * (size_t)i + k];
                } else {
                    r.radii[j] = radii[i];
                }
            }
        });
    }
    const size_t qn = (size_t)q;
    const int parts = std::max(r.sp.parts, 1);
    // device arena: inputs (ellipsoids: records, then the raw bodies), then
    // partial reductions
    r.d_centers = 0;
    r.d_raw = ell ? align256(qn * kBodyFloats * 4) : 0;
    r.d_part = ell ? r.d_raw + align256(qn * 40) : align256(qn * 16);
    const uint64_t dev_bytes = r.d_part + align256((size_t)parts * qn * part_words(1, r.full) * 4);
    // pinned host arena: input staging, then outputs
    size_t off = 0;
    auto take = [&](size_t b) {
        size_t o = off;
        off += align256(b);
        return o;
    };
    r.h_in = take(qn * (ell ? 40 : 16));
    r.h_label = take(qn);
    r.h_count = take(qn * 4);
    if (r.full) {
        r.h_min = take(qn * 4);
        r.h_soft = take(qn * 4);
        r.h_cost = take(qn * 4);
        r.h_nbr = take(qn * 4);
    }
    ReqSpec spec;
    spec.tiles = r.sp.n_tiles;
    spec.splits = parts;  // work items per tile
    spec.variant = (ell ? 4 : 0) + (r.full ? 2 : 0) + (r.ball ? 1 : 0);
    spec.item_pairs = (int64_t)r.sp.block * r.sp.qpl * r.sp.per_split;
    spec.dev_bytes = dev_bytes;
    spec.host_bytes = off;
    // the sort above ran without the lock (the worker keeps scheduling)
    std::unique_lock<std::mutex> lk(s->mu);
    if (s->fatal != CSPLAT_OK) return fail(s->fatal, s->fatal_msg);
    const int64_t t = s->sched->submit(spec, t_entry);
    if (t < 0) {
        ++s->st.refused;
        return fail(CSPLAT_E_BUSY, "server_submit: the request can never fit the memory budget");
    }
    s->recs[t] = std::move(r);
    ++s->st.submitted;
    *ticket = (uint64_t)t;
    lk.unlock();
    s->cv_work.notify_all();
    return CSPLAT_OK;
}

csplat_status csplat_server_submit(csplat_server *s, int32_t scene_id, int32_t kind, int64_t q,
                                   const float *centers, const float *radii, const csplat_reduce_opts *opts,
                                   const float *n_sigma, int32_t m, uint64_t *ticket)
{
    return submit_impl(s, scene_id, kind, q, centers, radii, nullptr, nullptr, opts, n_sigma, m, ticket);
}

csplat_status csplat_server_submit_ellipsoids(csplat_server *s, int32_t scene_id, int32_t kind, int64_t q,
                                              const float *centers, const float *quats, const float *axes,
                                              const csplat_reduce_opts *opts, const float *n_sigma, int32_t m,
                                              uint64_t *ticket)
{
    if (q > 0 && !quats) return fail(CSPLAT_E_INVALID, "server_submit_ellipsoids: NULL quaternions");
    static const float kNoBody[4] = {1.f, 0.f, 0.f, 0.f};
    return submit_impl(s, scene_id, kind, q, centers, nullptr, quats ? quats : kNoBody, axes, opts, n_sigma, m,
                       ticket);
}

static csplat_status collect(csplat_server *s, int64_t t, const csplat_outputs *out)
{
    // caller holds the lock; the request is Done
    const serve::ReqInfo *ri = s->sched->info(t);
    const Rec &r = s->recs[t];
    const char *h = s->host_arena + ri->host_off;
    const size_t qn = (size_t)r.q;
    if (out) {
        // back to the caller's query order
        auto scatter = [&](void *dst, size_t off, size_t elem) {
            if (!dst) return;
            char *d = static_cast<char *>(dst);
            const char *src = h + off;
            parallel_rows(qn, [&](size_t j0, size_t j1) {
                for (size_t j = j0; j < j1; ++j) std::memcpy(d + (size_t)r.perm[j] * elem, src + j * elem, elem);
            });
        };
        scatter(out->label, r.h_label, 1);
        scatter(out->count, r.h_count, 4);
        if (r.full) {
            scatter(out->min, r.h_min, 4);
            scatter(out->softmin, r.h_soft, 4);
            scatter(out->cost, r.h_cost, 4);
            scatter(out->nbr, r.h_nbr, 4);
        }
    }
    s->sched->finish(t);
    s->recs.erase(t);
    return CSPLAT_OK;
}

static csplat_status poll_locked(csplat_server *s, int64_t t, const csplat_outputs *out)
{
    const serve::ReqInfo *ri = s->sched->info(t);
    if (!ri) return fail(CSPLAT_E_NOT_FOUND, "server: unknown ticket");
    if (ri->state == State::Done) return collect(s, t, out);
    if (ri->state == State::Cancelled) {
        s->sched->finish(t);
        s->recs.erase(t);
        return fail(CSPLAT_E_CANCELLED, "server: the request was cancelled");
    }
    if (s->fatal != CSPLAT_OK) return fail(s->fatal, s->fatal_msg);
    return CSPLAT_E_PENDING;
}

csplat_status csplat_server_poll(csplat_server *s, uint64_t ticket, const csplat_outputs *out)
{
    if (!s) return fail(CSPLAT_E_INVALID, "server_poll: NULL server");
    std::lock_guard<std::mutex> lk(s->mu);
    return poll_locked(s, (int64_t)ticket, out);
}

csplat_status csplat_server_wait(csplat_server *s, uint64_t ticket, const csplat_outputs *out, int64_t timeout_ms)
{
    if (!s) return fail(CSPLAT_E_INVALID, "server_wait: NULL server");
    std::unique_lock<std::mutex> lk(s->mu);
    const auto t_end = std::chrono::steady_clock::now() + std::chrono::milliseconds(timeout_ms < 0 ? 0 : timeout_ms);
    for (;;) {
        csplat_status st = poll_locked(s, (int64_t)ticket, out);
        if (st != CSPLAT_E_PENDING) return st;
        if (timeout_ms < 0) {
            s->cv_done.wait_for(lk, std::chrono::milliseconds(100));
        } else {
            if (std::chrono::steady_clock::now() >= t_end) return CSPLAT_E_PENDING;
            s->cv_done.wait_until(lk, std::min(t_end, std::chrono::steady_clock::now() + std::chrono::milliseconds(100)));
        }
    }
}

csplat_status csplat_server_cancel(csplat_server *s, uint64_t ticket)
{
    if (!s) return fail(CSPLAT_E_INVALID, "server_cancel: NULL server");
    std::lock_guard<std::mutex> lk(s->mu);
    const serve::ReqInfo *ri = s->sched->info((int64_t)ticket);
    if (!ri || (ri->state != State::Queued && ri->state != State::Active))
        return fail(CSPLAT_E_NOT_FOUND, "server_cancel: unknown or finished ticket");
    const bool was_queued = ri->state == State::Queued;
    s->sched->cancel((int64_t)ticket, now_s());
    if (was_queued) ++s->st.cancelled;
    else if (s->sched->info((int64_t)ticket)->state == State::Cancelled) ++s->st.cancelled;
    s->cv_work.notify_all();
    s->cv_done.notify_all();
    return CSPLAT_OK;
}

csplat_status csplat_server_stats(csplat_server *s, csplat_serving_stats *out)
{
    if (!s || !out) return fail(CSPLAT_E_INVALID, "server_stats: NULL argument");
    std::lock_guard<std::mutex> lk(s->mu);
    *out = s->st;
    std::vector<double> v = s->lat_ms;
    if (!v.empty()) {
        std::sort(v.begin(), v.end());
        auto pct = [&](double p) {
            double idx = p * (double)(v.size() - 1);
            size_t lo = (size_t)idx;
            size_t hi = std::min(lo + 1, v.size() - 1);
            return v[lo] + (v[hi] - v[lo]) * (idx - (double)lo);
        };
        out->p50_ms = pct(0.50);
        out->p99_ms = pct(0.99);
        double sum = 0;
        for (double x : v) sum += x;
        out->mean_ms = sum / (double)v.size();
        out->max_ms = v.back();
    }
    if (s->first_admit >= 0 && s->last_done > s->first_admit) {
        out->busy_s = s->last_done - s->first_admit;
        out->pairs_per_s = (double)s->pairs_done / out->busy_s;
    }
    return CSPLAT_OK;
}

csplat_status csplat_server_latencies(csplat_server *s, double *ms, int64_t cap, int64_t *n)
{
    if (!s || !n || cap < 0 || (cap > 0 && !ms)) return fail(CSPLAT_E_INVALID, "server_latencies: bad argument");
    std::lock_guard<std::mutex> lk(s->mu);
    const int64_t have = (int64_t)s->lat_ms.size();
    std::copy(s->lat_ms.begin(), s->lat_ms.begin() + std::min(cap, have), ms);
    *n = have;
    return CSPLAT_OK;
}

}  // extern "C"
