// Internal declarations shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <functional>
#include <mutex>
#include <utility>
#include <vector>
#include <string>

#include "../../include/csplat.h"

namespace csplat {

// Per-Gaussian record of the float32 pair kernel: 12 floats (48 B, three
// float4s).  M = diag(s) R^T, so that for d = mu - c the linearised variance
// term V = d^T Sigma d = |M d|^2 is a sum of squares.
#ifndef CSPLAT_GAUSS_FLOATS
#define CSPLAT_GAUSS_FLOATS 12
#endif
constexpr int kGaussFloats = CSPLAT_GAUSS_FLOATS;  // mx my mz | M00..M22 (row-major) [| padding]
static_assert(kGaussFloats == 12 || kGaussFloats == 16, "records are three float4s, or four");
// Position of an integer cell (10 bits per axis) along a 3-D Hilbert curve
// (30-bit key), by Skilling's transform of the axes to the transposed index
// ("Programming the Hilbert curve", 2004) followed by bit interleaving.
// Consecutive keys are face-adjacent cells, so runs of the sorted order are
// compact in space (the culling chunks of the scene, the query groups of a
// wave).
__host__ __device__ inline uint32_t hilbert_key(uint32_t x, uint32_t y, uint32_t z)
{
    uint32_t X[3] = {x & 1023u, y & 1023u, z & 1023u};
    for (uint32_t Q = 512u; Q > 1u; Q >>= 1) {
        const uint32_t P = Q - 1u;
        for (int i = 0; i < 3; ++i) {
            if (X[i] & Q) {
                X[0] ^= P;  // invert
            } else {       // exchange the low bits of X[0] and X[i]
                const uint32_t t = (X[0] ^ X[i]) & P;
                X[0] ^= t;
                X[i] ^= t;
            }
        }
    }
    X[1] ^= X[0];  // Gray encode
    X[2] ^= X[1];
    uint32_t t = 0;
    for (uint32_t Q = 512u; Q > 1u; Q >>= 1)
        if (X[2] & Q) t ^= Q - 1u;
    X[0] ^= t;
    X[1] ^= t;
    X[2] ^= t;
    uint32_t key = 0;
    for (int b = 9; b >= 0; --b)
        key = (key << 3) | (((X[0] >> b) & 1u) << 2) | (((X[1] >> b) & 1u) << 1) | ((X[2] >> b) & 1u);
    return key;
}

// The same key without data-dependent branches (host side: the serving form
// sorts each request's spheres on the host, millions at a time).
inline uint32_t spread3_10(uint32_t v)  // bit i of v to bit 3i
{
    v &= 1023u;
    v = (v | (v << 16)) & 0x030000FFu;
    v = (v | (v << 8)) & 0x0300F00Fu;
    v = (v | (v << 4)) & 0x030C30C3u;
    v = (v | (v << 2)) & 0x09249249u;
    return v;
}

inline uint32_t hilbert_key_branchless(uint32_t x, uint32_t y, uint32_t z)
{
    uint32_t X[3] = {x & 1023u, y & 1023u, z & 1023u};
    for (uint32_t Q = 512u; Q > 1u; Q >>= 1) {
        const uint32_t P = Q - 1u;
        for (int i = 0; i < 3; ++i) {
            const uint32_t set = 0u - ((X[i] & Q) != 0u);        // all ones when bit Q of X[i] is set
            const uint32_t t = (X[0] ^ X[i]) & P & ~set;         // exchange otherwise
            X[0] ^= (P & set) ^ t;
            X[i] ^= t;
        }
    }
    X[1] ^= X[0];
    X[2] ^= X[1];
    // t = XOR of (Q - 1) over the set bits Q > 1 of X[2]: bit j of t is the
    // parity of X[2]'s bits above j
    uint32_t t = 0;
    for (int b = 9; b >= 1; --b) t ^= (0u - ((X[2] >> b) & 1u)) & ((1u << b) - 1u);
    X[0] ^= t;
    X[1] ^= t;
    X[2] ^= t;
    return (spread3_10(X[0]) << 2) | (spread3_10(X[1]) << 1) | spread3_10(X[2]);
}

// Prepared ellipsoidal body: centre (3), L = diag(1/a) R^T row-major (9), the
// reach constants qa = (smallest semi-axis)^2 and qk = largest / smallest, 0, 0.
constexpr int kBodyFloats = 16;

void set_error(const std::string &msg);
csplat_status fail(csplat_status code, const std::string &msg);
csplat_status hip_fail(hipError_t e, const char *what);

#define CSPLAT_HIP(call)                                      \
    do {                                                      \
        hipError_t e_ = (call);                               \
        if (e_ != hipSuccess) return ::csplat::hip_fail(e_, #call); \
    } while (0)

// Set a device as current for the duration of a scope.
struct DeviceGuard {
    int prev = -1;
    hipError_t err = hipSuccess;
    explicit DeviceGuard(int dev)
    {
        if (hipGetDevice(&prev) != hipSuccess) prev = -1;
        if (prev != dev) err = hipSetDevice(dev);
    }
    ~DeviceGuard()
    {
        if (prev >= 0) (void)hipSetDevice(prev);
    }
};

// A device buffer that grows on demand (never shrinks until freed).
// A growable device buffer, allocated and freed in the order of its owner's
// stream (stream-ordered allocation): growing it waits for nothing, the old
// block is released once the stream's earlier work is done.
struct DevBuf {
    void *ptr = nullptr;
    size_t bytes = 0;
    hipStream_t stream = nullptr;  // the owner's stream (set before the first reserve)
    hipError_t reserve(size_t want);
    void release();
    template <class T> T *as() const { return static_cast<T *>(ptr); }
};

}  // namespace csplat

struct csplat_scene {
    int device = 0;
    int64_t n_input = 0;
    int64_t n = 0;            // kept Gaussians
    float *gauss = nullptr;   // 12-float records in Hilbert order of the means, padded to whole
                              // culling chunks of 64 (pad records: mean at +inf, zero covariance)
    float mu_max = 0.f;       // max |mu| over the kept Gaussians
    float *cull = nullptr;    // per chunk of 64, then per sub-chunk of 16 (from record ceil(n / 64)),
                              // then per group of 1024 (from record ceil(n / 64) + ceil(n / 16)):
                              // bounding sphere centre, radius, largest scale (8 floats each)
    float box_lo[3] = {0, 0, 0}, box_scale[3] = {0, 0, 0};  // grid of the kept means (one cell size)
    // precision form (optional): per tile of 512 Gaussians the packed MFMA
    // operands (96 B per Gaussian) and 20 floats of metadata (origin, scale,
    // coefficient maxima), one set per dtype
    int64_t n_tiles = 0;
    void *feat_bf16 = nullptr;
    float *meta_bf16 = nullptr;
    void *feat_fp16 = nullptr;
    float *meta_fp16 = nullptr;
    // the same for ellipsoidal bodies (320 B per Gaussian, 24 floats per tile)
    void *feat_ell_bf16 = nullptr;
    float *meta_ell_bf16 = nullptr;
    void *feat_ell_fp16 = nullptr;
    float *meta_ell_fp16 = nullptr;
    uint64_t device_bytes = 0;
    // streams that read the scene, each with an event recorded after its
    // last use: freeing the scene waits for those events only (in stream
    // order, without blocking the host or other streams)
    mutable std::mutex use_mu;
    mutable std::vector<std::pair<hipStream_t, hipEvent_t>> uses;
};

struct csplat_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    int32_t m = 1;
    float n_sigma[CSPLAT_MAX_M] = {1.0f};
    csplat::DevBuf partial;    // split-N partial reductions
    csplat::DevBuf staging;    // host-pointer staging (inputs + outputs)
    csplat::DevBuf flags;      // validation flag; precision form: recheck counters
    csplat::DevBuf sortbuf;    // spatial sort of the queries (codes, permutation, sorted copies)
    csplat::DevBuf bodies;     // prepared ellipsoid records
    csplat::DevBuf minbuf;     // minimum search: per-query state, lists, gathered queries
    csplat_eval_stats stats{};
    int32_t *flag_counts = nullptr;  // device: rechecked queries per n_sigma (last eval)
    int32_t flag_m = 0;
    unsigned long long *chunk_counter = nullptr;  // device: culling chunks evaluated (last eval)
    int64_t pairs_per_chunk = 0;
    bool timing = false;
    bool timed = false;         // events of the last evaluation were recorded
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    float timed_ms = -1.f;      // >= 0: the dominant kernel's time summed over several launches
    // precision forms: the last value's recheck list (sorted indices), its
    // length and the sort permutation, all device memory of the workspace
    const int32_t *rk_list = nullptr, *rk_n = nullptr, *rk_perm = nullptr;
    int64_t rk_q = 0;
    int *check_host = nullptr;      // pinned: the device-side input check's flag
    int *check_dev = nullptr;       // its device address
    bool check_pending = false;     // a check is queued and not yet waited for
    hipEvent_t ev_check = nullptr;  // recorded after the check kernel
};

namespace csplat {

// Record the timing events around the dominant kernel of an evaluation.
inline void timing_begin(csplat_ctx *ctx)
{
    if (ctx->timing) (void)hipEventRecord(ctx->ev0, ctx->stream);
}
inline void timing_end(csplat_ctx *ctx)
{
    if (ctx->timing) {
        (void)hipEventRecord(ctx->ev1, ctx->stream);
        ctx->timed = true;
    }
}

// Blocks per compute unit that a launch aims for: several rounds of resident
// blocks, so that uneven work items even out (measured on MI355X: 64 beats
// 16 and 32, and 96-128 on the navigation workload, whose partials grow).
#ifndef CSPLAT_BLOCKS_PER_CU
#define CSPLAT_BLOCKS_PER_CU 64
#endif
int target_blocks(int device);
inline int ctx_target_blocks(const csplat_ctx *ctx) { return target_blocks(ctx->device); }

// Zero n int32 words on the stream with a kernel (safe under graph capture).
hipError_t zero_words(int32_t *p, size_t n, hipStream_t st);

// scene.hip
csplat_status scene_build(csplat_ctx *ctx, int64_t n, const float *means, const float *quats,
                          const float *scales, const float *opacity,
                          const csplat_scene_opts &opts, csplat_scene *scene);
// Frees the scene's device memory in the order of `st` (stream-ordered
// frees: the memory was allocated with hipMallocAsync).
void scene_release(csplat_scene *scene, hipStream_t st);
// abi.hip: records that `st` has queued work reading the scene (an event after
// it), so that freeing the scene waits for exactly that work.
void scene_note_use(const csplat_scene *scene, hipStream_t st, bool may_create = true);

// Parameters of one evaluation, precomputed on the host from the options.
struct EvalParams {
    int32_t m;
    int32_t k;
    float two_n[CSPLAT_MAX_M];    // 2 n_v            (sqrt(sigma^2) r^2 = 2 sqrt(V))
    float four_n2[CSPLAT_MAX_M];  // 4 n_v^2          (sqrt-free label test)
    float kt;                     // log2(e) / tau, or 1 when tau = 0
    float inv_kt;
    float g1, g0;                 // cost exponent in base 2: min(g0 - g1 t, 0)
    float d_max;
    float rn2;                    // neighbour radius squared (+inf: all)
    int32_t soft;                 // tau > 0
    float n_sigma[CSPLAT_MAX_M];  // the conservatism values as given
    float r_nbr;                  // neighbour radius (+inf: all)
    float n_max;                  // largest conservatism value
    int32_t cull;                 // skip chunks outside every ball / beyond every reach
};

struct EvalOut {
    uint8_t *label;
    int32_t *count;
    float *min;
    float *softmin;
    float *cost;
    int32_t *nbr;
    float *err;  // precision forms: certified bound of |min - exact minimum|
};

// Evaluation parameters from conservatism values and reduction options
// (validates the options; CSPLAT_E_INVALID with a message on error).
csplat_status build_params(const float *n_sigma, int m, const csplat_reduce_opts &o, EvalParams &p);
// 1 if p is a device (or managed) pointer, 0 for host memory.
int pointer_kind(const void *p);

// Device memory for an evaluation's workspace supplied by the caller (the
// sorted queries, then the split partials) in place of the context's
// growable buffers: nothing is allocated, and the split count is capped so
// that the partials fit (fewer, longer splits: the same counts, labels,
// minima and ball sizes; the softmin and cost sums in another order).
struct Workspace {
    char *base;
    size_t bytes;
};

// A copy of q query spheres sorted along the scene's Hilbert curve, with the
// permutation (sorted index -> caller index) and a zeroed 64-bit counter,
// all in the context's sort workspace (valid until the next evaluation).
struct SortedQueries {
    const float *c;
    const float *r;
    const int32_t *perm;
    unsigned long long *counter;
};
csplat_status sort_queries(csplat_ctx *ctx, const csplat_scene *sc, int q, const float *centers,
                           const float *radii, SortedQueries *out);
// The same for ellipsoid records (ell: `centers` holds kBodyFloats-float
// records, which are gathered into out->c; out->r is NULL).
csplat_status sort_bodies(csplat_ctx *ctx, const csplat_scene *sc, int q, const float *centers,
                          const float *radii, bool ell, SortedQueries *out, const Workspace *ws = nullptr);
// Device bytes the sort of q bodies needs (its part of a Workspace).
csplat_status sort_workspace_bytes(int q, bool ell, hipStream_t st, size_t *bytes);
// Ellipsoid records from centres (q x 3), (w, x, y, z) quaternions (q x 4) and
// semi-axes (q x 3), all device pointers, on the context stream.
csplat_status prepare_bodies(csplat_ctx *ctx, int q, const float *centers, const float *quats, const float *axes,
                             float *rec);
// Host-side check of ellipsoidal bodies: finite centres, finite nonzero
// quaternions, finite semi-axes > 0.
bool bodies_valid_host(int64_t q, const float *c, const float *quat, const float *ax);
// The same on any stream (the serving form's copy stream).
hipError_t prepare_bodies_on(hipStream_t st, int q, const float *centers, const float *quats, const float *axes,
                             float *rec);

// pair_fp32.hip: the float32 pair kernel and the split combine.
// `gate`, when given, runs after the pair kernel is queued and before
// anything that writes the outputs; an error from it is returned with no
// output written (the queued kernels write only the context's workspace).
csplat_status fp32_eval(csplat_ctx *ctx, const csplat_scene *scene, int64_t q,
                        const float *centers, const float *radii, const EvalParams &p,
                        const EvalOut &out, bool labels_only, bool ell = false,
                        const std::function<csplat_status()> &gate = {}, const Workspace *ws = nullptr);

// The minimum of s~^2 over every kept Gaussian for spheres (labels and
// counts optional), by the threshold passes of the task walk; the passes
// synchronise with the host once each (the next pass's size).
csplat_status fp32_min_eval(csplat_ctx *ctx, const csplat_scene *scene, int64_t q, const float *centers,
                            const float *radii, const EvalParams &p, const EvalOut &out,
                            const std::function<csplat_status()> &gate = {});

// precision.hip: MFMA form with certified recheck (labels and counts).
// gate: called once before the first kernel that writes an output (the
// caller's check of device inputs); an error from it is returned as is.
csplat_status precision_eval(csplat_ctx *ctx, const csplat_scene *scene, int64_t q,
                             const float *centers, const float *radii, const EvalParams &p,
                             const EvalOut &out, int precision,
                             const std::function<csplat_status()> &gate = {});
// Labels and counts of ellipsoid records (kBodyFloats floats each, the
// caller's order) in an MFMA precision form.
csplat_status precision_eval_ell(csplat_ctx *ctx, const csplat_scene *scene, int64_t q, const float *rec,
                                 const EvalParams &p, const EvalOut &out, int precision);
csplat_status precision_build(csplat_ctx *ctx, csplat_scene *scene, uint32_t features);

}  // namespace csplat
