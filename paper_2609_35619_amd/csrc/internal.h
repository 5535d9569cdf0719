// Internal declarations shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>

#include "../../include/csplat.h"

namespace csplat {

// Per-Gaussian record of the float32 pair kernel: 12 floats, read by scalar
// (wave-uniform) loads.  M = diag(s) R^T, so that for d = mu - c the
// linearised variance term V = d^T Sigma d = |M d|^2 is a sum of squares.
constexpr int kGaussFloats = 12;  // mx my mz | M00 M01 M02 | M10 M11 M12 | M20 M21 M22

// Per-Gaussian record of the MFMA precision form, in tile-local coordinates
// about the tile origin o_T (16 bf16 or fp16 values per feature row).
constexpr int kTile = 64;         // Gaussians per precision tile
constexpr int kFeat = 16;         // padded feature length (K of the contraction)

void set_error(const std::string &msg);
csplat_status fail(csplat_status code, const std::string &msg);
csplat_status hip_fail(hipError_t e, const char *what);

#define CSPLAT_HIP(call)                                      \
    do {                                                      \
        hipError_t e_ = (call);                               \
        if (e_ != hipSuccess) return ::csplat::hip_fail(e_, #call); \
    } while (0)

// A device buffer that grows on demand (never shrinks until freed).
struct DevBuf {
    void *ptr = nullptr;
    size_t bytes = 0;
    hipError_t reserve(size_t want);
    void release();
    template <class T> T *as() const { return static_cast<T *>(ptr); }
};

}  // namespace csplat

struct csplat_scene {
    int device = 0;
    int64_t n_input = 0;
    int64_t n = 0;            // kept Gaussians
    float *gauss = nullptr;   // n x 12 float32 records, Morton order
    // precision form (optional)
    int64_t n_tiles = 0;
    float *tile_origin = nullptr;   // n_tiles x 4 (ox, oy, oz, 0)
    float *tile_bound = nullptr;    // n_tiles x 4: max |mu'|, max s, max |Sigma|, max |Sigma mu'|
    void *feat_bf16 = nullptr;      // n_tiles*kTile x 2 x kFeat bf16 (D row, V row)
    void *feat_fp16 = nullptr;
    uint64_t device_bytes = 0;
};

struct csplat_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    int32_t m = 1;
    float n_sigma[CSPLAT_MAX_M] = {1.0f};
    csplat::DevBuf partial;    // split-N partial reductions
    csplat::DevBuf staging;    // host-pointer staging (inputs + outputs)
    csplat::DevBuf flags;      // precision form: flagged-query list and counters
    csplat_eval_stats stats{};
    bool timing = false;
    bool timed = false;         // events of the last evaluation were recorded
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
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

// scene.hip
csplat_status scene_build(csplat_ctx *ctx, int64_t n, const float *means, const float *quats,
                          const float *scales, const float *opacity,
                          const csplat_scene_opts &opts, csplat_scene *scene);
void scene_release(csplat_scene *scene);

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
};

struct EvalOut {
    uint8_t *label;
    int32_t *count;
    float *min;
    float *softmin;
    float *cost;
    int32_t *nbr;
};

// pair_fp32.hip: the float32 pair kernel and the split combine.
csplat_status fp32_eval(csplat_ctx *ctx, const csplat_scene *scene, int64_t q,
                        const float *centers, const float *radii, const EvalParams &p,
                        const EvalOut &out, bool labels_only);

// precision.hip: MFMA form with certified recheck (labels and counts).
csplat_status precision_eval(csplat_ctx *ctx, const csplat_scene *scene, int64_t q,
                             const float *centers, const float *radii, const EvalParams &p,
                             const EvalOut &out, int precision);
csplat_status precision_build(csplat_ctx *ctx, csplat_scene *scene, uint32_t features);

}  // namespace csplat
