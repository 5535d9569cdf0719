/*
 * csplat — CollisionSplatting robot-versus-3DGS metric on one MI355X (gfx950).
 *
 * C ABI.  Plain pointers and sizes; no exceptions cross it; every call returns
 * a csplat_status (0 = OK) and leaves a thread-local message for
 * csplat_last_error() on failure.  All floating-point inputs are IEEE float32,
 * row-major, little-endian.  Every allocation is owned by a context, scene or
 * server and released by its destroy/free call.
 *
 * The method (Sec. II-B of the paper): each Gaussian i (mean mu_i, covariance
 * Sigma_i = R_i S_i S_i^T R_i^T, Eq. 2) is treated as an uncertain point
 * obstacle.  For a robot sphere j (centre c_j, radius r_j; the ellipsoid of
 * Eq. 5-6 with a = b = c = r_j) the scaling-function distance is
 * s^2 = |mu_i - c_j|^2 / r_j^2 (Eq. 5); its linearised variance is
 * sigma^2 = g^T Sigma_i g with g = 2 (mu_i - c_j) / r_j^2 (Eq. 7); the
 * conservative metric is s~^2 = max(0, s^2 - n_sigma sqrt(sigma^2)) (Eq. 8).
 * Per query the pairs are reduced over the neighbourhood ball
 * N_j = { i : |mu_i - c_j| <= neighbor_radius }:
 *   count = #{ i in N_j : s~^2 < 1 },  label = count > k       (Sec. II-E)
 *   min   = min over N_j of s~^2 (+inf if N_j is empty)
 *   softmin = -tau log sum exp(-s~^2 / tau), evaluated about the minimum
 *             (the numerically stable softmin of Sec. II-B; tau = 0: min)
 *   cost  = mean over N_j of d_max exp(-gamma max(s~^2 - s_min, 0))
 *           (Eq. 11, averaged over neighbouring splats, Sec. II-D; 0 if empty)
 * Results are in s~^2 units (dimensionless, collision threshold 1).
 *
 * Evaluation calls: `centers`, `radii` and every non-NULL output must be all
 * device pointers or all host pointers.  Device pointers run asynchronously
 * on the context's stream; host pointers are staged through device memory and
 * the call returns when the outputs are written.  Outputs are query-major:
 * element [j * m + v] belongs to query j and conservatism value v.  All checks
 * run before any device work; on error no output is written.  q = 0 is a
 * no-op returning CSPLAT_OK.
 */
#ifndef CSPLAT_H
#define CSPLAT_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t csplat_status;
#define CSPLAT_OK 0
#define CSPLAT_E_INVALID 1   /* bad argument or input value */
#define CSPLAT_E_OOM 2       /* device or host allocation failed */
#define CSPLAT_E_DEVICE 3    /* HIP runtime error */
#define CSPLAT_E_BUSY 4      /* server: the request can never fit the budget */
#define CSPLAT_E_NOT_FOUND 5 /* server: unknown ticket or scene id */
#define CSPLAT_E_PENDING 6   /* server poll: not finished yet */
#define CSPLAT_E_CANCELLED 7 /* server: the request was cancelled */

#define CSPLAT_MAX_M 8 /* conservatism values per evaluation */

typedef struct csplat_ctx csplat_ctx;
typedef struct csplat_scene csplat_scene;
typedef struct csplat_server csplat_server;

/* Scene parameter conventions. */
#define CSPLAT_PARAM_ACTIVATED 0 /* linear scales (std. dev.), opacity in [0, 1] */
#define CSPLAT_PARAM_RAW_3DGS 1  /* log-scales and opacity logits (3DGS storage) */

/* Arithmetic of an evaluation. */
#define CSPLAT_PRECISION_FP32 0         /* plain float32 pair kernel */
#define CSPLAT_PRECISION_BF16_RECHECK 1 /* bf16 MFMA + certified fp32/fp64 recheck */
#define CSPLAT_PRECISION_FP16_RECHECK 2 /* fp16 MFMA + certified fp32/fp64 recheck */

/* Bits of csplat_scene_opts.precision_features: the packed MFMA operands of
 * the precision forms for spheres (96 B per Gaussian and dtype) and for
 * ellipsoidal bodies (320 B per Gaussian and dtype). */
#define CSPLAT_FEATURES_BF16 1u
#define CSPLAT_FEATURES_FP16 2u
#define CSPLAT_FEATURES_ELL_BF16 4u
#define CSPLAT_FEATURES_ELL_FP16 8u

typedef struct {
    int32_t param_mode;          /* CSPLAT_PARAM_* */
    float floater_opacity_max;   /* alpha_f: drop i iff alpha_i < alpha_f and  */
    float floater_extent_min;    /* max_k s_ik > e_f (Sec. II-C); alpha_f <= 0 disables */
    uint32_t precision_features; /* CSPLAT_FEATURES_* to build at load time */
} csplat_scene_opts;

typedef struct {
    int32_t k;             /* label = count > k (k >= 0; Sec. II-E "more than a small number") */
    float softmin_tau;     /* tau >= 0; 0 reports the hard minimum as softmin */
    float neighbor_radius; /* > 0, or +INFINITY for every kept Gaussian */
    float d_max;           /* Eq. 11, > 0 */
    float gamma;           /* Eq. 11, >= 0 */
    float s_min;           /* Eq. 11, the paper uses 1 */
    int32_t precision;     /* CSPLAT_PRECISION_*; the MFMA forms compute labels, counts (exact:
                              certified, the rest rechecked in fp64) and min with its error bound
                              err, over every kept Gaussian: they reject a finite neighbor_radius,
                              softmin, cost and nbr (CSPLAT_E_INVALID) */
    int32_t cull;          /* 1: sort the queries along a Hilbert curve and skip the
                              Gaussians (in groups of 1024, chunks of 64 and sub-chunks of 16
                              consecutive on the scene's curve) that provably lie outside a
                              query's neighbourhood ball (or, for labels, beyond the reach bound
                              n s_max + sqrt(n^2 s_max^2 + r^2) of Eq. 8); the results are the
                              same bits as with 0, which evaluates every pair.  With an infinite
                              ball, min without softmin, cost and nbr (labels and counts
                              optional) runs as passes of a threshold search that skip every
                              Gaussian provably above the query's minimum (the same bits as
                              every pair; one host synchronisation per pass); softmin and
                              cost with an infinite ball never cull. */
} csplat_reduce_opts;

/* Outputs of one evaluation; every pointer is nullable (not computed/written). */
typedef struct {
    uint8_t *label;  /* q x m, count > k */
    int32_t *count;  /* q x m */
    float *min;      /* q x m, s~^2 units */
    float *softmin;  /* q x m */
    float *cost;     /* q x m */
    int32_t *nbr;    /* q, |N_j| (size of the neighbourhood ball) */
    float *err;      /* q x m, precision forms only (with or without min): a certified bound
                        on |min - exact minimum| in s~^2 units (the minimum from the bf16/fp16
                        contraction is the middle of a certified interval; err is its
                        half-width plus float32 rounding) */
} csplat_outputs;

/* Statistics of the last evaluation on a context. */
typedef struct {
    int64_t pairs;          /* q * n_kept */
    int64_t flagged;        /* precision forms: queries rechecked in fp32 */
    int64_t flagged_fp64;   /* precision forms: queries rechecked in fp64 */
    int32_t splits;         /* Gaussian ranges evaluated side by side */
    int32_t queries_per_lane;
    int64_t kernel_pairs;   /* pairs the dominant kernel evaluated (after any culling) */
    float kernel_ms;        /* with timing on: duration of the dominant (pair) kernel,
                               measured with HIP events on the context stream; else -1 */
    uint64_t workspace_bytes; /* device bytes the context holds (partials, sorted queries,
                                 staging, body records, counters) */
    int32_t min_passes;     /* minimum over every kept Gaussian: walks of the threshold search
                               (kernel_ms then sums their pair kernels); else 0 */
} csplat_eval_stats;

/* Context: a device, a stream (its own if hip_stream is NULL, else the given
 * hipStream_t is borrowed and never destroyed) and a workspace that grows on
 * demand.  Not thread-safe: one context per thread of use. */
csplat_status csplat_ctx_create(int32_t device, void *hip_stream, csplat_ctx **out);
csplat_status csplat_ctx_destroy(csplat_ctx *ctx);

/* Load a 3DGS scene (Sec. II-A): n Gaussians with means (n x 3), quaternions
 * (n x 4, (w, x, y, z), any nonzero norm; normalised here), scales (n x 3) and
 * opacity (n).  Host pointers only; the inputs are copied and may be freed
 * after return.  On the device the parameters are validated and activated,
 * the floater filter applied, Sigma_i factored as M_i = diag(s_i) R_i^T and
 * the survivors sorted along a Hilbert curve.  n = 0 is allowed.
 * Errors: CSPLAT_E_INVALID (n < 0, NULL pointer with n > 0, a non-finite
 * value, a zero quaternion, a negative linear scale), CSPLAT_E_OOM,
 * CSPLAT_E_DEVICE.  opts may be NULL (activated, no filter, no features). */
csplat_status csplat_scene_load(csplat_ctx *ctx, int64_t n, const float *means,
                                const float *quats, const float *scales,
                                const float *opacity, const csplat_scene_opts *opts,
                                csplat_scene **out);
/* Scene files (Sec. II-A): the binary little-endian PLY layout written by the
 * 3DGS and 2DGS trainers.  Per vertex: x, y, z, opacity (logit), scale_0,
 * scale_1 and, for 3DGS, scale_2 (log; 2DGS files have two scales: the third
 * axis is flat, scale 0), rot_0..rot_3 ((w, x, y, z)); every other vertex
 * property (normals, spherical-harmonic colours) is skipped, as are other
 * elements after the vertices.  Property types: any PLY scalar type.
 *
 * csplat_ply_read parses the file on the host into activated parameters
 * (linear scales exp(s), opacity sigmoid(o), computed in double; quaternions
 * as stored): with capacity 0 it only sets *n; otherwise the arrays (n x 3,
 * n x 4, n x 3, n, caller-owned) must hold capacity >= n Gaussians.  No GPU
 * is needed.  csplat_scene_load_ply reads the file and loads it as
 * csplat_scene_load would (opts as there; param_mode is ignored).
 * Errors: CSPLAT_E_INVALID (cannot open, not binary little-endian PLY, a
 * missing property, list properties in the vertex element, truncated data,
 * capacity below n), then those of csplat_scene_load. */
csplat_status csplat_ply_read(const char *path, int64_t capacity, int64_t *n, float *means,
                              float *quats, float *scales, float *opacity);
csplat_status csplat_scene_load_ply(csplat_ctx *ctx, const char *path,
                                    const csplat_scene_opts *opts, csplat_scene **out);
/* Kept Gaussians and device bytes held by the scene (the VRAM figure). */
csplat_status csplat_scene_info(const csplat_scene *scene, int64_t *n_kept,
                                uint64_t *device_bytes);
/* Free the scene.  Returns without waiting: its device memory is released in
 * stream order once every evaluation queued on it (by any context, or an RRT
 * tree) has finished; only those streams are waited for (a stream that ran
 * csplat_eval_noalloc on the scene and nothing else is waited for whole).  A
 * server that serves the scene must be destroyed first. */
csplat_status csplat_scene_free(csplat_scene *scene);

/* The conservatism n_sigma of Eq. 8: m values (1..8), each finite and >= 0.
 * Stored in the context for later evaluations; on error the context is left
 * unchanged. */
csplat_status csplat_set_conservatism(csplat_ctx *ctx, const float *n_sigma, int32_t m);

/* Evaluate q query spheres (centres q x 3, radii q, each finite and > 0)
 * against the scene for the context's m conservatism values, computing only
 * the non-NULL outputs. */
csplat_status csplat_eval(csplat_ctx *ctx, const csplat_scene *scene, int64_t q,
                          const float *centers, const float *radii,
                          const csplat_reduce_opts *opts, const csplat_outputs *out);
/* Labels (and optionally counts) only: csplat_eval with label/count set. */
csplat_status csplat_eval_labels(csplat_ctx *ctx, const csplat_scene *scene, int64_t q,
                                 const float *centers, const float *radii,
                                 const csplat_reduce_opts *opts, uint8_t *label,
                                 int32_t *count);
/* Distances: min (required), softmin and cost (nullable). */
csplat_status csplat_eval_distance(csplat_ctx *ctx, const csplat_scene *scene, int64_t q,
                                   const float *centers, const float *radii,
                                   const csplat_reduce_opts *opts, float *min,
                                   float *softmin, float *cost);

/* For callers that cannot allocate device or pinned memory during a call
 * (harnesses that forbid hipMalloc, tight serving loops): csplat_eval with
 * the float32 path, allocating nothing.  Its workspace (the sorted queries and
 * the split partials) is a fixed CSPLAT_NOALLOC_SCRATCH_MB MiB array in the
 * library, one per GPU, held until the process ends; the context's check flag
 * is allocated by csplat_ctx_create.  Every array must be a device pointer
 * (host arrays would need staging).  The work is cut into fewer, longer
 * splits when the partials of the usual plan do not fit, so label, count, min
 * and nbr equal csplat_eval's bit for bit and softmin and cost agree to float32
 * rounding of the reordered sums.  Calls that overlap on one GPU (several
 * contexts or streams, or threads) share that array and race: serialise
 * them.  The call waits once for the device-side input check, like
 * csplat_eval with device pointers.  Errors: those of csplat_eval, and
 * CSPLAT_E_INVALID for host pointers, opts->precision other than
 * CSPLAT_PRECISION_FP32, q > CSPLAT_NOALLOC_MAX_Q, or a problem whose
 * workspace does not fit the array. */
#define CSPLAT_NOALLOC_SCRATCH_MB 64
#define CSPLAT_NOALLOC_MAX_Q 262144
csplat_status csplat_eval_noalloc(csplat_ctx *ctx, const csplat_scene *scene, int64_t q,
                                  const float *centers, const float *radii,
                                  const csplat_reduce_opts *opts, const csplat_outputs *out);

/* Ellipsoidal robot bodies (Eq. 5-6 with a general A_j, Sec. II-B): body j
 * has centre c_j (q x 3), orientation quaternion (q x 4, (w, x, y, z), any
 * nonzero norm; normalised here) and semi-axes (a, b, c) > 0 along its local
 * x, y, z axes (q x 3), so A_j = R_j diag(1/a^2, 1/b^2, 1/c^2) R_j^T and
 * s~^2 = max(0, s^2 - n sqrt(sigma^2)) with s^2 = d^T A d and
 * sigma^2 = 4 d^T A Sigma A d (Eq. 7-8).  A sphere is a = b = c = r.
 * Outputs, options, pointer rules and the neighbourhood ball (about c_j) are
 * those of csplat_eval.  The MFMA precision forms (opts->precision
 * BF16_RECHECK or FP16_RECHECK; the scene loaded with CSPLAT_FEATURES_ELL_BF16
 * or _ELL_FP16) compute labels and counts over every kept Gaussian: a
 * certified bound decides each pair, the undecided bodies are rechecked in
 * fp64, and both take B = L^T L in float32 from L = diag(1/a, 1/b, 1/c) R^T
 * (float32), so the counts are exact for that B (within float32 rounding of
 * A_j).  They reject min, softmin, cost, nbr, err and a finite
 * neighbor_radius.  Errors: CSPLAT_E_INVALID (as csplat_eval, or a
 * non-finite centre, a zero or non-finite quaternion, a semi-axis not finite
 * and > 0, or a precision form whose features the scene lacks). */
csplat_status csplat_eval_ellipsoids(csplat_ctx *ctx, const csplat_scene *scene, int64_t q,
                                     const float *centers, const float *quats, const float *axes,
                                     const csplat_reduce_opts *opts, const csplat_outputs *out);

/* Planner epilogues: reductions of per-query outputs over segments of
 * consecutive queries -- the links of a robot state or the points x links of
 * an RRT edge ("in collision if any link ...", Sec. II-E), the steps x links
 * of an MPPI rollout (the rollout's collision cost sums the per-body costs
 * over links and horizon, Sec. II-D, Eq. 11).  Segment s covers queries
 * [offsets[s], offsets[s+1]) (n_seg + 1 values rising from 0 to q); with
 * offsets NULL every segment has q / n_seg queries (q a multiple of n_seg).
 *   label (q x m) -> seg_any (n_seg x m): 1 iff some query of the segment has
 *                    label 1, else 0 (an empty segment gives 0);
 *   cost  (q x m) -> seg_cost (n_seg x m): the sum over the segment, in a
 *                    fixed order (bit-reproducible; 0 for an empty segment).
 * Either output may be NULL (not both); an output needs its input.  All
 * pointers host or all device, as for csplat_eval (device: asynchronous on
 * the context stream; device offsets are checked by a kernel and one stream
 * synchronisation first).  Errors: CSPLAT_E_INVALID (bad sizes or offsets,
 * mixed pointer kinds); nothing is written on error. */
csplat_status csplat_segment_reduce(csplat_ctx *ctx, int64_t q, int32_t m, int64_t n_seg,
                                    const int64_t *offsets, const uint8_t *label, const float *cost,
                                    uint8_t *seg_any, float *seg_cost);

/* ---------------------------------------------------------------------------
 * Batched RRT step on the GPU (Sec. II-E): the tree lives in device memory.
 * Each step draws n_batch configuration samples (or takes the caller's), finds
 * each sample's nearest tree node (Euclidean; ties to the lowest index),
 * expands it toward the sample by at most `step` (steer), checks the edge at
 * n_strides = ceil(step / resolution) points (the float32 quotient) spaced evenly from the node
 * (exclusive) to the new end (inclusive), each point placing the robot's
 * n_links spheres (a rigid template: offsets and radii), and appends the
 * collision-free edges' ends as new nodes in batch order.  A state is in
 * collision when any link has more than k Gaussians with s~^2 < 1 for the
 * conservatism n_sigma (the label of csplat_eval, over every kept Gaussian).
 * A configuration is the template's origin in 3-D (a rigid body that
 * translates).  Zero-length edges (a sample on its nearest node) are not
 * appended.  The collision check runs the float32 label path (culled, the same
 * labels as csplat_eval) on the context's stream; a step does not wait for
 * the device unless n_added is requested.
 */
typedef struct csplat_rrt csplat_rrt;
typedef struct {
    float lo[3], hi[3];     /* sampling box of configurations (lo < hi on every axis) */
    float step;             /* largest stride of an edge (> 0) */
    float resolution;       /* spacing of the collision checks along an edge (> 0) */
    float n_sigma;          /* conservatism (Eq. 8), finite and >= 0 */
    int32_t k;              /* label = count > k (k >= 0) */
    int32_t n_links;        /* spheres of the robot template (1..64) */
    const float *link_offsets; /* n_links x 3, host memory, copied at creation */
    const float *link_radii;   /* n_links, finite and > 0, host memory, copied */
    uint64_t seed;          /* of the counter-based sample generator (SplitMix64) */
} csplat_rrt_opts;

/* A tree with one root node (3 floats, host) and room for max_nodes nodes,
 * on the context's device and stream, over a loaded scene (which must outlive
 * the tree).  Errors: CSPLAT_E_INVALID (bad options, max_nodes < 1 or above
 * 2^26), CSPLAT_E_OOM, CSPLAT_E_DEVICE. */
csplat_status csplat_rrt_create(csplat_ctx *ctx, const csplat_scene *scene, const csplat_rrt_opts *opts,
                                int32_t max_nodes, const float *root, csplat_rrt **out);
csplat_status csplat_rrt_destroy(csplat_rrt *rrt);
/* One step with n_batch samples (1..65536; n_batch x n_strides x n_links <=
 * 2^24 spheres): `samples` (n_batch x 3, a device pointer; NULL: drawn
 * uniformly in the box by SplitMix64 on counter (seed, step, sample, axis)).
 * Nodes beyond max_nodes are dropped (the tree stops growing).  With n_added
 * (host) the call waits and reports the nodes appended.  Errors:
 * CSPLAT_E_INVALID, CSPLAT_E_DEVICE. */
csplat_status csplat_rrt_step(csplat_rrt *rrt, int32_t n_batch, const float *samples, int32_t *n_added);
/* The tree (waits for the stream): up to cap nodes' positions (cap x 3) and
 * parents (the root's is -1), host memory of the caller (either may be NULL);
 * *n = the number of nodes. */
csplat_status csplat_rrt_nodes(csplat_rrt *rrt, float *pos, int32_t *parent, int32_t cap, int32_t *n);
/* The last step's edges (waits for the stream), host arrays of its n_batch
 * entries (any may be NULL): the nearest node, the edge's end, and 1 if the
 * edge was collision-free and of positive length. */
csplat_status csplat_rrt_last_edges(csplat_rrt *rrt, int32_t *nearest, float *end, uint8_t *valid);

/* Timing mode (off by default): when on, every evaluation records HIP events
 * around its dominant kernel and csplat_last_stats waits for the second one. */
csplat_status csplat_ctx_set_timing(csplat_ctx *ctx, int32_t enable);
/* Statistics of the last evaluation (with timing on, waits for its kernel). */
csplat_status csplat_last_stats(csplat_ctx *ctx, csplat_eval_stats *stats);
/* ---------------------------------------------------------------------------
 * Serving form: resident scenes and continuous batching of planner requests
 * (MPPI rollout batches of shape (K, T, N_link), Sec. II-D, and RRT edge
 * checks of shape N_batch x N_strides x N_links, Sec. II-E).
 *
 * A server owns one device stream, a worker thread, a device arena of
 * `hbm_budget` bytes (query inputs and partial reductions of admitted
 * requests) and a pinned host arena of the same size (input staging and
 * outputs), both allocated at creation: serving itself allocates nothing.
 * Requests are admitted in arrival order while a slot and memory are free
 * (a request that does not fit yet does not block smaller later ones), cut
 * into work items (query tile x Gaussian range) and evaluated in bounded
 * steps together with whatever else is admitted; each step is a replay of a
 * captured HIP graph.  A request's results never depend on what it shares
 * the device with: they are bit-identical to csplat_eval on a context of the
 * same device with the same conservatism value and options.
 * Thread-safe: submit, poll, wait and cancel may be called from any thread.
 */
#define CSPLAT_SERVE_COST 0   /* label, count, min, softmin, cost, nbr (MPPI) */
#define CSPLAT_SERVE_LABELS 1 /* label, count (RRT edge checks) */

typedef struct {
    int64_t submitted, completed, cancelled, refused;
    int64_t steps;            /* graph replays issued */
    double p50_ms, p99_ms;    /* submit -> results in host memory, completed requests */
    double mean_ms, max_ms;
    double pairs_per_s;       /* Q x N_kept of completed requests / serving wall time */
    double busy_s;            /* first admission to last completion */
    int64_t shared_steps;     /* steps that evaluated work items of two or more requests */
    int32_t max_requests_per_step;
} csplat_serving_stats;

/* Create a server on `device` with `hbm_budget` bytes of device arena (and as
 * much pinned host memory) and at most `slots` (1..64) requests on the device
 * at a time.  Errors: CSPLAT_E_INVALID, CSPLAT_E_OOM, CSPLAT_E_DEVICE. */
csplat_status csplat_server_create(int32_t device, uint64_t hbm_budget, int32_t slots,
                                   csplat_server **out);
/* Stop the worker (in-flight steps finish first) and free everything. */
csplat_status csplat_server_destroy(csplat_server *srv);
/* Serve a loaded scene (same device; it must outlive the server). */
csplat_status csplat_server_add_scene(csplat_server *srv, const csplat_scene *scene,
                                      int32_t *scene_id);
/* Submit q query spheres (host arrays, copied before return) for `kind`
 * against scene `scene_id` with one conservatism value n_sigma (m must be 1)
 * and float32 options.  Returns a ticket.  CSPLAT_E_BUSY if the request can
 * never fit the budgets; CSPLAT_E_INVALID for bad arguments (the same checks
 * as csplat_eval); CSPLAT_E_NOT_FOUND for an unknown scene id. */
csplat_status csplat_server_submit(csplat_server *srv, int32_t scene_id, int32_t kind, int64_t q,
                                   const float *centers, const float *radii,
                                   const csplat_reduce_opts *opts, const float *n_sigma,
                                   int32_t m, uint64_t *ticket);
/* The same for q ellipsoidal bodies (Eq. 5-6, host arrays as in
 * csplat_eval_ellipsoids: centres q x 3, (w, x, y, z) quaternions q x 4,
 * semi-axes q x 3).  The bodies are prepared on the device by the kernel
 * csplat_eval_ellipsoids uses, so the results are the same bits as that call
 * with one conservatism value.  Errors: those of csplat_server_submit, and
 * CSPLAT_E_INVALID for the body checks of csplat_eval_ellipsoids. */
csplat_status csplat_server_submit_ellipsoids(csplat_server *srv, int32_t scene_id, int32_t kind, int64_t q,
                                              const float *centers, const float *quats, const float *axes,
                                              const csplat_reduce_opts *opts, const float *n_sigma, int32_t m,
                                              uint64_t *ticket);
/* Non-blocking: CSPLAT_E_PENDING while queued or running; CSPLAT_OK once
 * done, after copying the non-NULL outputs (host pointers, q x 1 each) and
 * forgetting the ticket; CSPLAT_E_CANCELLED (ticket forgotten);
 * CSPLAT_E_NOT_FOUND for an unknown ticket. */
csplat_status csplat_server_poll(csplat_server *srv, uint64_t ticket, const csplat_outputs *out);
/* Like poll, but blocks until the request is done or cancelled, or until
 * timeout_ms (< 0: no limit) has passed (then CSPLAT_E_PENDING). */
csplat_status csplat_server_wait(csplat_server *srv, uint64_t ticket, const csplat_outputs *out,
                                 int64_t timeout_ms);
/* Cancel a queued or running request (a running one stops after its
 * in-flight step).  CSPLAT_E_NOT_FOUND if unknown or already finished. */
csplat_status csplat_server_cancel(csplat_server *srv, uint64_t ticket);
csplat_status csplat_server_stats(csplat_server *srv, csplat_serving_stats *stats);
/* Latencies (submit -> results in host memory, milliseconds) of the completed
 * requests in completion order, for confidence intervals on the percentiles
 * of csplat_server_stats.  Copies min(cap, completed) values into `ms` (host
 * memory owned by the caller; may be NULL when cap is 0) and sets *n to the
 * number of completed requests.  CSPLAT_E_INVALID for a NULL server or n, or
 * cap < 0. */
csplat_status csplat_server_latencies(csplat_server *srv, double *ms, int64_t cap, int64_t *n);

/* Precision forms: the queries of the last evaluation (its last conservatism
 * value) whose label the certified bound left undecided and which were
 * rechecked in fp64, as indices into the caller's query array in sorted
 * (curve) order.  Copies min(cap, count) indices into `idx` (host memory of
 * the caller; NULL when cap is 0) and sets *n to the count (0 after a float32
 * evaluation).  Synchronises the context's stream. */
csplat_status csplat_last_rechecked(csplat_ctx *ctx, int32_t *idx, int64_t cap, int64_t *n);

/* Wait for all work queued on the context's stream. */
csplat_status csplat_synchronize(csplat_ctx *ctx);
/* Message of the last failed call on this thread ("" if none); valid until
 * the next csplat call on the same thread. */
const char *csplat_last_error(void);

#ifdef __cplusplus
}
#endif

#endif
