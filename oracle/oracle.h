/*
 * FP64 CPU oracle for the CollisionSplatting metric (test infrastructure only;
 * see oracle.c for the definition and its citations).
 */
#ifndef CSPLAT_ORACLE_H
#define CSPLAT_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define ORACLE_OK 0
#define ORACLE_E_INVALID 1
#define ORACLE_E_OOM 2
#define ORACLE_MAX_M 8

typedef struct {
    int32_t k;      /* label = count > k */
    double tau;     /* softmin temperature (0: hard min) */
    double r_nbr;   /* neighbourhood ball radius (+inf: all splats) */
    double d_max;   /* Eq. 11 */
    double gamma;   /* Eq. 11 */
    double s_min;   /* Eq. 11 */
    double eps;     /* relative band (in units of T) for count_lo / count_hi */
    double eps_ball; /* relative band of the ball boundary |d|^2 = r_nbr^2 */
} oracle_reduce;

/* Activate, filter and form Sigma for n Gaussians (float inputs, as stored).
 * raw_mode: scales are log-scales and opacity is a logit.
 * Outputs for the n_kept survivors, in input order: kept_index (nullable),
 * mu (n_kept x 3) and sigma (n_kept x 9, row-major). */
int oracle_prepare_scene(int64_t n, const float *means, const float *quats,
                         const float *scales, const float *opacity, int raw_mode,
                         double alpha_f, double extent_f, int64_t *n_kept,
                         int64_t *kept_index, double *mu, double *sigma);

/* Evaluate q robot bodies (centres q x 3, body matrices A q x 9) against the
 * n prepared Gaussians for m conservatism values.  Every output is q x m
 * (query-major) except nbr, nbr_lo, nbr_hi (q); any output pointer may be
 * NULL. */
int oracle_eval(int64_t n, const double *mu, const double *sigma, int64_t q,
                const double *centers, const double *A, int32_t m,
                const double *n_sigma, const oracle_reduce *o, int32_t *count,
                uint8_t *label, double *dmin, double *softmin, double *cost,
                int64_t *nbr, int64_t *nbr_lo, int64_t *nbr_hi,
                int32_t *count_lo, int32_t *count_hi,
                uint8_t *ambiguous, double *tstar, double *tsoft, double *tcost,
                int nthreads);

#ifdef __cplusplus
}
#endif

#endif
