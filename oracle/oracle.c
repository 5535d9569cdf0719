/*
 * FP64 CPU oracle for the CollisionSplatting robot-versus-3DGS metric.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path links, loads or
 * calls this file; only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark do.  It shares no code, header or constant generator
 * with the HIP library.
 *
 * It is the method written out plainly, pair by pair, in double precision,
 * with no blocking, culling or reordering:
 *
 *   Sec. II-A, Eq. 2    Sigma_i = R_i S_i S_i^T R_i^T, R from the (w,x,y,z)
 *                       unit quaternion, S_i = diag(scales).
 *   Sec. II-B, Eq. 5-6  s^2_ij = (mu_i - c_j)^T A_j (mu_i - c_j) with
 *                       A_j = R_E diag(1/a^2, 1/b^2, 1/c^2) R_E^T
 *                       (a sphere of radius r is A = I / r^2).
 *   Sec. II-B, Eq. 7    sigma^2_ij = g^T Sigma_i g with g the gradient of
 *                       s^2 at X = mu_i, i.e. g = 2 A_j (mu_i - c_j).
 *   Sec. II-B, Eq. 8    s~^2_ij = max(0, s^2_ij - n_sigma sqrt(sigma^2_ij)).
 *   Sec. II-B, end      the collision state of a link: numerically stable
 *                       softmin of s~^2 over the splats (log-sum-exp about
 *                       the minimum, temperature tau; tau = 0 is the min).
 *   Sec. II-C           floater filter: drop splats that are both of low
 *                       opacity (alpha < alpha_f) and large (max scale > e_f).
 *   Sec. II-D, Eq. 11   per-splat cost d_max exp(-gamma max(s~^2 - s_min, 0)),
 *                       averaged over the neighbouring splats.
 *   Sec. II-E           label: in collision iff more than k splats have
 *                       s~^2 < 1 (strict).
 *
 * Readings where the paper is silent: the neighbourhood of a query is the
 * ball ||mu_i - c_j|| <= r_nbr (r_nbr = +inf: every kept splat); the count,
 * min, softmin and cost all run over that ball; an empty ball gives
 * min = softmin = +inf and cost = 0.
 *
 * Diagnostics for tolerances: per pair T_ij = s^2 + n_sigma sqrt(sigma^2),
 * the magnitude before the cancellation in Eq. 8.  count_lo counts pairs with
 * s~^2 < 1 - eps T_ij that lie inside the ball by more than eps_ball
 * (|d|^2 <= r_nbr^2 (1 - eps_ball)); count_hi counts pairs with
 * s~^2 < 1 + eps T_ij and |d|^2 <= r_nbr^2 (1 + eps_ball).  A query is
 * ambiguous iff the labels of count_lo and count_hi differ.  nbr_lo / nbr_hi
 * bracket the ball size the same way.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#include "oracle.h"

/* Rotation matrix of a unit quaternion (w, x, y, z), Hamilton convention,
 * row-major: R maps the Gaussian's local frame to the world frame. */
static void quat_to_matrix(double w, double x, double y, double z, double R[9])
{
    R[0] = 1.0 - 2.0 * (y * y + z * z);
    R[1] = 2.0 * (x * y - w * z);
    R[2] = 2.0 * (x * z + w * y);
    R[3] = 2.0 * (x * y + w * z);
    R[4] = 1.0 - 2.0 * (x * x + z * z);
    R[5] = 2.0 * (y * z - w * x);
    R[6] = 2.0 * (x * z - w * y);
    R[7] = 2.0 * (y * z + w * x);
    R[8] = 1.0 - 2.0 * (x * x + y * y);
}

int oracle_prepare_scene(int64_t n, const float *means, const float *quats,
                         const float *scales, const float *opacity, int raw_mode,
                         double alpha_f, double extent_f, int64_t *n_kept,
                         int64_t *kept_index, double *mu, double *sigma)
{
    if (n < 0)
        return ORACLE_E_INVALID;
    /* validate everything first: nothing is written on error */
    for (int64_t i = 0; i < n; ++i) {
        for (int k = 0; k < 3; ++k)
            if (!isfinite(means[3 * i + k]) || !isfinite(scales[3 * i + k]))
                return ORACLE_E_INVALID;
        if (!raw_mode)
            for (int k = 0; k < 3; ++k)
                if (scales[3 * i + k] < 0.0f)
                    return ORACLE_E_INVALID;
        double nq = 0.0;
        for (int k = 0; k < 4; ++k) {
            if (!isfinite(quats[4 * i + k]))
                return ORACLE_E_INVALID;
            nq += (double)quats[4 * i + k] * (double)quats[4 * i + k];
        }
        if (nq == 0.0 || !isfinite(opacity[i]))
            return ORACLE_E_INVALID;
    }
    int64_t kept = 0;
    for (int64_t i = 0; i < n; ++i) {
        double s[3], alpha;
        for (int k = 0; k < 3; ++k)
            s[k] = raw_mode ? exp((double)scales[3 * i + k]) : (double)scales[3 * i + k];
        alpha = raw_mode ? 1.0 / (1.0 + exp(-(double)opacity[i])) : (double)opacity[i];
        /* Sec. II-C floater filter (disabled when alpha_f <= 0) */
        double smax = fmax(s[0], fmax(s[1], s[2]));
        if (alpha_f > 0.0 && alpha < alpha_f && smax > extent_f)
            continue;
        double w = quats[4 * i + 0], x = quats[4 * i + 1], y = quats[4 * i + 2], z = quats[4 * i + 3];
        double nq = sqrt(w * w + x * x + y * y + z * z);
        double R[9];
        quat_to_matrix(w / nq, x / nq, y / nq, z / nq, R);
        /* Eq. 2: Sigma = R diag(s^2) R^T, formed explicitly */
        double *S = sigma + 9 * kept;
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) {
                double acc = 0.0;
                for (int k = 0; k < 3; ++k)
                    acc += R[3 * a + k] * (s[k] * s[k]) * R[3 * b + k];
                S[3 * a + b] = acc;
            }
        for (int k = 0; k < 3; ++k)
            mu[3 * kept + k] = (double)means[3 * i + k];
        if (kept_index)
            kept_index[kept] = i;
        ++kept;
    }
    *n_kept = kept;
    return ORACLE_OK;
}

/* Neumaier's compensated summation. */
typedef struct {
    double s, c;
} nsum;

static void nsum_add(nsum *a, double v)
{
    double t = a->s + v;
    if (fabs(a->s) >= fabs(v))
        a->c += (a->s - t) + v;
    else
        a->c += (v - t) + a->s;
    a->s = t;
}

static double nsum_get(const nsum *a) { return a->s + a->c; }

static double quad3(const double *M, const double *u, const double *v)
{
    double acc = 0.0;
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b)
            acc += u[a] * M[3 * a + b] * v[b];
    return acc;
}

int oracle_eval(int64_t n, const double *mu, const double *sigma, int64_t q,
                const double *centers, const double *A, int32_t m,
                const double *n_sigma, const oracle_reduce *o, int32_t *count,
                uint8_t *label, double *dmin, double *softmin, double *cost,
                int64_t *nbr, int64_t *nbr_lo, int64_t *nbr_hi,
                int32_t *count_lo, int32_t *count_hi,
                uint8_t *ambiguous, double *tstar, double *tsoft, double *tcost,
                int nthreads)
{
    if (n < 0 || q < 0 || m < 1 || m > ORACLE_MAX_M || !o)
        return ORACLE_E_INVALID;
    for (int v = 0; v < m; ++v)
        if (!(n_sigma[v] >= 0.0) || !isfinite(n_sigma[v]))
            return ORACLE_E_INVALID;
    if (o->k < 0 || !(o->tau >= 0.0) || !(o->r_nbr > 0.0) || !(o->gamma >= 0.0))
        return ORACLE_E_INVALID;
    const double r2nbr = isinf(o->r_nbr) ? INFINITY : o->r_nbr * o->r_nbr;
    /* ball membership within eps_ball of the boundary is a rounding-level call */
    const double r2lo = isinf(o->r_nbr) ? INFINITY : r2nbr * (1.0 - o->eps_ball);
    const double r2hi = isinf(o->r_nbr) ? INFINITY : r2nbr * (1.0 + o->eps_ball);
    int err = 0;

#ifdef _OPENMP
    if (nthreads <= 0)
        nthreads = omp_get_max_threads();
#pragma omp parallel num_threads(nthreads)
#endif
    {
        /* per-thread scratch: s~^2 and T for every neighbouring pair */
        double *st = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1) * (size_t)m);
        double *tt = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1) * (size_t)m);
        unsigned char *bb = (unsigned char *)malloc((size_t)(n > 0 ? n : 1));
        if (!st || !tt || !bb) {
#ifdef _OPENMP
#pragma omp atomic write
#endif
            err = 1;
        }
#ifdef _OPENMP
#pragma omp for schedule(static)
#endif
        for (int64_t j = 0; j < q; ++j) {
            if (!st || !tt || !bb)
                continue;
            const double *c = centers + 3 * j;
            const double *Aj = A + 9 * j;
            int64_t nn = 0, nlo = 0, nhi = 0, nin = 0;
            for (int64_t i = 0; i < n; ++i) {
                double d[3] = {mu[3 * i] - c[0], mu[3 * i + 1] - c[1], mu[3 * i + 2] - c[2]};
                double dd = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
                if (!(dd <= r2hi))
                    continue; /* outside the neighbourhood ball (and its band) */
                /* bit 0: in the ball; bit 1: in for certain; bit 2: in the upper band */
                bb[nn] = (unsigned char)((dd <= r2nbr) | ((dd <= r2lo) << 1) | 4);
                nin += dd <= r2nbr;
                nlo += dd <= r2lo;
                nhi += 1;
                double s2 = quad3(Aj, d, d); /* Eq. 5 at X = mu_i */
                double g[3];                 /* gradient of s^2 at X = mu_i */
                for (int a = 0; a < 3; ++a)
                    g[a] = 2.0 * (Aj[3 * a] * d[0] + Aj[3 * a + 1] * d[1] + Aj[3 * a + 2] * d[2]);
                double var = quad3(sigma + 9 * i, g, g); /* Eq. 7 */
                double sd = sqrt(var > 0.0 ? var : 0.0);
                for (int v = 0; v < m; ++v) {
                    double red = s2 - n_sigma[v] * sd; /* Eq. 8 */
                    st[(size_t)v * n + nn] = red > 0.0 ? red : 0.0;
                    tt[(size_t)v * n + nn] = s2 + n_sigma[v] * sd;
                }
                ++nn;
            }
            if (nbr)
                nbr[j] = nin;
            if (nbr_lo)
                nbr_lo[j] = nlo;
            if (nbr_hi)
                nbr_hi[j] = nhi;
            /* count diagnostics over the candidates of the widened ball */
            int64_t cand = nn;
            for (int v = 0; v < m; ++v) {
                const double *x = st + (size_t)v * n;
                const double *T = tt + (size_t)v * n;
                int64_t clo = 0, chi = 0;
                for (int64_t i = 0; i < cand; ++i) {
                    clo += (bb[i] & 2) && x[i] < 1.0 - o->eps * T[i];
                    chi += x[i] < 1.0 + o->eps * T[i];
                }
                if (count_lo)
                    count_lo[(size_t)j * m + v] = (int32_t)clo;
                if (count_hi)
                    count_hi[(size_t)j * m + v] = (int32_t)chi;
                if (ambiguous)
                    ambiguous[(size_t)j * m + v] = (clo > o->k) != (chi > o->k);
            }
            /* keep the pairs of the ball itself, in order, for the reductions */
            nn = 0;
            for (int64_t i = 0; i < cand; ++i) {
                if (!(bb[i] & 1))
                    continue;
                for (int v = 0; v < m; ++v) {
                    st[(size_t)v * n + nn] = st[(size_t)v * n + i];
                    tt[(size_t)v * n + nn] = tt[(size_t)v * n + i];
                }
                ++nn;
            }
            for (int v = 0; v < m; ++v) {
                const double *x = st + (size_t)v * n;
                const double *T = tt + (size_t)v * n;
                int64_t cnt = 0;
                double mn = INFINITY;
                for (int64_t i = 0; i < nn; ++i) {
                    cnt += x[i] < 1.0;
                    if (x[i] < mn)
                        mn = x[i];
                }
                /* largest T among pairs whose value lies within the tolerance band
                 * of the minimum: any of them may be the minimiser under rounding */
                double tb = 1.0;
                for (int64_t i = 0; i < nn; ++i)
                    if (x[i] - mn <= o->eps * T[i] && T[i] > tb)
                        tb = T[i];
                double sm = mn, ts = tb;
                if (nn > 0 && o->tau > 0.0) {
                    nsum acc = {0.0, 0.0}, wt = {0.0, 0.0};
                    for (int64_t i = 0; i < nn; ++i) {
                        double e = exp(-(x[i] - mn) / o->tau);
                        nsum_add(&acc, e);
                        nsum_add(&wt, e * T[i]);
                    }
                    double S = nsum_get(&acc);
                    sm = mn - o->tau * log(S);
                    ts = fmax(tb, nsum_get(&wt) / S);
                }
                double cs = 0.0, tc = 1.0;
                if (nn > 0) {
                    nsum acc = {0.0, 0.0}, wt = {0.0, 0.0};
                    for (int64_t i = 0; i < nn; ++i) {
                        double ex = x[i] - o->s_min;
                        double e = o->d_max * exp(-o->gamma * (ex > 0.0 ? ex : 0.0)); /* Eq. 11 */
                        nsum_add(&acc, e);
                        nsum_add(&wt, e * T[i]);
                    }
                    double S = nsum_get(&acc);
                    cs = S / (double)nn;
                    tc = S > 0.0 ? fmax(1.0, nsum_get(&wt) / S) : 1.0;
                }
                size_t oi = (size_t)j * m + v;
                if (count)
                    count[oi] = (int32_t)cnt;
                if (label)
                    label[oi] = cnt > o->k;
                if (dmin)
                    dmin[oi] = mn;
                if (softmin)
                    softmin[oi] = sm;
                if (cost)
                    cost[oi] = cs;
                if (tstar)
                    tstar[oi] = tb;
                if (tsoft)
                    tsoft[oi] = ts;
                if (tcost)
                    tcost[oi] = tc;
            }
        }
        free(st);
        free(tt);
        free(bb);
    }
    return err ? ORACLE_E_OOM : ORACLE_OK;
}
