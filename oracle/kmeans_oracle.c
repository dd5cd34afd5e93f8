/*
 * kmeans_oracle.c -- plain FP64 CPU oracle for Lloyd's K-means iteration.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the library path may call, link or
 * load this file: only the tests, the smoke check and the CPU-baseline leg of
 * the benchmark use it.  It shares no code, header or constant with the GPU
 * path.
 *
 * It writes out the definitions of the paper's section "The Lloyd's
 * Algorithm" and the error test of "Serial Lloyd's Algorithm":
 *   reassignment  z_i^{t+1} = argmin_k ||x_i - mu_k^t||_2^2
 *   mean          mu_k^{t+1} = sum_i 1(z_i^{t+1}=k) x_i / sum_i 1(z_i^{t+1}=k)
 *   error         E = sum_k ||mu_k^{t+1} - mu_k^t||_2^2, iterate while E >= tol
 * in float64, with float32 inputs widened exactly.  Readings where the paper
 * is silent:
 *   - ties in the argmin go to the lowest cluster index (strict '<' scan);
 *   - an empty cluster keeps its previous centre (the paper's quotient is 0/0);
 *   - the loop stops when E < tol (strict) or after max_iter updates;
 *     T counts the updates performed;
 *   - the returned labels and objective are recomputed against the final
 *     centres, so labels and means are consistent;
 *   - with assign_f32 != 0 the distances of the reassignment step use the
 *     centres rounded to float32 (then widened exactly), i.e. the same centre
 *     values a float32 device kernel compares against; sums, means and E are
 *     always float64.
 * Labels are 0-based (the paper numbers clusters 1..K).
 *
 * The sums over points run in point order with Neumaier (compensated)
 * summation, so the result does not depend on the thread count.  OpenMP only
 * parallelises the per-point argmin, which is independent per point.
 *
 * Data layout: X is d rows of N float32, row j at X + j*ld (structure of
 * arrays, the paper's X in R^{d x N}); centres are K x d float64, row-major.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define OR_OK 0
#define OR_EINVAL (-1)
#define OR_ENOMEM (-4)

int oracle_threads(int n) {
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
    return omp_get_max_threads();
#else
    (void)n;
    return 1;
#endif
}

static int check_args(const float *X, int64_t N, int64_t ld, int d, int K,
                      const double *mu) {
    if (!X || !mu || N < 1 || ld < N || d < 1 || K < 1) return OR_EINVAL;
    return OR_OK;
}

/* Neumaier compensated accumulator. */
typedef struct { double s, c; } nsum;
static inline void nadd(nsum *a, double v) {
    double t = a->s + v;
    if (fabs(a->s) >= fabs(v)) a->c += (a->s - t) + v;
    else                       a->c += (v - t) + a->s;
    a->s = t;
}
static inline double nval(const nsum *a) { return a->s + a->c; }

/* Centre values the distance step compares against. */
static void assign_centres(const double *mu, int K, int d, int assign_f32,
                           double *out) {
    for (int i = 0; i < K * d; ++i)
        out[i] = assign_f32 ? (double)(float)mu[i] : mu[i];
}

/*
 * Reassignment step.  For every point: the squared distance to each centre in
 * float64, the first index attaining the minimum, the minimum, and the
 * smallest distance among the other centres (+inf when K == 1), which the
 * parity tests use to recognise near-ties.
 * labels, dmin, dsecond may each be NULL.
 */
int oracle_assign(const float *X, int64_t N, int64_t ld, int d, int K,
                  const double *mu, int assign_f32, int32_t *labels,
                  double *dmin, double *dsecond) {
    int rc = check_args(X, N, ld, d, K, mu);
    if (rc) return rc;
    double *m = (double *)malloc(sizeof(double) * (size_t)K * d);
    if (!m) return OR_ENOMEM;
    assign_centres(mu, K, d, assign_f32, m);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < N; ++i) {
        double best = INFINITY, second = INFINITY;
        int32_t arg = 0;
        for (int k = 0; k < K; ++k) {
            double D = 0.0;
            for (int j = 0; j < d; ++j) {
                double diff = (double)X[(int64_t)j * ld + i] - m[k * d + j];
                D += diff * diff;
            }
            if (D < best) {
                second = best;
                best = D;
                arg = k;
            } else if (D < second) {
                second = D;
            }
        }
        if (labels) labels[i] = arg;
        if (dmin) dmin[i] = best;
        if (dsecond) dsecond[i] = second;
    }
    free(m);
    return OR_OK;
}

/*
 * Mean-calculation step for given labels: per-cluster counts and sums of the
 * points, the new centres (an empty cluster keeps mu_t), and
 * E = sum_k ||mu_next_k - mu_t_k||^2.  counts, sums, E, empty may be NULL.
 */
int oracle_update(const float *X, int64_t N, int64_t ld, int d, int K,
                  const int32_t *labels, const double *mu_t, int64_t *counts,
                  double *sums, double *mu_next, double *E, int64_t *empty) {
    int rc = check_args(X, N, ld, d, K, mu_t);
    if (rc) return rc;
    if (!labels || !mu_next) return OR_EINVAL;
    nsum *S = (nsum *)calloc((size_t)K * d, sizeof(nsum));
    int64_t *n = (int64_t *)calloc((size_t)K, sizeof(int64_t));
    if (!S || !n) {
        free(S); free(n);
        return OR_ENOMEM;
    }
    for (int64_t i = 0; i < N; ++i) {
        int k = labels[i];
        if (k < 0 || k >= K) {
            free(S); free(n);
            return OR_EINVAL;
        }
        n[k] += 1;
        for (int j = 0; j < d; ++j) nadd(&S[k * d + j], (double)X[(int64_t)j * ld + i]);
    }
    int64_t n_empty = 0;
    double Eacc = 0.0;
    for (int k = 0; k < K; ++k) {
        for (int j = 0; j < d; ++j) {
            double s = nval(&S[k * d + j]);
            double v = n[k] > 0 ? s / (double)n[k] : mu_t[k * d + j];
            double sh = v - mu_t[k * d + j];
            Eacc += sh * sh;
            mu_next[k * d + j] = v;
            if (sums) sums[k * d + j] = s;
        }
        if (n[k] == 0) n_empty++;
        if (counts) counts[k] = n[k];
    }
    if (E) *E = Eacc;
    if (empty) *empty = n_empty;
    free(S); free(n);
    return OR_OK;
}

/*
 * One Lloyd update from centres mu_t: the reassignment step, then the mean
 * step on its labels, and the objective J_t = sum_i min_k D_ik of mu_t.
 * Outputs (each may be NULL except mu_next): labels[N], counts[K], sums[K*d],
 * mu_next[K*d], E, J, empty (number of clusters with no point).
 */
int oracle_step(const float *X, int64_t N, int64_t ld, int d, int K,
                const double *mu_t, int assign_f32, int32_t *labels,
                int64_t *counts, double *sums, double *mu_next, double *E,
                double *J, int64_t *empty) {
    int rc = check_args(X, N, ld, d, K, mu_t);
    if (rc) return rc;
    if (!mu_next) return OR_EINVAL;
    int32_t *z = (int32_t *)malloc(sizeof(int32_t) * (size_t)N);
    double *dm = (double *)malloc(sizeof(double) * (size_t)N);
    if (!z || !dm) {
        free(z); free(dm);
        return OR_ENOMEM;
    }
    oracle_assign(X, N, ld, d, K, mu_t, assign_f32, z, dm, NULL);
    rc = oracle_update(X, N, ld, d, K, z, mu_t, counts, sums, mu_next, E, empty);
    if (!rc) {
        nsum Jacc = {0.0, 0.0};
        for (int64_t i = 0; i < N; ++i) nadd(&Jacc, dm[i]);
        if (J) *J = nval(&Jacc);
        if (labels) memcpy(labels, z, sizeof(int32_t) * (size_t)N);
    }
    free(z); free(dm);
    return rc;
}

/*
 * Lloyd's algorithm from mu0 until E < tol or max_iter updates.
 * Outputs: mu_out[K*d] (final centres), labels[N] (against the final centres,
 * may be NULL), *T (updates performed), *E_last (E of the last update),
 * *J_final (objective of the final centres), *converged (E_last < tol),
 * E_hist/J_hist[max_iter] (E_t and J_t per update, may be NULL),
 * *empty_events (sum over updates of the number of empty clusters).
 */
int oracle_fit(const float *X, int64_t N, int64_t ld, int d, int K,
               const double *mu0, double tol, int max_iter, int assign_f32,
               double *mu_out, int32_t *labels, int *T, double *E_last,
               double *J_final, int *converged, double *E_hist,
               double *J_hist, int64_t *empty_events) {
    int rc = check_args(X, N, ld, d, K, mu0);
    if (rc) return rc;
    if (!mu_out || max_iter < 1 || !(tol >= 0.0)) return OR_EINVAL;
    size_t kd = (size_t)K * d;
    double *cur = (double *)malloc(sizeof(double) * kd);
    double *nxt = (double *)malloc(sizeof(double) * kd);
    double *dm = (double *)malloc(sizeof(double) * (size_t)N);
    if (!cur || !nxt || !dm) {
        free(cur); free(nxt); free(dm);
        return OR_ENOMEM;
    }
    memcpy(cur, mu0, sizeof(double) * kd);
    int t = 0;
    double E = INFINITY;
    int64_t ev = 0;
    while (t < max_iter) {
        double Jt = 0.0;
        int64_t emp = 0;
        rc = oracle_step(X, N, ld, d, K, cur, assign_f32, NULL, NULL, NULL, nxt,
                         &E, &Jt, &emp);
        if (rc) break;
        if (E_hist) E_hist[t] = E;
        if (J_hist) J_hist[t] = Jt;
        ev += emp;
        memcpy(cur, nxt, sizeof(double) * kd);
        t += 1;
        if (E < tol) break;
    }
    if (!rc) {
        nsum Jacc = {0.0, 0.0};
        oracle_assign(X, N, ld, d, K, cur, assign_f32, labels, dm, NULL);
        for (int64_t i = 0; i < N; ++i) nadd(&Jacc, dm[i]);
        memcpy(mu_out, cur, sizeof(double) * kd);
        if (T) *T = t;
        if (E_last) *E_last = E;
        if (J_final) *J_final = nval(&Jacc);
        if (converged) *converged = (E < tol) ? 1 : 0;
        if (empty_events) *empty_events = ev;
    }
    free(cur); free(nxt); free(dm);
    return rc;
}
