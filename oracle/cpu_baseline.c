/* FP64 Chebyshev low-pass filter of a signal block over a CSR graph, in plain
 * C with OpenMP over rows.  TEST INFRASTRUCTURE ONLY: the CPU baseline that the
 * bench times on the host cores, checked against the NumPy oracle.  It shares
 * no code with the HIP library.
 *
 * Computes Y = sum_{j=0..p} a_j T_j(Lt) R with Lt = (2/lmax) L - I,
 * L = S - W (Sec. 2.1), by T_0 = R, T_1 = Lt R, T_{j+1} = 2 Lt T_j - T_{j-1}
 * (the fast filter of Sec. 2.4 in the Chebyshev basis).  Row-major n x r.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* out = Lt x (scale 1) or 2 Lt x - prev (scale 2) */
static void apply(int64_t n, const int32_t *rp, const int32_t *ci, const double *w,
                  const double *s, double lmax, const double *x, const double *prev,
                  double *out, int64_t r, int two)
{
#pragma omp parallel for schedule(dynamic, 256)
    for (int64_t i = 0; i < n; i++) {
        double o[r];   /* row of L x; out may alias prev, so it is written last */
        const double *xi = x + i * r;
        for (int64_t c = 0; c < r; c++) o[c] = s[i] * xi[c];
        for (int32_t e = rp[i]; e < rp[i + 1]; e++) {
            const double we = w ? w[e] : 1.0;
            const double *xk = x + (int64_t)ci[e] * r;
            for (int64_t c = 0; c < r; c++) o[c] -= we * xk[c];
        }
        for (int64_t c = 0; c < r; c++) {
            double v = (2.0 / lmax) * o[c] - xi[c];
            out[i * r + c] = two ? 2.0 * v - prev[i * r + c] : v;
        }
    }
}

int oracle_cheb_filter(int64_t n, const int32_t *rp, const int32_t *ci, const double *w,
                       double lmax, const double *a, int p, const double *R, int64_t r,
                       double *Y)
{
    double *s = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    double *t0 = (double *)malloc(sizeof(double) * (size_t)(n * r > 0 ? n * r : 1));
    double *t1 = (double *)malloc(sizeof(double) * (size_t)(n * r > 0 ? n * r : 1));
    if (!s || !t0 || !t1) { free(s); free(t0); free(t1); return 1; }
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; i++) {
        double acc = 0.0;
        for (int32_t e = rp[i]; e < rp[i + 1]; e++) acc += w ? w[e] : 1.0;
        s[i] = acc;
    }
#pragma omp parallel for schedule(static)
    for (int64_t q = 0; q < n * r; q++) { t0[q] = R[q]; Y[q] = a[0] * R[q]; }
    double *prev = t0, *cur = t1;
    if (p >= 1) {
        apply(n, rp, ci, w, s, lmax, prev, NULL, cur, r, 0);
#pragma omp parallel for schedule(static)
        for (int64_t q = 0; q < n * r; q++) Y[q] += a[1] * cur[q];
    }
    for (int j = 1; j < p; j++) {
        /* T_{j+1} overwrites T_{j-1}: row i of prev is read only by row i */
        apply(n, rp, ci, w, s, lmax, cur, prev, prev, r, 1);
        double *tmp = prev; prev = cur; cur = tmp;
#pragma omp parallel for schedule(static)
        for (int64_t q = 0; q < n * r; q++) Y[q] += a[j + 1] * cur[q];
    }
    free(s); free(t0); free(t1);
    return 0;
}

/* <x, y>_F of two n x r row-major blocks */
static double dot_block(int64_t nr, const double *x, const double *y)
{
    double acc = 0.0;
#pragma omp parallel for schedule(static) reduction(+:acc)
    for (int64_t q = 0; q < nr; q++) acc += x[q] * y[q];
    return acc;
}

/* Moments of the eigenvalue count (Sec. 3.2): mu_j = <R, T_j(Lt) R>_F for
 * j = 0..p, by the same three-term recurrence as the filter above. */
int oracle_cheb_moments(int64_t n, const int32_t *rp, const int32_t *ci, const double *w,
                        double lmax, int p, const double *R, int64_t r, double *mu)
{
    double *s = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    double *t0 = (double *)malloc(sizeof(double) * (size_t)(n * r > 0 ? n * r : 1));
    double *t1 = (double *)malloc(sizeof(double) * (size_t)(n * r > 0 ? n * r : 1));
    if (!s || !t0 || !t1) { free(s); free(t0); free(t1); return 1; }
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; i++) {
        double acc = 0.0;
        for (int32_t e = rp[i]; e < rp[i + 1]; e++) acc += w ? w[e] : 1.0;
        s[i] = acc;
    }
    memcpy(t0, R, sizeof(double) * (size_t)(n * r));
    mu[0] = dot_block(n * r, R, t0);
    double *prev = t0, *cur = t1;
    if (p >= 1) {
        apply(n, rp, ci, w, s, lmax, prev, NULL, cur, r, 0);
        mu[1] = dot_block(n * r, R, cur);
    }
    for (int j = 1; j < p; j++) {
        apply(n, rp, ci, w, s, lmax, cur, prev, prev, r, 1);
        double *tmp = prev; prev = cur; cur = tmp;
        mu[j + 1] = dot_block(n * r, R, cur);
    }
    free(s); free(t0); free(t1);
    return 0;
}

int oracle_num_threads(void)
{
    int t = 1;
#pragma omp parallel
    {
#pragma omp single
        {
#ifdef _OPENMP
            extern int omp_get_num_threads(void);
            t = omp_get_num_threads();
#endif
        }
    }
    return t;
}

/* Sets the number of OpenMP threads used by the next calls (0 or less keeps it). */
void oracle_set_threads(int t)
{
#ifdef _OPENMP
    extern void omp_set_num_threads(int);
    if (t > 0) omp_set_num_threads(t);
#else
    (void)t;
#endif
}
