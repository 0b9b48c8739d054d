/* Oracle stage 5 of Algorithm 1 in plain C + OpenMP, FP64, libm exp/sqrt.
 *
 * TEST INFRASTRUCTURE ONLY: used to time the oracle on host cores and as a second
 * evaluation of stage 5 inside the oracle.  Not part of the product path.
 *
 * Paper passage: Sec. 4.4.2, Algorithm 1, stage 5: Z'_k = sum_l Gamma(x_k, x_l) Y'_l,
 * the kernel entries computed on the fly, several rows in parallel (one row per
 * iteration of the parallel loop here).  Kernel formulas as in oracle/covariance.py.
 *
 * Layout: X is n x d row-major (point-major), Y and Z are n x b row-major.
 * kind: 0 exp, 1 sqexp, 2 exp_l1, 3 const, 4 lin.
 */
#include <math.h>
#include <omp.h>
#include <stdint.h>

/* Rows [r0, r1) of Z' only (Z holds r1 - r0 rows), on `nthreads` threads (0 = the
 * OpenMP default): a bounded sample of the same work for timing on host cores. */
int oracle_stage5_rows(int d, int64_t n, const double *X, int b, const double *Y,
                       int kind, double sigma2, const double *ell, int64_t r0, int64_t r1,
                       int nthreads, double *Z)
{
    if (d < 1 || d > 3 || n < 0 || b < 1 || r0 < 0 || r1 > n || r0 > r1) return -1;
    double inv[3] = {1.0, 1.0, 1.0};
    for (int k = 0; k < d; ++k) inv[k] = 1.0 / ell[k];
    if (nthreads <= 0) nthreads = omp_get_max_threads();
#pragma omp parallel for schedule(dynamic, 16) num_threads(nthreads)
    for (int64_t i = r0; i < r1; ++i) {
        double *zi = Z + (i - r0) * b;
        for (int j = 0; j < b; ++j) zi[j] = 0.0;
        for (int64_t l = 0; l < n; ++l) {
            double g;
            if (kind == 0 || kind == 1) {
                double r2 = 0.0;
                for (int k = 0; k < d; ++k) {
                    double t = (X[i * d + k] - X[l * d + k]) * inv[k];
                    r2 += t * t;
                }
                g = sigma2 * (kind == 0 ? exp(-sqrt(r2)) : exp(-r2));
            } else if (kind == 2) {
                double s = 0.0;
                for (int k = 0; k < d; ++k) s += fabs(X[i * d + k] - X[l * d + k]) * inv[k];
                g = sigma2 * exp(-s);
            } else if (kind == 3) {
                g = sigma2;
            } else {
                double s = 1.0;
                for (int k = 0; k < d; ++k) s += X[i * d + k] * X[l * d + k];
                g = sigma2 * s;
            }
            const double *yl = Y + l * b;
            for (int j = 0; j < b; ++j) zi[j] += g * yl[j];
        }
    }
    return 0;
}

int oracle_stage5(int d, int64_t n, const double *X, int b, const double *Y,
                  int kind, double sigma2, const double *ell, double *Z)
{
    return oracle_stage5_rows(d, n, X, b, Y, kind, sigma2, ell, 0, n, 0, Z);
}
