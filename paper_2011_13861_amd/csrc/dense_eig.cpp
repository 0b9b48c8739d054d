// Dense symmetric eigensolver for the Rayleigh-Ritz step (host, FP64).
//
// Householder reduction to tridiagonal form, then implicit symmetric QR steps with the
// Wilkinson shift (Golub and Van Loan, Matrix Computations, Sec. 8.3), accumulating
// every reflection and rotation so that A = Z diag(w) Z^T.  Matrices are small (the
// projected operator of the block eigensolver, n <= a few hundred).
#include <algorithm>
#include <cmath>
#include <limits>
#include <numeric>
#include <vector>

#include "kl_internal.h"

namespace kl {

namespace {

// Host kernels are built for the baseline x86-64 target and for x86-64-v3 (AVX2, FMA); the
// loader picks the clone the CPU supports.
#define KL_HOST_CLONES __attribute__((target_clones("arch=x86-64-v3", "default")))

// Householder reduction a <- H a H to tridiagonal form (d diagonal, e sub-diagonal);
// reflector k is I - beta[k] v_k v_k^T acting on rows / columns k+1..n-1, with v_k stored
// in row k of V.  Only the lower triangle of the working copy is read and updated: the
// symmetric product p = A22 v takes each off-diagonal entry twice (a dot product and an
// axpy along its row) and the rank-2 update touches j <= i only.
KL_HOST_CLONES
void tridiagonalise_raw(int n, double *a, double *d, double *e, double *V, double *beta, double *p, double *q) {
    for (int k = 0; k + 2 < n; ++k) {
        const int m = n - k - 1;
        double *v = V + size_t(k) * n;
        double nrm2 = 0.0;
        for (int i = 0; i < m; ++i) {
            v[i] = a[size_t(k + 1 + i) * n + k];
            nrm2 += v[i] * v[i];
        }
        d[k] = a[size_t(k) * n + k];
        if (nrm2 == 0.0) { e[k] = 0.0; beta[k] = 0.0; continue; }
        const double nrm = std::sqrt(nrm2);
        const double alpha = v[0] > 0 ? -nrm : nrm;
        v[0] -= alpha;
        double vv = 0.0;
#pragma omp simd reduction(+ : vv)
        for (int i = 0; i < m; ++i) vv += v[i] * v[i];
        const double b = 2.0 / vv;
        beta[k] = b;
        e[k] = alpha;
        // p = A22 v from the lower triangle (row i of A22 is a + (k+1+i) n + k+1, entries j <= i)
        for (int i = 0; i < m; ++i) p[i] = 0.0;
        for (int i = 0; i < m; ++i) {
            const double *row = a + size_t(k + 1 + i) * n + k + 1;
            const double vi = v[i];
            double s = row[i] * vi;
#pragma omp simd reduction(+ : s)
            for (int j = 0; j < i; ++j) {
                s += row[j] * v[j];
                p[j] += row[j] * vi;
            }
            p[i] += s;
        }
        double pv = 0.0;
#pragma omp simd reduction(+ : pv)
        for (int i = 0; i < m; ++i) {
            p[i] *= b;
            pv += p[i] * v[i];
        }
        // q = p - (b/2)(p.v) v,  A22 -= v q^T + q v^T  (lower triangle)
        const double K = 0.5 * b * pv;
        for (int i = 0; i < m; ++i) q[i] = p[i] - K * v[i];
        for (int i = 0; i < m; ++i) {
            double *row = a + size_t(k + 1 + i) * n + k + 1;
            const double vi = v[i], qi = q[i];
            for (int j = 0; j <= i; ++j) row[j] -= vi * q[j] + qi * v[j];
        }
    }
    if (n >= 2) {
        d[n - 2] = a[size_t(n - 2) * n + (n - 2)];
        e[n - 2] = a[size_t(n - 1) * n + (n - 2)];
    }
    d[n - 1] = a[size_t(n - 1) * n + (n - 1)];
    e[n - 1] = 0.0;
}

void tridiagonalise(int n, const double *A, std::vector<double> &d, std::vector<double> &e,
                    std::vector<double> &V, std::vector<double> &beta) {
    std::vector<double> a(A, A + size_t(n) * n);     // working copy, row-major (lower triangle used)
    d.assign(n, 0.0);
    e.assign(n, 0.0);
    V.assign(size_t(n) * n, 0.0);
    beta.assign(n, 0.0);
    std::vector<double> p(n), q(n);
    tridiagonalise_raw(n, a.data(), d.data(), e.data(), V.data(), beta.data(), p.data(), q.data());
}

// X (n x nv, column-major) <- H_0 H_1 ... H_{n-3} X.  With from_identity, X starts as the
// identity, whose columns j <= k are untouched by reflector k and are skipped.
KL_HOST_CLONES
void apply_reflectors_raw(int n, int nv, const double *V, const double *beta, double *X, bool from_identity) {
    for (int k = n - 3; k >= 0; --k) {
        if (beta[k] == 0.0) continue;
        const int m = n - k - 1;
        const double *v = V + size_t(k) * n;
        for (int j = from_identity ? k + 1 : 0; j < nv; ++j) {
            double *col = X + size_t(j) * n + k + 1;
            double s = 0.0;
#pragma omp simd reduction(+ : s)
            for (int i = 0; i < m; ++i) s += v[i] * col[i];
            s *= beta[k];
            for (int i = 0; i < m; ++i) col[i] -= s * v[i];
        }
    }
}

void apply_reflectors(int n, int nv, const std::vector<double> &V, const std::vector<double> &beta, double *X,
                      bool from_identity) {
    apply_reflectors_raw(n, nv, V.data(), beta.data(), X, from_identity);
}
}  // namespace

// A: n x n symmetric, row-major (read only).  w: eigenvalues, descending.
// Z: column-major n x n, column j = unit eigenvector of w[j].  Returns false if the QR
// iteration does not converge.
bool sym_eig(int n, const double *A, double *w, double *Z) {
    if (n <= 0) return true;
    std::vector<double> d, e, V, beta;
    tridiagonalise(n, A, d, e, V, beta);
    // ---- accumulate Q = H_0 H_1 ... H_{n-3}, column-major in Z ------------------------
    for (size_t i = 0; i < size_t(n) * n; ++i) Z[i] = 0.0;
    for (int i = 0; i < n; ++i) Z[size_t(i) * n + i] = 1.0;
    apply_reflectors(n, n, V, beta, Z, true);
    // ---- implicit symmetric QR with Wilkinson shift -------------------------------------
    const double eps = std::numeric_limits<double>::epsilon();
    int h = n - 1, iter = 0;
    while (h > 0) {
        if (std::fabs(e[h - 1]) <= eps * (std::fabs(d[h - 1]) + std::fabs(d[h]))) {
            e[h - 1] = 0.0;
            --h;
            iter = 0;
            continue;
        }
        if (++iter > 60) return false;
        int l = h - 1;
        while (l > 0 && std::fabs(e[l - 1]) > eps * (std::fabs(d[l - 1]) + std::fabs(d[l]))) --l;
        const double delta = 0.5 * (d[h - 1] - d[h]);
        const double eh = e[h - 1];
        const double sg = delta >= 0 ? 1.0 : -1.0;
        const double mu = d[h] - eh * eh / (delta + sg * std::hypot(delta, eh));
        double x = d[l] - mu, z = e[l];
        for (int k = l; k < h; ++k) {
            const double r = std::sqrt(x * x + z * z);      // |x|, |z| ~ ||T||: no overflow
            const double c = r > 0 ? x / r : 1.0;
            const double s = r > 0 ? -z / r : 0.0;
            if (k > l) e[k - 1] = r;
            const double ak = d[k], bk = e[k], ck = d[k + 1];
            d[k] = ak * c * c - 2.0 * bk * c * s + ck * s * s;
            d[k + 1] = ak * s * s + 2.0 * bk * c * s + ck * c * c;
            e[k] = (ak - ck) * c * s + bk * (c * c - s * s);
            if (k + 1 < h) {
                z = -s * e[k + 1];
                e[k + 1] = c * e[k + 1];
                x = e[k];
            }
            double *zk = &Z[size_t(k) * n], *zk1 = &Z[size_t(k + 1) * n];
            for (int i = 0; i < n; ++i) {
                const double u = zk[i], t = zk1[i];
                zk[i] = c * u - s * t;
                zk1[i] = s * u + c * t;
            }
        }
    }
    // ---- sort descending --------------------------------------------------------------
    std::vector<int> order(n);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](int i, int j) { return d[i] > d[j]; });
    std::vector<double> Zs(size_t(n) * n);
    for (int j = 0; j < n; ++j) {
        w[j] = d[order[j]];
        std::copy(&Z[size_t(order[j]) * n], &Z[size_t(order[j]) * n] + n, &Zs[size_t(j) * n]);
    }
    std::copy(Zs.begin(), Zs.end(), Z);
    return true;
}

namespace {

// Eigenvalues of the symmetric tridiagonal (d, e) by implicit QR with the Wilkinson shift,
// without vectors; w receives them in descending order.
bool tridiagonal_eigenvalues(int n, std::vector<double> d, std::vector<double> e, double *w) {
    const double eps = std::numeric_limits<double>::epsilon();
    int h = n - 1, iter = 0;
    while (h > 0) {
        if (std::fabs(e[h - 1]) <= eps * (std::fabs(d[h - 1]) + std::fabs(d[h]))) {
            e[h - 1] = 0.0;
            --h;
            iter = 0;
            continue;
        }
        if (++iter > 60) return false;
        int l = h - 1;
        while (l > 0 && std::fabs(e[l - 1]) > eps * (std::fabs(d[l - 1]) + std::fabs(d[l]))) --l;
        const double delta = 0.5 * (d[h - 1] - d[h]);
        const double eh = e[h - 1];
        const double sg = delta >= 0 ? 1.0 : -1.0;
        const double mu = d[h] - eh * eh / (delta + sg * std::hypot(delta, eh));
        double x = d[l] - mu, z = e[l];
        for (int k = l; k < h; ++k) {
            const double r = std::sqrt(x * x + z * z);      // |x|, |z| ~ ||T||: no overflow
            const double c = r > 0 ? x / r : 1.0;
            const double s = r > 0 ? -z / r : 0.0;
            if (k > l) e[k - 1] = r;
            const double ak = d[k], bk = e[k], ck = d[k + 1];
            d[k] = ak * c * c - 2.0 * bk * c * s + ck * s * s;
            d[k + 1] = ak * s * s + 2.0 * bk * c * s + ck * c * c;
            e[k] = (ak - ck) * c * s + bk * (c * c - s * s);
            if (k + 1 < h) {
                z = -s * e[k + 1];
                e[k + 1] = c * e[k + 1];
                x = e[k];
            }
        }
    }
    std::sort(d.begin(), d.end(), [](double a, double b) { return a > b; });
    std::copy(d.begin(), d.end(), w);
    return true;
}

// LU factorisation with partial pivoting of the tridiagonal T - lambda I (reciprocal
// pivots rdd, multipliers dl, super-diagonals du, du2 after row interchanges; piv[i] marks
// an interchange of rows i and i + 1).  Zero pivots are replaced by `tiny`.
inline void tri_lu_factor(int n, const double *d, const double *e, double lambda, double tiny, double *rdd, double *dl,
                   double *du, double *du2, char *piv) {
    // rdd holds the pivots themselves until the end of the sweep
    for (int i = 0; i < n; ++i) { rdd[i] = d[i] - lambda; du2[i] = 0.0; piv[i] = 0; }
    for (int i = 0; i + 1 < n; ++i) { dl[i] = e[i]; du[i] = e[i]; }
    dl[n - 1] = du[n - 1] = 0.0;
    for (int i = 0; i + 1 < n; ++i) {
        if (std::fabs(rdd[i]) >= std::fabs(dl[i])) {
            if (rdd[i] == 0.0) rdd[i] = tiny;
            const double f = dl[i] / rdd[i];
            dl[i] = f;
            rdd[i + 1] -= f * du[i];
        } else {
            const double f = rdd[i] / dl[i];
            rdd[i] = dl[i];
            dl[i] = f;
            const double t = du[i];
            du[i] = rdd[i + 1];
            rdd[i + 1] = t - f * rdd[i + 1];
            if (i + 2 < n) {
                du2[i] = du[i + 1];
                du[i + 1] = -f * du[i + 1];
            }
            piv[i] = 1;
        }
    }
    if (rdd[n - 1] == 0.0) rdd[n - 1] = tiny;
    for (int i = 0; i < n; ++i) rdd[i] = 1.0 / rdd[i];
}

// x <- (T - lambda I)^{-1} x from the factors above
inline void tri_lu_solve(int n, const double *rdd, const double *dl, const double *du, const double *du2,
                         const char *piv, double *x) {
    for (int i = 0; i + 1 < n; ++i) {
        if (piv[i]) {
            const double t = x[i];
            x[i] = x[i + 1];
            x[i + 1] = t - dl[i] * x[i];
        } else {
            x[i + 1] -= dl[i] * x[i];
        }
    }
    x[n - 1] *= rdd[n - 1];
    if (n > 1) x[n - 2] = (x[n - 2] - du[n - 2] * x[n - 1]) * rdd[n - 2];
    for (int i = n - 3; i >= 0; --i) x[i] = (x[i] - du[i] * x[i + 1] - du2[i] * x[i + 2]) * rdd[i];
}

// Eigenvectors of the tridiagonal (d, e) for its nv largest eigenvalues w[0..nv-1]
// (descending) by inverse iteration: two steps from a seeded random vector (the shifts are
// eigenvalues accurate to rounding, so the second step already converges); eigenvalues
// closer than 1e-3 ||T|| form a cluster whose vectors are orthogonalised against each
// other at every step, and equal ones are separated by a tiny shift.  X: n x nv,
// column-major.  work: 5 n doubles, piv: n chars.  Returns false on a breakdown.
KL_HOST_CLONES
bool tridiagonal_vectors_raw(int n, const double *d, const double *e, const double *w, int nv, double *X,
                             double *work, char *piv) {
    const double eps = std::numeric_limits<double>::epsilon();
    double tnorm = 0.0;
    for (int i = 0; i < n; ++i)
        tnorm = std::max(tnorm, std::fabs(d[i]) + (i + 1 < n ? std::fabs(e[i]) : 0.0) + (i > 0 ? std::fabs(e[i - 1]) : 0.0));
    if (tnorm == 0.0) tnorm = 1.0;
    const double ortol = 1e-3 * tnorm, pertol = 10.0 * eps * tnorm, tiny = eps * tnorm;
    double *rdd = work, *dl = work + n, *du = work + 2 * n, *du2 = work + 3 * n;
    uint64_t state = 0x2545F4914F6CDD1Dull;
    int cs = 0;                  // first index of the current cluster
    double lam_prev = 0.0;
    for (int j = 0; j < nv; ++j) {
        double lam = w[j];
        if (j > 0 && w[j - 1] - w[j] > ortol) cs = j;
        if (j > cs && lam_prev - lam < pertol) lam = lam_prev - pertol;
        lam_prev = lam;
        tri_lu_factor(n, d, e, lam, tiny, rdd, dl, du, du2, piv);
        double *x = X + size_t(j) * n;
        for (int i = 0; i < n; ++i) {     // splitmix64 uniform on [-1, 1)
            uint64_t z = (state += 0x9E3779B97F4A7C15ull);
            z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
            z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
            z ^= z >> 31;
            x[i] = 2.0 * (double(z >> 11) * (1.0 / 9007199254740992.0)) - 1.0;
        }
        for (int it = 0; it < 2; ++it) {
            tri_lu_solve(n, rdd, dl, du, du2, piv, x);
            for (int c = cs; c < j; ++c) {
                const double *y = X + size_t(c) * n;
                double s = 0.0;
#pragma omp simd reduction(+ : s)
                for (int i = 0; i < n; ++i) s += x[i] * y[i];
#pragma omp simd
                for (int i = 0; i < n; ++i) x[i] -= s * y[i];
            }
            double nrm = 0.0;
#pragma omp simd reduction(+ : nrm)
            for (int i = 0; i < n; ++i) nrm += x[i] * x[i];
            nrm = std::sqrt(nrm);
            if (!(nrm > 0.0) || !std::isfinite(nrm)) return false;
            const double r = 1.0 / nrm;
#pragma omp simd
            for (int i = 0; i < n; ++i) x[i] *= r;
        }
    }
    return true;
}

}  // namespace

// All n eigenvalues (descending, w) and the eigenvectors of the nv largest (Z, n x nv
// column-major): tridiagonalisation, eigenvalues by QR without vectors, eigenvectors of
// the tridiagonal by inverse iteration, then the Householder reflectors applied to them.
bool sym_eig_partial(int n, const double *A, double *w, double *Z, int nv) {
    if (n <= 0) return true;
    if (nv >= n || n <= 2) {
        std::vector<double> Zf(size_t(n) * n);
        if (!sym_eig(n, A, w, Zf.data())) return false;
        std::copy(Zf.begin(), Zf.begin() + size_t(n) * std::min(nv, n), Z);
        return true;
    }
    std::vector<double> d, e, V, beta;
    tridiagonalise(n, A, d, e, V, beta);
    if (!tridiagonal_eigenvalues(n, d, e, w)) return false;
    std::vector<double> X(size_t(n) * nv), work(size_t(5) * n);
    std::vector<char> piv(n);
    if (!tridiagonal_vectors_raw(n, d.data(), e.data(), w, nv, X.data(), work.data(), piv.data())) return false;
    // back-transformation: X <- H_0 H_1 ... H_{n-3} X
    apply_reflectors(n, nv, V, beta, X.data(), false);
    std::copy(X.begin(), X.end(), Z);
    return true;
}

// Orthonormalising transform of a Gram matrix G = W^T W (n x n, row-major, symmetric):
// the Cholesky factor G = R^T R (R upper triangular) and T = R^{-1}, so that W T has
// orthonormal columns spanning the columns of W.  T: column-major n x n (upper
// triangular).  Returns false, leaving T unspecified, when a pivot r_jj^2 falls to
// rel_tol max_i G_ii or below (numerical rank deficiency: the caller uses the
// eigen-decomposition instead).
bool chol_orth_transform(int n, const double *G, double *T, double rel_tol, double *min_sine) {
    if (min_sine) *min_sine = 0.0;
    if (n <= 0) return true;
    double dmax = 0.0;
    for (int i = 0; i < n; ++i) dmax = std::max(dmax, G[size_t(i) * n + i]);
    if (!(dmax > 0.0) || !std::isfinite(dmax)) return false;
    const double floor_ = rel_tol * dmax;
    std::vector<double> R(size_t(n) * n, 0.0);     // row-major upper triangle
    for (int j = 0; j < n; ++j) {
        double d = G[size_t(j) * n + j];
        for (int k = 0; k < j; ++k) d -= R[size_t(k) * n + j] * R[size_t(k) * n + j];
        if (!(d > floor_)) return false;
        const double rjj = std::sqrt(d);
        R[size_t(j) * n + j] = rjj;
        // sine of the angle between column j and the span of the columns before it
        const double sj = rjj / std::sqrt(G[size_t(j) * n + j]);
        if (min_sine && (j == 0 || sj < *min_sine)) *min_sine = sj;
        const double inv = 1.0 / rjj;
        for (int c = j + 1; c < n; ++c) {
            double v = G[size_t(j) * n + c];
            for (int k = 0; k < j; ++k) v -= R[size_t(k) * n + j] * R[size_t(k) * n + c];
            R[size_t(j) * n + c] = v * inv;
        }
    }
    // T = R^{-1}: back substitution column by column (T upper triangular)
    for (size_t e = 0; e < size_t(n) * n; ++e) T[e] = 0.0;
    for (int c = 0; c < n; ++c) {
        double *t = T + size_t(c) * n;                // column c of T
        t[c] = 1.0 / R[size_t(c) * n + c];
        for (int i = c - 1; i >= 0; --i) {
            double v = 0.0;
            for (int k = i + 1; k <= c; ++k) v += R[size_t(i) * n + k] * t[k];
            t[i] = -v / R[size_t(i) * n + i];
        }
    }
    return true;
}

}  // namespace kl

extern "C" kl_status kl_symeig_partial(int32_t n, const double *A, double *w, double *Z, int32_t nv) {
    if (n < 0 || nv < 0 || nv > n || (n > 0 && (!A || !w || (nv > 0 && !Z)))) {
        kl::set_error("kl_symeig_partial: invalid arguments");
        return KL_EINVAL;
    }
    for (int64_t i = 0; i < int64_t(n) * n; ++i)
        if (!std::isfinite(A[i])) { kl::set_error("kl_symeig_partial: non-finite input"); return KL_ENUMERIC; }
    if (!kl::sym_eig_partial(n, A, w, Z, nv)) {
        kl::set_error("kl_symeig_partial: iteration did not converge");
        return KL_ENOCONV;
    }
    return KL_OK;
}

extern "C" kl_status kl_symeig(int32_t n, const double *A, double *w, double *Z) {
    if (n < 0 || (n > 0 && (!A || !w || !Z))) {
        kl::set_error("kl_symeig: invalid arguments");
        return KL_EINVAL;
    }
    for (int64_t i = 0; i < int64_t(n) * n; ++i)
        if (!std::isfinite(A[i])) { kl::set_error("kl_symeig: non-finite input"); return KL_ENUMERIC; }
    if (!kl::sym_eig(n, A, w, Z)) { kl::set_error("kl_symeig: QR iteration did not converge"); return KL_ENOCONV; }
    return KL_OK;
}
