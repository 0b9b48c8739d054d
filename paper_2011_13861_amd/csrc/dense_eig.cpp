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

// A: n x n symmetric, row-major (read only).  w: eigenvalues, descending.
// Z: column-major n x n, column j = unit eigenvector of w[j].  Returns false if the QR
// iteration does not converge.
bool sym_eig(int n, const double *A, double *w, double *Z) {
    if (n <= 0) return true;
    std::vector<double> a(A, A + size_t(n) * n);     // working copy, row-major
    std::vector<double> d(n, 0.0), e(n, 0.0);
    std::vector<double> V(size_t(n) * n, 0.0);        // Householder vectors, row k = v_k
    std::vector<double> beta(n, 0.0), p(n), q(n);
    // ---- tridiagonalisation: a <- H a H, column by column -----------------------------
    for (int k = 0; k + 2 < n; ++k) {
        const int m = n - k - 1;
        double *v = &V[size_t(k) * n];
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
        for (int i = 0; i < m; ++i) vv += v[i] * v[i];
        const double b = 2.0 / vv;
        beta[k] = b;
        e[k] = alpha;
        // p = b * A22 v,  q = p - (b/2)(p.v) v,  A22 -= v q^T + q v^T
        for (int i = 0; i < m; ++i) {
            const double *row = &a[size_t(k + 1 + i) * n + k + 1];
            double s = 0.0;
            for (int j = 0; j < m; ++j) s += row[j] * v[j];
            p[i] = b * s;
        }
        double pv = 0.0;
        for (int i = 0; i < m; ++i) pv += p[i] * v[i];
        const double K = 0.5 * b * pv;
        for (int i = 0; i < m; ++i) q[i] = p[i] - K * v[i];
        for (int i = 0; i < m; ++i) {
            double *row = &a[size_t(k + 1 + i) * n + k + 1];
            const double vi = v[i], qi = q[i];
            for (int j = 0; j < m; ++j) row[j] -= vi * q[j] + qi * v[j];
        }
    }
    if (n >= 2) {
        d[n - 2] = a[size_t(n - 2) * n + (n - 2)];
        e[n - 2] = a[size_t(n - 1) * n + (n - 2)];
    }
    d[n - 1] = a[size_t(n - 1) * n + (n - 1)];
    e[n - 1] = 0.0;
    // ---- accumulate Q = H_0 H_1 ... H_{n-3}, column-major in Z ------------------------
    for (size_t i = 0; i < size_t(n) * n; ++i) Z[i] = 0.0;
    for (int i = 0; i < n; ++i) Z[size_t(i) * n + i] = 1.0;
    for (int k = n - 3; k >= 0; --k) {
        if (beta[k] == 0.0) continue;
        const int m = n - k - 1;
        const double *v = &V[size_t(k) * n];
        // Q[k+1:, k+1:] <- (I - b v v^T) Q[k+1:, k+1:]; columns are contiguous
        for (int c = k + 1; c < n; ++c) {
            double *col = &Z[size_t(c) * n + k + 1];
            double s = 0.0;
            for (int i = 0; i < m; ++i) s += v[i] * col[i];
            s *= beta[k];
            for (int i = 0; i < m; ++i) col[i] -= s * v[i];
        }
    }
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
            const double r = std::hypot(x, z);
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

}  // namespace kl

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
