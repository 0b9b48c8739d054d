// Dense symmetric eigensolver for the Rayleigh-Ritz step (host, FP64).
//
// Householder reduction to tridiagonal form, then implicit symmetric QR steps with the
// Wilkinson shift (Golub and Van Loan, Matrix Computations, Sec. 8.3), accumulating
// every reflection and rotation so that A = Z diag(w) Z^T.  Matrices are small (the
// projected operator of the block eigensolver, n <= a few hundred).
#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <functional>
#include <limits>
#include <mutex>
#include <numeric>
#include <thread>
#include <vector>

#include <unistd.h>

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

// Tolerances of the inverse iteration below, from ||T||_1 of the tridiagonal (d, e).
struct InvIterTol {
    double ortol, pertol, tiny;
};
InvIterTol inv_iter_tol(int n, const double *d, const double *e) {
    const double eps = std::numeric_limits<double>::epsilon();
    double tnorm = 0.0;
    for (int i = 0; i < n; ++i)
        tnorm = std::max(tnorm, std::fabs(d[i]) + (i + 1 < n ? std::fabs(e[i]) : 0.0) + (i > 0 ? std::fabs(e[i - 1]) : 0.0));
    if (tnorm == 0.0) tnorm = 1.0;
    return {1e-3 * tnorm, 10.0 * eps * tnorm, eps * tnorm};
}

// Eigenvectors j0 .. j1 - 1 of the tridiagonal (d, e) for the eigenvalues w[j] (descending)
// by inverse iteration: two steps from a seeded random vector (the shifts are eigenvalues
// accurate to rounding, so the second step already converges); eigenvalues closer than
// ortol form a cluster whose vectors are orthogonalised against each other at every step,
// and equal ones are separated by a tiny shift.  j0 must start a cluster (j0 = 0, or
// w[j0 - 1] - w[j0] > ortol).  The start of vector j is entries j n + 1 .. j n + n of one
// splitmix64 stream, so that vectors can be computed in any order.  X: n x nv, column-major
// (column j written).  work: 5 n doubles, piv: n chars.  Returns false on a breakdown.
KL_HOST_CLONES
bool tridiagonal_vectors_range(int n, const double *d, const double *e, const double *w, int j0, int j1,
                               const InvIterTol &tol, double *X, double *work, char *piv) {
    double *rdd = work, *dl = work + n, *du = work + 2 * n, *du2 = work + 3 * n;
    int cs = j0;                 // first index of the current cluster
    double lam_prev = 0.0;
    for (int j = j0; j < j1; ++j) {
        double lam = w[j];
        if (j > j0 && w[j - 1] - w[j] > tol.ortol) cs = j;
        if (j > cs && lam_prev - lam < tol.pertol) lam = lam_prev - tol.pertol;
        lam_prev = lam;
        tri_lu_factor(n, d, e, lam, tol.tiny, rdd, dl, du, du2, piv);
        double *x = X + size_t(j) * n;
        uint64_t state = 0x2545F4914F6CDD1Dull + uint64_t(j) * uint64_t(n) * 0x9E3779B97F4A7C15ull;
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

// All nv vectors in one sequence.
bool tridiagonal_vectors_raw(int n, const double *d, const double *e, const double *w, int nv, double *X,
                             double *work, char *piv) {
    return tridiagonal_vectors_range(n, d, e, w, 0, nv, inv_iter_tol(n, d, e), X, work, piv);
}

// The largest nv eigenvalues of the symmetric tridiagonal (d, e2 = squared off-diagonals)
// by bisection on the Sturm count (the number of negative pivots of the LDL^T factorisation
// of T - x I is the number of eigenvalues below x; a pivot smaller than pivmin in magnitude
// is replaced by -pivmin), from the Gershgorin interval [glo, ghi], until an interval is no
// wider than 2 eps max(|lo|, |hi|) + pivmin.  Eigenvalues j0 .. j0 + kBisectChains - 1 (the
// chains interleaved, so that their divisions overlap); w[j] for j < nv, descending.
constexpr int kBisectChains = 16;
KL_HOST_CLONES
void bisect_top(int n, const double *d, const double *e2, double pivmin, double glo, double ghi, int j0, int nv,
                double *w) {
    constexpr int C = kBisectChains;
    const double eps = std::numeric_limits<double>::epsilon();
    double lo[C], hi[C];
    int below[C];                                  // n - 1 - j: eigenvalues below the wanted one
    for (int c = 0; c < C; ++c) {
        lo[c] = glo;
        hi[c] = ghi;
        below[c] = n - 1 - std::min(j0 + c, nv - 1);
    }
    for (int it = 0; it < 128; ++it) {
        double mid[C], q[C];
        int cnt[C];
        bool done = true;
        for (int c = 0; c < C; ++c) {
            mid[c] = 0.5 * (lo[c] + hi[c]);
            if (hi[c] - lo[c] > 2.0 * eps * std::max(std::fabs(lo[c]), std::fabs(hi[c])) + pivmin) done = false;
        }
        if (done) break;
        for (int c = 0; c < C; ++c) {
            const double t = d[0] - mid[c];
            q[c] = std::fabs(t) < pivmin ? -pivmin : t;
            cnt[c] = q[c] < 0.0 ? 1 : 0;
        }
        for (int i = 1; i < n; ++i) {
            const double di = d[i], ei = e2[i - 1];
#pragma omp simd
            for (int c = 0; c < C; ++c) {
                double t = (di - mid[c]) - ei / q[c];
                t = std::fabs(t) < pivmin ? -pivmin : t;
                q[c] = t;
                cnt[c] += t < 0.0 ? 1 : 0;
            }
        }
        for (int c = 0; c < C; ++c) {
            if (cnt[c] <= below[c]) lo[c] = mid[c];
            else hi[c] = mid[c];
        }
    }
    for (int c = 0; c < C && j0 + c < nv; ++c) w[j0 + c] = 0.5 * (lo[c] + hi[c]);
}

// A persistent team of host threads for the projected eigensolve: the tasks of a job are
// taken in order from an atomic counter by the calling thread and the workers.  One job at a
// time: a caller that finds the team busy (the batched solver resumes several problems on
// host threads at once) runs its tasks alone.  Workers spin briefly after a job (the next one
// of the same solve follows within a fraction of a millisecond), then sleep.
class HostTeam {
public:
    static HostTeam &get() {
        static HostTeam *team = new HostTeam();    // never destroyed: workers live as long as the process
        return *team;
    }
    void run(int ntasks, const std::function<void(int)> &fn) {
        std::unique_lock<std::mutex> job_lock(job_, std::try_to_lock);
        // (a forked child has none of the workers)
        if (!job_lock.owns_lock() || workers_.empty() || ntasks < 2 || getpid() != pid_) {
            for (int t = 0; t < ntasks; ++t) fn(t);
            return;
        }
        // a worker that is late for the previous job may take a task of this one as soon as
        // next_ is reset: everything it reads is written before, done_ included
        fn_ = &fn;
        ntasks_ = ntasks;
        done_.store(0);
        next_.store(0);
        {
            std::lock_guard<std::mutex> g(m_);
            gen_.fetch_add(1, std::memory_order_release);
        }
        cv_.notify_all();
        take_tasks();
        while (done_.load(std::memory_order_acquire) < ntasks) std::this_thread::yield();
    }

private:
    HostTeam() : pid_(getpid()) {
        const unsigned hw = std::thread::hardware_concurrency();
        const int nw = int(std::min(7u, hw > 1 ? hw - 1 : 0u));
        for (int i = 0; i < nw; ++i) workers_.emplace_back([this] { loop(); });
        for (auto &t : workers_) t.detach();
    }
    void take_tasks() {
        for (;;) {
            const int t = next_.fetch_add(1);
            if (t >= ntasks_) return;
            (*fn_)(t);
            done_.fetch_add(1, std::memory_order_release);
        }
    }
    void loop() {
        uint64_t seen = 0;
        for (;;) {
            // spin for about 0.3 ms on the job generation, then sleep until the next job
            const auto t0 = std::chrono::steady_clock::now();
            while (gen_.load(std::memory_order_acquire) == seen &&
                   std::chrono::steady_clock::now() - t0 < std::chrono::microseconds(300))
                std::this_thread::yield();
            if (gen_.load(std::memory_order_acquire) == seen) {
                std::unique_lock<std::mutex> l(m_);
                cv_.wait(l, [&] { return gen_.load(std::memory_order_acquire) != seen; });
            }
            seen = gen_.load(std::memory_order_acquire);
            take_tasks();
        }
    }
    const pid_t pid_;
    std::mutex job_, m_;
    std::condition_variable cv_;
    std::vector<std::thread> workers_;
    std::atomic<uint64_t> gen_{0};
    std::atomic<int> next_{0}, done_{0};
    int ntasks_ = 0;
    const std::function<void(int)> *fn_ = nullptr;
};

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

// The nv largest eigenvalues (descending, w[0..nv-1]) and their eigenvectors (Z, n x nv
// column-major): tridiagonalisation, the eigenvalues by bisection (tasks of 16 on the host
// team), eigenvectors of the tridiagonal by inverse iteration (tasks of whole clusters), and
// the back-transformation (column chunks); use_team = false runs the tasks on the calling
// thread.  Results do not depend on how the tasks are shared.
bool sym_eig_top(int n, const double *A, int nv, double *w, double *Z, bool use_team) {
    if (n <= 0 || nv <= 0) return true;
    if (nv >= n || n <= 2) {
        std::vector<double> wf(n), Zf(size_t(n) * n);
        if (!sym_eig(n, A, wf.data(), Zf.data())) return false;
        std::copy(wf.begin(), wf.begin() + std::min(nv, n), w);
        std::copy(Zf.begin(), Zf.begin() + size_t(n) * std::min(nv, n), Z);
        return true;
    }
    std::vector<double> d, e, V, beta;
    tridiagonalise(n, A, d, e, V, beta);
    // Gershgorin interval, widened by a few ulps of ||T||, and the pivot floor
    std::vector<double> e2(n, 0.0);
    double glo = std::numeric_limits<double>::infinity(), ghi = -glo, e2max = 0.0;
    for (int i = 0; i < n; ++i) {
        const double r = (i > 0 ? std::fabs(e[i - 1]) : 0.0) + (i + 1 < n ? std::fabs(e[i]) : 0.0);
        glo = std::min(glo, d[i] - r);
        ghi = std::max(ghi, d[i] + r);
        if (i + 1 < n) {
            e2[i] = e[i] * e[i];
            e2max = std::max(e2max, e2[i]);
        }
    }
    const double tn = std::max(std::fabs(glo), std::fabs(ghi));
    const double eps = std::numeric_limits<double>::epsilon();
    glo -= 4.0 * eps * tn + std::numeric_limits<double>::min();
    ghi += 4.0 * eps * tn + std::numeric_limits<double>::min();
    const double pivmin = std::numeric_limits<double>::min() * std::max(1.0, e2max);
    // the tasks below on the host team, or one after another on this thread
    auto run = [&](int ntasks, const std::function<void(int)> &fn) {
        if (use_team) HostTeam::get().run(ntasks, fn);
        else
            for (int t = 0; t < ntasks; ++t) fn(t);
    };
    run((nv + kBisectChains - 1) / kBisectChains, [&](int t) {
        bisect_top(n, d.data(), e2.data(), pivmin, glo, ghi, t * kBisectChains, nv, w);
    });
    for (int j = 0; j < nv; ++j)
        if (!std::isfinite(w[j])) return false;
    // inverse iteration in tasks of whole clusters (about 8 vectors each where clusters allow)
    const InvIterTol tol = inv_iter_tol(n, d.data(), e.data());
    std::vector<int> starts{0};
    for (int j = 1; j < nv; ++j)
        if (w[j - 1] - w[j] > tol.ortol && j - starts.back() >= 8) starts.push_back(j);
    starts.push_back(nv);
    const int ntask = int(starts.size()) - 1;
    std::vector<double> work(size_t(5) * n * ntask);
    std::vector<char> piv(size_t(n) * ntask);
    std::vector<char> ok(ntask, 1);
    run(ntask, [&](int t) {
        ok[t] = tridiagonal_vectors_range(n, d.data(), e.data(), w, starts[t], starts[t + 1], tol, Z,
                                          work.data() + size_t(5) * n * t, piv.data() + size_t(n) * t) ? 1 : 0;
    });
    for (int t = 0; t < ntask; ++t)
        if (!ok[t]) return false;
    // back-transformation Z <- H_0 H_1 ... H_{n-3} Z, in chunks of 8 columns
    constexpr int kCols = 8;
    run((nv + kCols - 1) / kCols, [&](int t) {
        const int c0 = t * kCols, nc = std::min(kCols, nv - c0);
        apply_reflectors_raw(n, nc, V.data(), beta.data(), Z + size_t(c0) * n, false);
    });
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

extern "C" kl_status kl_symeig_top(int32_t n, const double *A, int32_t nv, double *w, double *Z) {
    if (n < 0 || nv < 0 || nv > n || (nv > 0 && (!A || !w || !Z))) {
        kl::set_error("kl_symeig_top: invalid arguments");
        return KL_EINVAL;
    }
    for (int64_t i = 0; i < int64_t(n) * n; ++i)
        if (!std::isfinite(A[i])) { kl::set_error("kl_symeig_top: non-finite input"); return KL_ENUMERIC; }
    if (!kl::sym_eig_top(n, A, nv, w, Z)) {
        kl::set_error("kl_symeig_top: eigensolve failed");
        return KL_ENOCONV;
    }
    return KL_OK;
}
