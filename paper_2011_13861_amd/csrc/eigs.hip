// Block eigensolver for the k leading eigenpairs of A~' (standard form, Sec. 4.1).
//
// The paper solves the standard eigenproblem with implicitly restarted Lanczos, one
// vector at a time, calling Algorithm 1 once per iteration (Sec. 4.4.2).  Here the
// Krylov space is grown a block of b vectors at a time, so that every stage-5 launch
// contracts the covariance tile with b columns on the matrix cores:
//   - basis V (N x m, orthonormal) and AV = A~' V are kept on the device in FP64;
//   - expansion: the newest block of AV, orthogonalised against V twice (classical
//     Gram-Schmidt, twice) and orthonormalised through the eigen-decomposition of its
//     b x b Gram matrix;
//   - Rayleigh-Ritz: H = V^T AV (FP64, symmetrised), dense symmetric eigensolve,
//     Ritz vectors X = V S, residuals R = AV S - X Theta computed explicitly;
//   - thick restart: keep the k + guard leading Ritz vectors; the next block spans the
//     dominant directions of their residuals (the next Krylov block in exact arithmetic);
//   - mixed precision: with a low-precision stage 5 the iteration runs until the
//     residuals reach the level that precision can certify, then AV is recomputed
//     with the FP64 apply and the same iteration finishes in FP64, so that the final
//     criterion is met under the FP64 operator.
// Converged when ||A~' x_i - theta_i x_i|| <= max(tol theta_i, abs_floor theta_1), i <= k.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <new>
#include <random>
#include <sstream>
#include <string>
#include <thread>

#include "kl_internal.h"

namespace kl {

namespace {

constexpr int kT = 256;

// Checks a block for non-finite values: flag[0] = 1 if any.
__global__ __launch_bounds__(kT) void finite_kernel(const double *__restrict__ X, int64_t n,
                                                    int *__restrict__ flag) {
    for (int64_t i = int64_t(blockIdx.x) * kT + threadIdx.x; i < n; i += int64_t(gridDim.x) * kT)
        if (!isfinite(X[i])) flag[0] = 1;
}

}  // namespace

struct SolverCache {
    hipStream_t s = nullptr;
    // second stream of the Rayleigh-Ritz step: the Ritz vectors, their residuals and norms
    // are formed there while the main stream applies the operator to the next block
    hipStream_t s2 = nullptr;
    hipEvent_t ev = nullptr;    // orders s2 after the basis written on s
    hipEvent_t ev_wait[2] = {nullptr, nullptr};   // host waits on s and on s2 (polled)
    int64_t N = 0;
    int mcap = 0, ccap = 0;
    double *V = nullptr, *AV = nullptr, *Vt = nullptr, *AVt = nullptr, *W = nullptr;
    double *R = nullptr;        // residuals of the kept Ritz vectors (N x mcap)
    double *C = nullptr, *C2 = nullptr, *part = nullptr, *dtheta = nullptr, *dnorm = nullptr;
    double *rpart = nullptr;    // partial sums of the residual norms
    int *dflag = nullptr;
    // pinned host staging of the small transfers (hipHostMalloc): a device-to-host
    // region (Gram matrices, blocks of H, residual norms) and one host-to-device region
    // per source (orthonormalising transform, Ritz vectors, Ritz values); every region
    // is reused only after a stream synchronisation that follows its last transfer
    double *pin = nullptr;
    size_t pin_region = 0;      // doubles per region (5 regions: the fifth takes the norms)
};

namespace {

void release_buffers(SolverCache &c) {
    hipFree(c.V); hipFree(c.AV); hipFree(c.Vt); hipFree(c.AVt); hipFree(c.W); hipFree(c.R);
    hipFree(c.C); hipFree(c.C2); hipFree(c.part); hipFree(c.rpart); hipFree(c.dtheta); hipFree(c.dnorm);
    hipFree(c.dflag);
    if (c.pin) hipHostFree(c.pin);
    c.V = c.AV = c.Vt = c.AVt = c.W = c.R = c.C = c.C2 = c.part = c.rpart = c.dtheta = c.dnorm = nullptr;
    c.pin = nullptr;
    c.pin_region = 0;
    c.dflag = nullptr;
    c.N = 0;
    c.mcap = c.ccap = 0;
}

// Standard normal values for a random block: element i uses two 53-bit uniforms from
// splitmix64 of (seed, 2i) and (seed, 2i + 1) and the Box-Muller transform.
__device__ __forceinline__ uint64_t mix64(uint64_t z) {
    z += 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

__global__ __launch_bounds__(kT) void normal_fill_kernel(double *__restrict__ X, int64_t n, uint64_t seed) {
    for (int64_t i = int64_t(blockIdx.x) * kT + threadIdx.x; i < n; i += int64_t(gridDim.x) * kT) {
        const uint64_t a = mix64(seed ^ mix64(2 * uint64_t(i))), b = mix64(seed ^ mix64(2 * uint64_t(i) + 1));
        const double u1 = (double(a >> 11) + 1.0) * (1.0 / 9007199254740992.0);   // (0, 1]
        const double u2 = double(b >> 11) * (1.0 / 9007199254740992.0);
        X[i] = sqrt(-2.0 * log(u1)) * cospi(2.0 * u2);
    }
}

void launch_normal_fill(double *X, int64_t n, uint64_t seed, hipStream_t s) {
    const int64_t g = std::min<int64_t>(1024, (n + kT - 1) / kT);
    hipLaunchKernelGGL(normal_fill_kernel, dim3(unsigned(std::max<int64_t>(g, 1))), dim3(kT), 0, s, X, n, seed);
}

struct Solver {
    kl_problem *P;
    hipStream_t s = nullptr;
    hipStream_t s2 = nullptr;   // Rayleigh-Ritz stream (NULL: everything on s)
    hipEvent_t ev = nullptr;
    hipEvent_t ev_wait[2] = {nullptr, nullptr};   // see wait()
    int64_t N = 0;
    int b = 32, k = 1, keep = 1, mmax = 1;
    double *V = nullptr, *AV = nullptr, *Vt = nullptr, *AVt = nullptr, *W = nullptr, *R = nullptr;
    double *C = nullptr, *C2 = nullptr, *dtheta = nullptr, *dnorm = nullptr, *part = nullptr, *rpart = nullptr;
    int *dflag = nullptr;
    // pinned staging regions (see SolverCache)
    double *pin_d2h = nullptr, *pin_T = nullptr, *pin_S = nullptr, *pin_theta = nullptr, *pin_norm = nullptr;
    std::vector<double> H;      // mmax x mmax, row-major, host
    int m = 0;                  // current basis size
    int last = 0;               // columns [m - last, m) are the newest block
    bool last_refilled = false; // the last orth_into_basis replaced directions by random ones
    int applies[4] = {0, 0, 0, 0}, block_applies[4] = {0, 0, 0, 0}, restarts = 0;

    kl_status check(hipError_t e, const char *what) {
        if (e == hipSuccess) return KL_OK;
        std::ostringstream os;
        os << "kl_eigs: " << what << ": " << hipGetErrorString(e);
        set_error(os.str());
        return e == hipErrorOutOfMemory ? KL_ENOMEM : KL_EHIP;
    }
    // Waits on the host for the work queued on st (s or s2) so far.  The waits inside a step
    // are short (a Gram product, the residual norms), so an event recorded on st is polled:
    // a blocking stream synchronisation may sleep until an interrupt wakes the thread, which
    // costs tens of microseconds per wait.  The batched solver's runs (no second stream),
    // which share the host cores, keep the blocking form.
    kl_status wait(hipStream_t st) {
        hipEvent_t e = ev_wait[st == s2 && s2 ? 1 : 0];
        if (!e || !s2) return check(hipStreamSynchronize(st), "sync");
        kl_status r;
        if ((r = check(hipEventRecord(e, st), "event")) != KL_OK) return r;
        for (;;) {
            const hipError_t q = hipEventQuery(e);
            if (q == hipSuccess) return KL_OK;
            if (q != hipErrorNotReady) return check(q, "event query");
        }
    }
    // C = A^T B   (A: N x ma, B: N x nb, ld N) -> C (ma x nb, ld ma), device; split-N
    // Gram kernel (tall-skinny shapes)
    kl_status gemm_tn(const double *A, int ma, const double *B, int nb, double *Cout) {
        launch_gram(A, N, ma, B, N, nb, N, part, Cout, P->n_cu, s);
        return check(hipGetLastError(), "gram kernel");
    }
    // Out = alpha A S + beta Out   (A: N x ma, S: ma x nb with ld lds)
    kl_status gemm_nn(const double *A, int ma, const double *S, int lds, int nb, double alpha,
                      double beta, double *Out, hipStream_t on = nullptr) {
        launch_gemm_nn(A, N, ma, S, lds, nb, N, alpha, beta, Out, N, on ? on : s);
        return check(hipGetLastError(), "gemm kernel");
    }

    kl_status apply(int precision, const double *x, double *y, int ncols) {
        for (int c0 = 0; c0 < ncols; c0 += kBW) {
            const int nb = std::min(kBW, ncols - c0);
            kl_status st = apply_chunk(P, precision, nb, x + int64_t(c0) * N, N, y + int64_t(c0) * N, N, s);
            if (st != KL_OK) return st;
            block_applies[precision] += 1;
        }
        applies[precision] += ncols;
        return KL_OK;
    }

    // H[0:m, c0:c1] = V^T AV[:, c0:c1] (and the mirrored rows).
    kl_status update_H(int c0, int c1) {
        const int nc = c1 - c0;
        kl_status st = gemm_tn(V, c1, AV + int64_t(c0) * N, nc, C);
        if (st != KL_OK) return st;
        const double *hc = pin_d2h;
        if ((st = check(hipMemcpyAsync(pin_d2h, C, size_t(c1) * nc * 8, hipMemcpyDeviceToHost, s), "copy H")) != KL_OK)
            return st;
        if ((st = wait(s)) != KL_OK) return st;
        for (int j = 0; j < nc; ++j)
            for (int i = 0; i < c1; ++i) {
                const double v = hc[size_t(j) * c1 + i];
                const int col = c0 + j;
                if (i < c0) {
                    H[size_t(i) * mmax + col] = v;
                    H[size_t(col) * mmax + i] = v;
                } else {
                    H[size_t(i) * mmax + col] = v;   // diagonal block, symmetrised below
                }
            }
        for (int i = c0; i < c1; ++i)
            for (int j = i + 1; j < c1; ++j) {
                const double a = 0.5 * (H[size_t(i) * mmax + j] + H[size_t(j) * mmax + i]);
                H[size_t(i) * mmax + j] = H[size_t(j) * mmax + i] = a;
            }
        return KL_OK;
    }

    // Re-orthonormalises W = V[:, m:m+ncols], already orthonormal and orthogonal to
    // V[:, :m] up to rounding, with one Gram product: [C1; G] = [V | W]^T W (V and W are
    // adjacent columns), G = Z diag(w) Z^T on the host, then W <- (W - V C1) T with
    // T = Z diag(w)^(-1/2).  The Gram matrix of W - V C1 is G - C1^T C1, which differs
    // from G by the square of rounding-size terms, so G is used.  On a numerically rank
    // deficient G nothing is changed and ok stays false.  Wb receives a copy of the result.
    kl_status reorth_short(double *Wb, int ncols, bool &ok) {
        kl_status st;
        ok = false;
        double *dst = V + int64_t(m) * N;
        const int mt = m + ncols;
        if ((st = gemm_tn(V, mt, dst, ncols, C)) != KL_OK) return st;
        if ((st = check(hipMemcpyAsync(pin_d2h, C, size_t(mt) * ncols * 8, hipMemcpyDeviceToHost, s),
                        "copy Gram")) != KL_OK)
            return st;
        if ((st = wait(s)) != KL_OK) return st;
        std::vector<double> G(size_t(ncols) * ncols);
        for (int j = 0; j < ncols; ++j)
            for (int i = 0; i < ncols; ++i) G[size_t(i) * ncols + j] = pin_d2h[size_t(j) * mt + m + i];
        for (int i = 0; i < ncols; ++i)
            for (int j = i + 1; j < ncols; ++j) {
                const double a = 0.5 * (G[size_t(i) * ncols + j] + G[size_t(j) * ncols + i]);
                G[size_t(i) * ncols + j] = G[size_t(j) * ncols + i] = a;
            }
        // T = R^{-1} (G = R^T R); on a small pivot, T = Z diag(w)^(-1/2) from G = Z diag(w) Z^T
        double *T = pin_T;
        if (!chol_orth_transform(ncols, G.data(), T, 1e-24)) {
            std::vector<double> w(ncols), Z(size_t(ncols) * ncols);
            if (!sym_eig(ncols, G.data(), w.data(), Z.data())) {
                set_error("kl_eigs: Gram eigen-decomposition failed");
                return KL_ENUMERIC;
            }
            if (!(w[ncols - 1] > std::max(w[0], 1e-300) * 1e-26)) return KL_OK;
            for (int j = 0; j < ncols; ++j) {
                const double sc = 1.0 / std::sqrt(w[j]);
                for (int i = 0; i < ncols; ++i) T[size_t(j) * ncols + i] = Z[size_t(j) * ncols + i] * sc;
            }
        }
        // W -= V C1 (C1: the first m rows of the device Gram result, ld mt)
        if (m > 0 && (st = gemm_nn(V, m, C, mt, ncols, -1.0, 1.0, dst)) != KL_OK) return st;
        // the upload follows the product that reads C1 on the stream
        if ((st = check(hipMemcpyAsync(C, T, size_t(ncols) * ncols * 8, hipMemcpyHostToDevice, s), "copy T")) != KL_OK)
            return st;
        if ((st = gemm_nn(dst, ncols, C, ncols, ncols, 1.0, 0.0, Wb)) != KL_OK) return st;
        if ((st = check(hipMemcpyAsync(dst, Wb, size_t(N) * ncols * 8, hipMemcpyDeviceToDevice, s), "copy W")) != KL_OK)
            return st;
        ok = true;
        return KL_OK;
    }

    // Orthonormalises the ncols columns of W against V[:, :m] and among themselves and
    // writes `want` orthonormal columns to V[:, m:m+want], spanning the dominant
    // directions of W; rank deficiency is filled with seeded random directions.  With
    // c_holds_vtw the device buffer C already holds V[:, :m]^T W (m x ncols, as the
    // last update_H left it) and the first Gram product is not recomputed.
    // One Cholesky pass leaves the columns orthonormal to about eps kappa^2 and orthogonal
    // to V (after the two Gram-Schmidt rounds) to about eps kappa, kappa the condition of
    // the block after Gram-Schmidt; when no column lies within asin(0.1) of the span of the
    // columns before it, kappa is at most about 10 sqrt(ncols) and the second pass is
    // skipped.
    kl_status orth_into_basis(double *Wb, int ncols, int want, std::mt19937_64 &rng, bool c_holds_vtw = false) {
        kl_status st;
        std::vector<double> G, w, Z;
        double *dst = V + int64_t(m) * N;
        last_refilled = false;
        // pass 0 selects the `want` dominant directions; later passes re-orthonormalise
        // them (twice is enough unless a direction had to be replaced by a random one)
        bool refilled = true, well_conditioned = false;
        for (int pass = 0; pass < 4 && (pass < 2 || refilled); ++pass) {
            if (pass > 0 && !refilled && well_conditioned) break;
            if (pass > 0 && !refilled) {
                // the block is orthonormal and orthogonal to V up to rounding: one pass of
                // the short form (falls through to the full one if it meets rank deficiency)
                bool ok = false;
                if ((st = reorth_short(Wb, ncols, ok)) != KL_OK) return st;
                if (ok) break;
            }
            refilled = false;
            for (int cgs = 0; cgs < 2; ++cgs) {
                if (m == 0) break;
                if (!(pass == 0 && cgs == 0 && c_holds_vtw) && (st = gemm_tn(V, m, Wb, ncols, C)) != KL_OK)
                    return st;
                if ((st = gemm_nn(V, m, C, m, ncols, -1.0, 1.0, Wb)) != KL_OK) return st;
            }
            // Gram matrix of W and its eigen-decomposition
            if ((st = gemm_tn(Wb, ncols, Wb, ncols, C)) != KL_OK) return st;
            if ((st = check(hipMemcpyAsync(pin_d2h, C, size_t(ncols) * ncols * 8, hipMemcpyDeviceToHost, s),
                            "copy G")) != KL_OK)
                return st;
            if ((st = wait(s)) != KL_OK) return st;
            G.assign(pin_d2h, pin_d2h + size_t(ncols) * ncols);
            for (int i = 0; i < ncols; ++i)
                for (int j = i + 1; j < ncols; ++j) {
                    const double a = 0.5 * (G[size_t(i) * ncols + j] + G[size_t(j) * ncols + i]);
                    G[size_t(i) * ncols + j] = G[size_t(j) * ncols + i] = a;
                }
            // pass 0 keeps the `want` dominant directions (fewer if W has fewer columns:
            // the rest is filled at random); later passes keep every column.  When every
            // column is kept, the Cholesky factor of G gives the transform (T = R^{-1});
            // otherwise, or on a small pivot, the eigen-decomposition G = Z diag(w) Z^T
            // (T = Z[:, :good] diag(w)^(-1/2), the dominant directions first)
            const int out_cols = pass == 0 ? want : ncols;
            double *T = pin_T;
            int good = 0;
            double min_sine = 0.0;
            if (out_cols == ncols && chol_orth_transform(ncols, G.data(), T, 1e-24, &min_sine)) {
                good = ncols;
                well_conditioned = pass == 0 && min_sine >= 0.1;
            } else {
                w.assign(ncols, 0.0);
                Z.assign(size_t(ncols) * ncols, 0.0);
                if (!sym_eig(ncols, G.data(), w.data(), Z.data())) {
                    set_error("kl_eigs: Gram eigen-decomposition failed");
                    return KL_ENUMERIC;
                }
                const double thresh = std::max(w[0], 1e-300) * 1e-26;
                while (good < std::min(out_cols, ncols) && w[good] > thresh) ++good;
                for (int j = 0; j < good; ++j) {
                    const double sc = 1.0 / std::sqrt(w[j]);
                    for (int i = 0; i < ncols; ++i) T[size_t(j) * ncols + i] = Z[size_t(j) * ncols + i] * sc;
                }
            }
            if (good > 0 &&
                (st = check(hipMemcpyAsync(C, T, size_t(ncols) * good * 8, hipMemcpyHostToDevice, s), "copy T")) != KL_OK)
                return st;
            if ((st = gemm_nn(Wb, ncols, C, ncols, good, 1.0, 0.0, dst)) != KL_OK) return st;
            if (good < out_cols) {
                // replace the missing directions by random vectors; the next pass
                // orthonormalises them
                refilled = true;
                last_refilled = true;
                launch_normal_fill(dst + int64_t(good) * N, int64_t(N) * (out_cols - good), rng(), s);
            }
            ncols = out_cols;
            if ((st = check(hipMemcpyAsync(Wb, dst, size_t(N) * ncols * 8, hipMemcpyDeviceToDevice, s),
                            "copy W")) != KL_OK)
                return st;
        }
        return KL_OK;
    }
};

// The problem's solver cache and its stream (created on first use).
kl_status ensure_solver_stream(kl_problem *P) {
    if (!P->solver) {
        P->solver = new (std::nothrow) SolverCache();
        if (!P->solver) { set_error("kl_eigs: host allocation failed"); return KL_ENOMEM; }
    }
    SolverCache &c = *P->solver;
    hipError_t e = hipSuccess;
    if (!c.s && (e = hipStreamCreate(&c.s)) != hipSuccess) c.s = nullptr;
    if (e == hipSuccess && !c.s2 && (e = hipStreamCreate(&c.s2)) != hipSuccess) c.s2 = nullptr;
    if (e == hipSuccess && !c.ev && (e = hipEventCreateWithFlags(&c.ev, hipEventDisableTiming)) != hipSuccess)
        c.ev = nullptr;
    for (int i = 0; i < 2 && e == hipSuccess; ++i)
        if (!c.ev_wait[i] && (e = hipEventCreateWithFlags(&c.ev_wait[i], hipEventDisableTiming)) != hipSuccess)
            c.ev_wait[i] = nullptr;
    if (e != hipSuccess) {
        set_error(std::string("kl_eigs: stream: ") + hipGetErrorString(e));
        return KL_EHIP;
    }
    return KL_OK;
}

// Grows the problem's solver cache to hold an N x mmax basis (and N x cmax work block).
kl_status acquire_cache(kl_problem *P, int64_t N, int mmax, int cmax) {
    kl_status st = ensure_solver_stream(P);
    if (st != KL_OK) return st;
    SolverCache &c = *P->solver;
    auto hip = [](hipError_t e, const char *what) -> kl_status {
        if (e == hipSuccess) return KL_OK;
        set_error(std::string("kl_eigs: ") + what + ": " + hipGetErrorString(e));
        return e == hipErrorOutOfMemory ? KL_ENOMEM : KL_EHIP;
    };
    if (c.N == N && c.mcap >= mmax && c.ccap >= cmax) return KL_OK;
    release_buffers(c);
    const int mc = std::max(mmax, c.N == N ? c.mcap : 0), cc = std::max(cmax, c.N == N ? c.ccap : 0);
    const size_t nb = size_t(N) * mc * sizeof(double);
    if ((st = hip(hipMalloc(&c.V, nb), "alloc V")) != KL_OK ||
        (st = hip(hipMalloc(&c.AV, nb), "alloc AV")) != KL_OK ||
        (st = hip(hipMalloc(&c.Vt, nb), "alloc Vt")) != KL_OK ||
        (st = hip(hipMalloc(&c.AVt, nb), "alloc AVt")) != KL_OK ||
        (st = hip(hipMalloc(&c.W, size_t(N) * cc * sizeof(double)), "alloc W")) != KL_OK ||
        (st = hip(hipMalloc(&c.R, nb), "alloc R")) != KL_OK ||
        (st = hip(hipMalloc(&c.C, size_t(cc) * cc * sizeof(double)), "alloc C")) != KL_OK ||
        (st = hip(hipMalloc(&c.C2, size_t(cc) * cc * sizeof(double)), "alloc C2")) != KL_OK ||
        // split partials of the Gram kernel: its row ranges times a cmax x cmax product
        (st = hip(hipMalloc(&c.part, size_t(gram_part_elems(N, std::max(mc, cc), std::max(mc, cc))) * sizeof(double)),
                  "alloc gram partials")) != KL_OK ||
        (st = hip(hipMalloc(&c.rpart, size_t(residual_chunks(N)) * mc * sizeof(double)),
                  "alloc residual partials")) != KL_OK ||
        (st = hip(hipMalloc(&c.dtheta, size_t(mc) * 8), "alloc theta")) != KL_OK ||
        (st = hip(hipMalloc(&c.dnorm, size_t(mc) * 8), "alloc norms")) != KL_OK ||
        (st = hip(hipMalloc(&c.dflag, sizeof(int)), "alloc flag")) != KL_OK) {
        release_buffers(c);
        return st;
    }
    c.pin_region = size_t(std::max(mc, cc)) * size_t(std::max(mc, cc));
    if ((st = hip(hipHostMalloc(reinterpret_cast<void **>(&c.pin), 5 * c.pin_region * sizeof(double),
                                hipHostMallocDefault), "alloc pinned staging")) != KL_OK) {
        c.pin = nullptr;
        release_buffers(c);
        return st;
    }
    c.N = N;
    c.mcap = mc;
    c.ccap = cc;
    return KL_OK;
}

int default_guard(int k, int b) { return std::max(std::max(8, b / 4), (3 * k + 9) / 10); }

enum { AFTER_NONE = 0, AFTER_START, AFTER_SWITCH, AFTER_EXPAND };

struct EigRun {
    kl_problem *P = nullptr;
    Solver S;
    double tol = 1e-6, floor_rel = 1e-12, lo_floor = 0.0;
    bool refine = false;
    bool coeffs = false;                    // return B-spline coefficients v = L^{-T} v'
    int max_applies = 0;
    int precision = KL_F64;                 // precision of the current phase
    std::mt19937_64 rng;
    std::vector<double> theta, Sm, norms;
    double best_lo = INFINITY, t_host_eig = 0.0, max_rel = INFINITY;
    int stall = 0, converged = 0;
    bool done = false;
    bool overlap = true;                    // host Rayleigh-Ritz overlapped with the next expansion
    // the operator application the run waits for
    int pending_prec = KL_F64, pending_cols = 0, after = AFTER_NONE, last_add = 0;
    // the basis satisfies the block Arnoldi relation A V[:, :m - last] in span V[:, :m]:
    // every expansion so far kept all directions of the operator image of the newest
    // block (no truncation, no random refill); only then is the next Krylov block a
    // valid continuation of a thick restart (it spans the residuals of the Ritz vectors)
    bool krylov_ok = true;
    bool pending_keeps_krylov = true;       // the pending expansion keeps the relation
    bool pending_done = false;              // the pending application was already made
    double *pending_x = nullptr, *pending_y = nullptr;

    kl_status configure(kl_problem *P_, const kl_eigs_opts *opts);
    kl_status begin(const double *x0, int nvec0);
    kl_status after_apply();
    kl_status finish(double *evals, double *evecs, int64_t ldv, kl_eigs_report *rep, double t_solve);
    void count_apply(int prec, int cols);

  private:
    kl_status rr_step();
    void set_pending(int prec, double *x, double *y, int cols, int after_);
};

}  // namespace

void free_solver_cache(SolverCache *c) {
    if (!c) return;
    if (c->s) hipStreamSynchronize(c->s);
    if (c->s2) hipStreamSynchronize(c->s2);
    release_buffers(*c);
    if (c->s) hipStreamDestroy(c->s);
    if (c->s2) hipStreamDestroy(c->s2);
    if (c->ev) hipEventDestroy(c->ev);
    for (hipEvent_t e : c->ev_wait)
        if (e) hipEventDestroy(e);
    delete c;
}

// The solver stream of P (created on first use) waits for the work queued on `caller`
// so far: a start block or an apply the caller issued there is complete before the
// solver reads or overwrites the shared buffers.
kl_status order_after(kl_problem *P, hipStream_t caller) {
    kl_status st = ensure_solver_stream(P);
    if (st != KL_OK) return st;
    hipEvent_t e;
    if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) {
        set_error("kl_eigs: hipEventCreate failed");
        return KL_EHIP;
    }
    hipError_t err = hipEventRecord(e, caller);
    if (err == hipSuccess) err = hipStreamWaitEvent(P->solver->s, e, 0);
    (void)hipEventDestroy(e);
    if (err != hipSuccess) {
        set_error(std::string("kl_eigs: ordering after the caller's stream: ") + hipGetErrorString(err));
        return KL_EHIP;
    }
    return KL_OK;
}

// ---- one eigensolve as a resumable run ----------------------------------------------
// The run stops at every operator application (pending_*); the caller applies A~' in
// the pending precision to the pending columns (alone, or together with other runs in
// one batched launch) and resumes with after_apply().

kl_status EigRun::configure(kl_problem *P_, const kl_eigs_opts *opts) {
    P = P_;
    if (!opts) { set_error("kl_eigs: NULL argument"); return KL_EINVAL; }
    const int64_t N = P->hs.N;
    if (opts->k < 1 || opts->k > N) { set_error("kl_eigs: k must be in 1..N"); return KL_EINVAL; }
    if (opts->precision < KL_F64 || opts->precision > KL_BF16X3) {
        set_error("kl_eigs: unsupported precision");
        return KL_EINVAL;
    }
    S.P = P;
    S.N = N;
    S.k = opts->k;
    S.b = opts->block > 0 ? opts->block : 32;
    if (S.b > kBW * 8) { set_error("kl_eigs: block too large"); return KL_EINVAL; }
    tol = opts->tol > 0 ? opts->tol : 1e-6;
    floor_rel = opts->abs_floor > 0 ? opts->abs_floor : 1e-12;
    const int guard = opts->guard > 0 ? opts->guard : default_guard(S.k, S.b);
    S.keep = S.k + guard;
    S.mmax = opts->max_basis > 0 ? opts->max_basis : S.keep + 3 * S.b;
    if (S.mmax < S.keep + S.b) S.mmax = S.keep + S.b;
    if (S.mmax > N) S.mmax = int(N);
    if (S.b > S.mmax) S.b = S.mmax;
    if (S.keep > S.mmax - S.b) S.keep = std::max(S.k, S.mmax - S.b);
    if (S.keep > S.mmax) S.keep = S.mmax;
    max_applies = opts->max_applies > 0 ? opts->max_applies : int(std::min<int64_t>(
        int64_t(400) * S.b + 20 * S.k, 4000000));
    precision = opts->precision;
    refine = precision != KL_F64 && opts->refine_fp64 != 0;
    // low-precision floor: relative accuracy the low-precision apply can certify
    lo_floor = opts->lo_floor > 0 ? opts->lo_floor
               : precision == KL_F32 ? 2e-6 : precision == KL_BF16X3 ? 5e-5 : precision == KL_BF16 ? 5e-3 : 0.0;
    if (opts->coeffs != 0 && opts->coeffs != 1) { set_error("kl_eigs: coeffs must be 0 or 1"); return KL_EINVAL; }
    coeffs = opts->coeffs == 1;
    rng.seed(opts->seed);
    return KL_OK;
}

kl_status EigRun::begin(const double *x0, int nvec0) {
    kl_status st;
    const int64_t N = S.N;
    // b spare basis columns hold the speculative block of a restart step (see rr_step);
    // C and the Gram partials hold the (mmax + b) x b products of its orthonormalisation
    const int cmax = std::max(S.mmax + S.b, S.keep + S.b);
    if ((st = acquire_cache(P, N, S.mmax + S.b, cmax)) != KL_OK) return st;
    {
        SolverCache &c = *P->solver;
        S.s = c.s;
        S.V = c.V; S.AV = c.AV; S.Vt = c.Vt; S.AVt = c.AVt; S.W = c.W; S.R = c.R;
        S.C = c.C; S.C2 = c.C2; S.part = c.part; S.rpart = c.rpart; S.dtheta = c.dtheta; S.dnorm = c.dnorm;
        S.dflag = c.dflag;
        S.s2 = overlap ? c.s2 : nullptr;
        S.ev = c.ev;
        S.ev_wait[0] = c.ev_wait[0];
        S.ev_wait[1] = c.ev_wait[1];
        S.pin_d2h = c.pin;
        S.pin_T = c.pin + c.pin_region;
        S.pin_S = c.pin + 2 * c.pin_region;
        S.pin_theta = c.pin + 3 * c.pin_region;
        S.pin_norm = c.pin + 4 * c.pin_region;
    }
    S.H.assign(size_t(S.mmax) * S.mmax, 0.0);
    const int b0 = S.b;
    const int from_x0 = std::min<int>(nvec0, b0);
    if (from_x0 > 0) {
        if ((st = S.check(hipMemcpy2DAsync(S.W, size_t(N) * 8, x0, size_t(N) * 8, size_t(N) * 8, from_x0,
                                           hipMemcpyDeviceToDevice, S.s), "copy x0")) != KL_OK)
            return st;
        if ((st = S.check(hipMemsetAsync(S.dflag, 0, sizeof(int), S.s), "memset")) != KL_OK) return st;
        hipLaunchKernelGGL(finite_kernel, dim3(256), dim3(kT), 0, S.s, S.W, int64_t(N) * from_x0, S.dflag);
        int flag = 0;
        if ((st = S.check(hipMemcpyAsync(&flag, S.dflag, sizeof(int), hipMemcpyDeviceToHost, S.s), "flag")) != KL_OK)
            return st;
        if ((st = S.check(hipStreamSynchronize(S.s), "sync")) != KL_OK) return st;
        if (flag) { set_error("kl_eigs: non-finite start block"); return KL_ENUMERIC; }
    }
    if (from_x0 < b0) launch_normal_fill(S.W + int64_t(from_x0) * N, int64_t(N) * (b0 - from_x0), rng(), S.s);
    S.m = 0;
    krylov_ok = true;
    pending_keeps_krylov = true;
    if ((st = S.orth_into_basis(S.W, b0, b0, rng)) != KL_OK) return st;
    set_pending(precision, S.V, S.AV, b0, AFTER_START);
    return KL_OK;
}

void EigRun::set_pending(int prec, double *x, double *y, int cols, int after_) {
    pending_done = false;
    pending_prec = prec;
    pending_x = x;
    pending_y = y;
    pending_cols = cols;
    after = after_;
}

void EigRun::count_apply(int prec, int cols) {
    S.applies[prec] += cols;
    S.block_applies[prec] += (cols + kBW - 1) / kBW;
}

kl_status EigRun::after_apply() {
    kl_status st;
    const int64_t N = S.N;
    pending_cols = 0;
    switch (after) {
    case AFTER_START:
        S.m = S.b;
        S.last = S.b;
        if ((st = S.update_H(0, S.b)) != KL_OK) return st;
        return rr_step();
    case AFTER_SWITCH: {
        const int kk = S.m;
        std::fill(S.H.begin(), S.H.end(), 0.0);
        if ((st = S.update_H(0, kk)) != KL_OK) return st;
        S.last = kk;
        // expand with every residual direction of the FP64 operator: the kept vectors are
        // Ritz vectors of the low-precision operator, so (unlike after a restart within
        // one precision) their residuals are not confined to one block
        launch_residual(S.V, S.AV, S.dtheta, N, N, kk, S.W, S.rpart, S.dnorm, S.s);
        const int add = int(std::min<int64_t>(std::min(kk, S.mmax - S.m), N - S.m));
        krylov_ok = false;                  // low-precision Ritz vectors under the FP64 operator
        if (add > 0) {
            if ((st = S.orth_into_basis(S.W, kk, add, rng)) != KL_OK) return st;
            krylov_ok = add == kk && !S.last_refilled;
            pending_keeps_krylov = true;
            last_add = add;
            set_pending(precision, S.V + int64_t(S.m) * N, S.AV + int64_t(S.m) * N, add, AFTER_EXPAND);
            return KL_OK;
        }
        return rr_step();
    }
    case AFTER_EXPAND: {
        const int add = last_add;
        if ((st = S.update_H(S.m, S.m + add)) != KL_OK) return st;
        S.m += add;
        S.last = add;
        krylov_ok = krylov_ok && pending_keeps_krylov;
        return rr_step();
    }
    default:
        return KL_OK;
    }
}

kl_status EigRun::rr_step() {
    using clock = std::chrono::steady_clock;
    kl_status st;
    const int64_t N = S.N;
    const int total_applies = S.applies[0] + S.applies[1] + S.applies[2] + S.applies[3];
    const bool must_restart = S.m + S.b > S.mmax;
    // ---- Rayleigh-Ritz on the current basis --------------------------------------------
    const int m = S.m;
    std::vector<double> Hm(size_t(m) * m);
    for (int i = 0; i < m; ++i)
        for (int j = 0; j < m; ++j) Hm[size_t(i) * m + j] = S.H[size_t(i) * S.mmax + j];
    // the kk kept Ritz values (theta[0 .. kk - 1]) and their Ritz vectors (m x kk, column-major)
    const int kk = std::min(S.keep, m);
    theta.assign(m, 0.0);
    Sm.assign(size_t(m) * kk, 0.0);
    // The next Krylov block (the newest block of AV orthonormalised against the basis)
    // does not depend on the Ritz pairs: it is formed on the GPU while the host solves
    // the projected problem, and discarded if the check below stops the iteration or
    // switches precision.  On a restart step it goes to the b spare columns past mmax
    // and continues the restarted basis when the basis satisfies the block Arnoldi
    // relation and the block kept every direction: the residuals of the Ritz vectors
    // then lie in the span of that block, so it is the same continuation as the
    // orthonormalised residuals (otherwise the residuals are used).
    const int add_next = int(std::min<int64_t>(S.b, N - S.m));
    const bool speculate = overlap && add_next > 0;
    // the Ritz vectors are formed on the second stream from V, AV[:, :m] as they stand now
    // (the next block written below only touches columns >= m)
    const hipStream_t rs = S.s2 ? S.s2 : S.s;
    if (rs != S.s) {
        if ((st = S.check(hipEventRecord(S.ev, S.s), "event")) != KL_OK) return st;
        if ((st = S.check(hipStreamWaitEvent(rs, S.ev, 0), "event wait")) != KL_OK) return st;
    }
    const bool spec_apply = speculate && max_rel > 10.0 * tol;
    bool blk_full = false;                  // the speculative block kept every direction
    bool eig_ok = false;
    double eig_s = 0.0;
    auto solve_projected = [&]() {
        const auto te0 = clock::now();
        // (the batched solver's runs, which proceed in parallel on host threads, keep off the
        // host team)
        eig_ok = sym_eig_top(m, Hm.data(), kk, theta.data(), Sm.data(), overlap);
        eig_s = std::chrono::duration<double>(clock::now() - te0).count();
    };
    if (speculate) {
        std::thread worker(solve_projected);
        st = S.check(hipMemcpyAsync(S.W, S.AV + int64_t(S.m - S.last) * N, size_t(N) * S.last * 8,
                                    hipMemcpyDeviceToDevice, S.s), "copy block");
        // C still holds V^T AV[:, m - last:m] from update_H, the first product of the
        // orthonormalisation of this block
        if (st == KL_OK) st = S.orth_into_basis(S.W, S.last, add_next, rng, true);
        blk_full = add_next == S.last && !S.last_refilled;
        // while the previous check was far from the criterion, the operator application
        // of the next block is queued as well, so that it runs on the GPU while the host
        // still solves the projected problem (near convergence it would be wasted)
        if (st == KL_OK && spec_apply)
            st = S.apply(precision, S.V + int64_t(S.m) * N, S.AV + int64_t(S.m) * N, add_next);
        worker.join();
        if (st != KL_OK) return st;
    } else {
        solve_projected();
    }
    t_host_eig += eig_s;
    if (!eig_ok) { set_error("kl_eigs: projected eigenproblem did not converge"); return KL_ENUMERIC; }
    for (double t : theta)
        if (!std::isfinite(t)) { set_error("kl_eigs: non-finite Ritz value"); return KL_ENUMERIC; }
    // X = V S[:, :kk] -> Vt,  AX = AV S[:, :kk] -> AVt, residuals R = AX - X Theta and their
    // norms, on the Rayleigh-Ritz stream: the check below need not wait for the operator
    // application of the next block queued on the main stream
    std::copy(Sm.begin(), Sm.begin() + size_t(m) * kk, S.pin_S);
    if ((st = S.check(hipMemcpyAsync(S.C2, S.pin_S, size_t(m) * kk * 8, hipMemcpyHostToDevice, rs), "copy S")) != KL_OK)
        return st;
    if ((st = S.gemm_nn(S.V, m, S.C2, m, kk, 1.0, 0.0, S.Vt, rs)) != KL_OK) return st;
    if ((st = S.gemm_nn(S.AV, m, S.C2, m, kk, 1.0, 0.0, S.AVt, rs)) != KL_OK) return st;
    std::copy(theta.begin(), theta.begin() + kk, S.pin_theta);
    if ((st = S.check(hipMemcpyAsync(S.dtheta, S.pin_theta, size_t(kk) * 8, hipMemcpyHostToDevice, rs),
                      "copy theta")) != KL_OK)
        return st;
    launch_residual(S.Vt, S.AVt, S.dtheta, N, N, kk, S.R, S.rpart, S.dnorm, rs);
    if ((st = S.check(hipMemcpyAsync(S.pin_norm, S.dnorm, size_t(kk) * 8, hipMemcpyDeviceToHost, rs),
                      "copy norms")) != KL_OK)
        return st;
    // every later use of Vt, AVt, R and dtheta is queued after this host synchronisation
    if ((st = S.wait(rs)) != KL_OK) return st;
    norms.assign(S.pin_norm, S.pin_norm + kk);
    const double t1 = std::fabs(theta[0]);
    converged = 0;
    max_rel = 0.0;
    bool lo_ok = true;
    const int kc = std::min(S.k, kk);
    for (int i = 0; i < kc; ++i) {
        const double target = std::max(tol * std::fabs(theta[i]), floor_rel * t1);
        if (norms[i] <= target) ++converged;
        max_rel = std::max(max_rel, norms[i] / std::max(std::fabs(theta[i]), 1e-300));
        if (norms[i] > std::max(target, lo_floor * t1)) lo_ok = false;
    }
    const bool all = converged == kc && kc == S.k;
    // stagnation of the low-precision phase: no halving of the largest relative
    // residual over three Rayleigh-Ritz steps
    if (precision != KL_F64) {
        if (max_rel < 0.5 * best_lo) { best_lo = max_rel; stall = 0; }
        else if (++stall >= 3) lo_ok = true;
    }
    if (precision == KL_F64 || !refine) {
        if (all || S.m >= N) { done = true; return KL_OK; }
    } else if (lo_ok || S.m >= N) {
        // ---- switch to FP64: recompute AV of the kept Ritz basis --------------------
        precision = KL_F64;
        std::swap(S.V, S.Vt);
        S.m = kk;
        S.restarts += 1;
        set_pending(KL_F64, S.V, S.AV, kk, AFTER_SWITCH);
        return KL_OK;
    }
    if (total_applies >= max_applies) { done = true; return KL_OK; }
    if (speculate && !must_restart) {
        // the next block was formed and applied above
        last_add = add_next;
        pending_keeps_krylov = blk_full;
        set_pending(precision, S.V + int64_t(S.m) * N, S.AV + int64_t(S.m) * N, add_next, AFTER_EXPAND);
        pending_done = spec_apply;
        return KL_OK;
    }
    if (speculate && krylov_ok && blk_full) {
        // ---- thick restart continued by the speculative block ------------------------
        // kept Ritz vectors X (and AX) are in Vt[:, :kk] (AVt); the block formed above is
        // orthonormal to the old basis, hence to X: it moves next to them
        if ((st = S.check(hipMemcpyAsync(S.Vt + int64_t(kk) * N, S.V + int64_t(m) * N, size_t(N) * add_next * 8,
                                         hipMemcpyDeviceToDevice, S.s), "copy block")) != KL_OK)
            return st;
        if (spec_apply &&
            (st = S.check(hipMemcpyAsync(S.AVt + int64_t(kk) * N, S.AV + int64_t(m) * N, size_t(N) * add_next * 8,
                                         hipMemcpyDeviceToDevice, S.s), "copy block")) != KL_OK)
            return st;
        std::swap(S.V, S.Vt);
        std::swap(S.AV, S.AVt);
        S.m = kk;
        std::fill(S.H.begin(), S.H.end(), 0.0);
        for (int i = 0; i < kk; ++i) S.H[size_t(i) * S.mmax + i] = theta[i];
        S.restarts += 1;
        last_add = add_next;
        pending_keeps_krylov = true;
        set_pending(precision, S.V + int64_t(kk) * N, S.AV + int64_t(kk) * N, add_next, AFTER_EXPAND);
        pending_done = spec_apply;
        return KL_OK;
    }
    const int add = int(std::min<int64_t>(S.b, N - (must_restart ? kk : S.m)));
    if (must_restart) {
        // ---- thick restart -------------------------------------------------------
        const int newest = S.last;
        std::swap(S.V, S.Vt);
        std::swap(S.AV, S.AVt);
        S.m = kk;
        std::fill(S.H.begin(), S.H.end(), 0.0);
        for (int i = 0; i < kk; ++i) S.H[size_t(i) * S.mmax + i] = theta[i];
        S.restarts += 1;
        // residuals of the kept vectors are in R (residual_kernel above).  If the old
        // basis had the Arnoldi relation they span at most as many directions as its
        // newest block had columns, and the restarted basis keeps the relation when all
        // of them are kept; a newest block wider than `add` (the one that follows the
        // switch to FP64 holds every residual direction of the kept vectors) loses it
        if (add <= 0) { done = true; return KL_OK; }
        if ((st = S.orth_into_basis(S.R, kk, add, rng)) != KL_OK) return st;
        pending_keeps_krylov = newest <= add && !S.last_refilled;
    } else {
        // ---- block Krylov expansion from the newest block of AV --------------------
        if (add <= 0) { done = true; return KL_OK; }
        if ((st = S.check(hipMemcpyAsync(S.W, S.AV + int64_t(S.m - S.last) * N, size_t(N) * S.last * 8,
                                         hipMemcpyDeviceToDevice, S.s), "copy block")) != KL_OK)
            return st;
        if ((st = S.orth_into_basis(S.W, S.last, add, rng)) != KL_OK) return st;
        pending_keeps_krylov = add == S.last && !S.last_refilled;
    }
    last_add = add;
    set_pending(precision, S.V + int64_t(S.m) * N, S.AV + int64_t(S.m) * N, add, AFTER_EXPAND);
    return KL_OK;
}

kl_status EigRun::finish(double *evals, double *evecs, int64_t ldv, kl_eigs_report *rep, double t_solve) {
    const int64_t N = S.N;
    const int kout = std::min<int>(S.k, int(theta.size()));
    for (int i = 0; i < S.k; ++i) evals[i] = i < kout ? theta[i] : 0.0;
    launch_copy_cols(S.Vt, N, evecs, ldv, N, kout, S.s);
    // B-spline coefficients v = L^{-T} v' (Sec. 4.1); W (N x cmax >= k columns) is free now
    if (coeffs && kout > 0) launch_to_coefficients(P, evecs, ldv, kout, S.W, S.s);
    kl_status st = S.check(hipGetLastError(), "coefficient transform");
    if (st != KL_OK) return st;
    if ((st = S.check(hipStreamSynchronize(S.s), "sync")) != KL_OK) return st;
    if (rep) {
        for (int p = 0; p < 4; ++p) {
            rep->n_applies[p] = S.applies[p];
            rep->n_block_applies[p] = S.block_applies[p];
        }
        rep->n_restarts = S.restarts;
        rep->converged = converged;
        rep->t_setup = P->t_setup;
        rep->t_solve = t_solve;
        rep->t_host_eig = t_host_eig;
        rep->max_rel_residual = max_rel;
    }
    if (converged < S.k) {
        std::ostringstream os;
        os << "kl_eigs: " << converged << " of " << S.k << " pairs converged within " << max_applies << " applies";
        set_error(os.str());
        return KL_ENOCONV;
    }
    return KL_OK;
}

}  // namespace kl

using namespace kl;

extern "C" kl_status kl_eigs(kl_problem *P, const kl_eigs_opts *opts, const double *x0,
                             int32_t nvec0, double *evals, double *evecs, int64_t ldv,
                             kl_eigs_report *rep, void *stream) {
    using clock = std::chrono::steady_clock;
    const auto t0 = clock::now();
    if (!P || P->host_only) { set_error("kl_eigs: NULL or host-only handle"); return KL_EINVAL; }
    if (!opts || !evals || !evecs) { set_error("kl_eigs: NULL argument"); return KL_EINVAL; }
    if (ldv < P->hs.N) { set_error("kl_eigs: ldv < N"); return KL_EINVAL; }
    if (nvec0 < 0 || (nvec0 > 0 && !x0)) { set_error("kl_eigs: bad start block"); return KL_EINVAL; }
    EigRun run;
    kl_status st = run.configure(P, opts);
    if (st != KL_OK) return st;
    if ((st = order_after(P, static_cast<hipStream_t>(stream))) != KL_OK) return st;
    if ((st = run.begin(x0, nvec0)) != KL_OK) return st;
    while (!run.done) {
        if (!run.pending_done &&
            (st = run.S.apply(run.pending_prec, run.pending_x, run.pending_y, run.pending_cols)) != KL_OK)
            return st;
        if ((st = run.after_apply()) != KL_OK) return st;
    }
    return run.finish(evals, evecs, ldv, rep, std::chrono::duration<double>(clock::now() - t0).count());
}

namespace kl {
namespace {

// Runs fn(i) for i < n on up to 16 host threads.
template <typename F>
void parallel_for(int n, F fn) {
    const int hw = int(std::max(1u, std::thread::hardware_concurrency()));
    const int T = std::min(n, std::min(16, hw));
    if (T <= 1) {
        for (int i = 0; i < n; ++i) fn(i);
        return;
    }
    std::atomic<int> next(0);
    std::vector<std::thread> th;
    th.reserve(T);
    for (int t = 0; t < T; ++t)
        th.emplace_back([&]() {
            for (;;) {
                const int i = next.fetch_add(1);
                if (i >= n) break;
                fn(i);
            }
        });
    for (auto &t : th) t.join();
}

}  // namespace
}  // namespace kl

// Every problem of the batch runs the same block eigensolver as kl_eigs, in lockstep:
// the operator applications of all runs that wait for one are made by one replay of the
// batch's apply graph (runs that converged are masked off), and the rest of each run's
// step (orthogonalisation, Rayleigh-Ritz, restarts) proceeds on host threads, each run
// on its own stream.
extern "C" kl_status kl_eigs_batch(kl_batch *B, const kl_eigs_opts *opts, double *evals, double *evecs,
                                   kl_eigs_report *reps, void *stream) {
    using clock = std::chrono::steady_clock;
    const auto t0 = clock::now();
    if (!B || !opts || !evals || !evecs) { set_error("kl_eigs_batch: NULL argument"); return KL_EINVAL; }
    if (opts->precision != KL_F64 && opts->precision != KL_F32) {
        set_error("kl_eigs_batch: the batched path supports KL_F64 and KL_F32");
        return KL_EINVAL;
    }
    const int n = batch_size(B);
    std::vector<EigRun> runs(n);
    std::vector<kl_status> stv(n, KL_OK);
    std::vector<std::string> msg(n);
    std::vector<int64_t> N(n), off(n);
    for (int i = 0; i < n; ++i) {
        kl_status st = kl_batch_info(B, i, &N[i], nullptr, &off[i]);
        if (st == KL_OK) st = runs[i].configure(batch_problem(B, i), opts);
        if (st != KL_OK) return st;
        runs[i].overlap = false;      // the runs already proceed in parallel on host threads
    }
    auto first_error = [&]() -> kl_status {
        for (int i = 0; i < n; ++i)
            if (stv[i] != KL_OK && stv[i] != KL_ENOCONV) {
                std::ostringstream os;
                os << "kl_eigs_batch: problem " << i << ": " << msg[i];
                set_error(os.str());
                return stv[i];
            }
        return KL_OK;
    };
    auto record = [&](int i, kl_status st) {
        stv[i] = st;
        if (st != KL_OK) msg[i] = kl_last_error();
    };
    for (int i = 0; i < n; ++i) {
        kl_status st0 = order_after(batch_problem(B, i), static_cast<hipStream_t>(stream));
        if (st0 != KL_OK) return st0;
    }
    parallel_for(n, [&](int i) { record(i, runs[i].begin(nullptr, 0)); });
    kl_status st = first_error();
    if (st != KL_OK) return st;
    hipStream_t bs = batch_stream(B);
    std::vector<hipEvent_t> ev(n, nullptr);
    hipEvent_t evb = nullptr;
    auto release = [&]() {
        for (hipEvent_t e : ev)
            if (e) (void)hipEventDestroy(e);
        if (evb) (void)hipEventDestroy(evb);
    };
    for (int i = 0; i < n && st == KL_OK; ++i)
        if (hipEventCreateWithFlags(&ev[i], hipEventDisableTiming) != hipSuccess) st = KL_EHIP;
    if (st == KL_OK && hipEventCreateWithFlags(&evb, hipEventDisableTiming) != hipSuccess) st = KL_EHIP;
    if (st != KL_OK) { release(); set_error("kl_eigs_batch: event creation failed"); return st; }
    std::vector<int> nv(n);
    std::vector<const double *> xs(n);
    std::vector<double *> ys(n);
    for (;;) {
        bool any = false;
        for (int i = 0; i < n; ++i) any = any || !runs[i].done;
        if (!any) break;
        const int precs[2] = {int(opts->precision), opts->precision == KL_F64 ? -1 : int(KL_F64)};
        for (int prec : precs) {
            if (prec < 0) continue;
            int maxcols = 0;
            for (int i = 0; i < n; ++i)
                if (!runs[i].done && runs[i].pending_cols > 0 && runs[i].pending_prec == prec)
                    maxcols = std::max(maxcols, runs[i].pending_cols);
            if (maxcols == 0) continue;
            for (int i = 0; i < n; ++i)
                if (!runs[i].done && runs[i].pending_cols > 0 && runs[i].pending_prec == prec) {
                    (void)hipEventRecord(ev[i], runs[i].S.s);
                    (void)hipStreamWaitEvent(bs, ev[i], 0);
                }
            for (int c0 = 0; c0 < maxcols && st == KL_OK; c0 += kBW) {
                for (int i = 0; i < n; ++i) {
                    const bool part = !runs[i].done && runs[i].pending_prec == prec && runs[i].pending_cols > c0;
                    nv[i] = part ? std::min(kBW, runs[i].pending_cols - c0) : 0;
                    xs[i] = part ? runs[i].pending_x + int64_t(c0) * N[i] : nullptr;
                    ys[i] = part ? runs[i].pending_y + int64_t(c0) * N[i] : nullptr;
                }
                st = batch_apply(B, prec, nv.data(), xs.data(), N.data(), ys.data(), N.data(), bs);
            }
            if (st != KL_OK) { release(); return st; }
            (void)hipEventRecord(evb, bs);
            for (int i = 0; i < n; ++i)
                if (!runs[i].done && runs[i].pending_cols > 0 && runs[i].pending_prec == prec) {
                    (void)hipStreamWaitEvent(runs[i].S.s, evb, 0);
                    runs[i].count_apply(prec, runs[i].pending_cols);
                }
        }
        parallel_for(n, [&](int i) {
            if (!runs[i].done) record(i, runs[i].after_apply());
        });
        if ((st = first_error()) != KL_OK) { release(); return st; }
    }
    const double t_solve = std::chrono::duration<double>(clock::now() - t0).count();
    parallel_for(n, [&](int i) {
        const int k = runs[i].S.k;
        record(i, runs[i].finish(evals + int64_t(i) * k, evecs + int64_t(k) * off[i], N[i], reps ? reps + i : nullptr,
                                 t_solve));
    });
    release();
    if ((st = first_error()) != KL_OK) return st;
    for (int i = 0; i < n; ++i)
        if (stv[i] == KL_ENOCONV) {
            std::ostringstream os;
            os << "kl_eigs_batch: problem " << i << ": " << msg[i];
            set_error(os.str());
            return KL_ENOCONV;
        }
    return KL_OK;
}
