// Truncated KL expansion at the interpolation Greville points (Sec. 3.2): zero-mean field
// samples sum_i sqrt(lambda_i) phi_i(x) xi_i and the variance sum_i lambda_i phi_i(x)^2, with
// phi_i = (sum_j v_j B_j) / sqrt(det DF) (Sec. 3.4) and v = L^{-T} v' (Sec. 4.1).
//
// The Kronecker product of the factors E_k = B_k(g) L_k^{-T} (the forward stages of the
// operator with E_k in place of C_k, all modes of a pass in one call where the buffer holds
// their intermediates, else 32 at a time; the first two directions in one launch where the
// operator fuses them) gives the unscaled values of all modes of a pass in
// the split-partials buffer; one more launch forms
// A[x][i] = Phi[x][i] sqrt(lambda_i) / J(x) while staging it, adds its squares to the
// variance, and computes F = A xi on the FP64 matrix cores, each sample column of F written
// once per pass (one pass unless the modes exceed what the buffer holds).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>

#include "kl_internal.h"

namespace kl {
namespace {

typedef double doublex4 __attribute__((ext_vector_type(4)));

constexpr int kKgRows = 64;      // rows of F per workgroup (4 waves x 16)
constexpr int kKgCols = 64;      // samples of F per workgroup (4 tiles of 16 per wave)
constexpr int kKgK = 32;         // modes staged in LDS per step
constexpr int kKgMaxModes = 256; // modes per pass (their sqrt(lambda) travel in the arguments)

struct ModeScale {
    double v[kKgMaxModes];
};

// Largest leading dimension of xi and F for which the lane offsets of a tile, in bytes,
// fit in 32 bits (7 ldxi + 31 and 3 ldf + 63 elements): the loads and stores then take one
// scalar base per row or column and a fixed 32-bit lane offset, with no per-lane 64-bit
// address arithmetic.  Larger leading dimensions, and tiles on the sample or row edge, take
// per-lane clamped 64-bit addresses.
constexpr int64_t kKgNarrowLd = int64_t(1) << 26;

template <typename T>
__device__ __forceinline__ const T *at_bytes(const T *base, uint32_t off) {
    return reinterpret_cast<const T *>(reinterpret_cast<const char *>(base) + off);
}
template <typename T>
__device__ __forceinline__ T *at_bytes(T *base, uint32_t off) {
    return reinterpret_cast<T *>(reinterpret_cast<char *>(base) + off);
}

struct KgLds {
    double A[kKgK][kKgRows + 1];   // A^T chunk [mode][row]
    double B[kKgK][kKgCols + 1];   // xi chunk [mode][sample]
    double V[4][kKgRows];          // variance partials of the four waves
};

// Staging loads of one chunk of kKgK modes from k0 (see kle_gemm_tile), into registers.
template <bool WITH_F, bool INTERIOR, int UA, int UB>
__device__ __forceinline__ void kg_load_chunk(double (&av)[UA], double (&bv)[UB], const double *__restrict__ Phi,
                                              int64_t ldp, int64_t row0, uint32_t offA, int wave, int K, int k0,
                                              const double *__restrict__ xi, int64_t ldxi, int m, int j0, int bs,
                                              int bk) {
    const int kc = min(kKgK, K - k0);
#pragma unroll
    for (int u = 0; u < UA; ++u) av[u] = *at_bytes(Phi + int64_t(k0 + min(wave + 4 * u, kc - 1)) * ldp + row0, offA);
    if constexpr (WITH_F) {
        if constexpr (INTERIOR) {
            const uint32_t offB = (uint32_t(bs) * uint32_t(ldxi) + uint32_t(min(bk, kc - 1))) * 8u;
#pragma unroll
            for (int u = 0; u < UB; ++u) bv[u] = *at_bytes(xi + int64_t(j0 + 8 * u) * ldxi + k0, offB);
        } else {
#pragma unroll
            for (int u = 0; u < UB; ++u) {
                const int col = min(j0 + bs + 8 * u, m - 1);
                bv[u] = xi[int64_t(col) * ldxi + k0 + min(bk, kc - 1)];
            }
        }
    }
}

// One tile of kle_gemm_kernel.  INTERIOR: the tile's 64 rows and 64 samples lie inside F
// and the leading dimensions are narrow, so xi and F are addressed by a scalar base per
// sample column plus a fixed 32-bit lane offset; otherwise every lane clamps its own 64-bit
// addresses into the arrays.  The two forms are separate branches of the kernel, so that
// neither form's address set-up runs on the other's tiles.
template <bool WITH_F, bool INTERIOR>
__device__ __forceinline__ void kle_gemm_tile(KgLds &L, const double *__restrict__ Phi, int64_t ldp, int64_t Nt,
                                              int K, const double *__restrict__ J, const ModeScale &sc,
                                              const double *__restrict__ xi, int64_t ldxi, int m,
                                              double *__restrict__ F, int64_t ldf, double *__restrict__ var,
                                              int first, int64_t row0, int j0) {
    const int tid = threadIdx.x;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6), lane = tid & 63;
    const int li = lane & 15, lk = lane >> 4;
    // A staging: a thread stages row `lane` of the tile for modes wave + 4 u; rows past Nt
    // read row Nt - 1 and are zeroed by the factor 1/J = 0
    const bool row_live = row0 + lane < Nt;
    const double sinv = row_live ? 1.0 / J[row0 + lane] : 0.0;
    const uint32_t offA = uint32_t(min(int64_t(lane), Nt - 1 - row0)) * 8u;
    // B staging: a thread stages mode bk of samples bs + 8 u (modes contiguous in xi)
    const int bs = tid >> 5, bk = tid & (kKgK - 1);
    double vpart = 0.0;
    doublex4 acc[kKgCols / 16];
#pragma unroll
    for (int t = 0; t < kKgCols / 16; ++t)
#pragma unroll
        for (int r = 0; r < 4; ++r) acc[t][r] = 0.0;
    constexpr int kUA = (kKgK * kKgRows) / 256, kUB = (kKgK * kKgCols) / 256;
    // every load of a chunk is issued before the first wait; addresses are clamped into the
    // arrays and the out-of-range values replaced by zeros in LDS.  The next chunk's loads are
    // issued once this chunk is in LDS, so that they are in flight during its products.
    double av[kUA], bv[WITH_F ? kUB : 1];
    kg_load_chunk<WITH_F, INTERIOR>(av, bv, Phi, ldp, row0, offA, wave, K, 0, xi, ldxi, m, j0, bs, bk);
    for (int k0 = 0; k0 < K; k0 += kKgK) {
        const int kc = min(kKgK, K - k0);
        __syncthreads();
#pragma unroll
        for (int u = 0; u < kUA; ++u) {
            const int kk = wave + 4 * u;
            const double a = av[u] * (kk < kc ? sc.v[k0 + kk] : 0.0) * sinv;
            L.A[kk][lane] = a;
            vpart = fma(a, a, vpart);
        }
        if constexpr (WITH_F) {
            if (INTERIOR && kc == kKgK) {
#pragma unroll
                for (int u = 0; u < kUB; ++u) L.B[bk][bs + 8 * u] = bv[u];
            } else {
#pragma unroll
                for (int u = 0; u < kUB; ++u) L.B[bk][bs + 8 * u] = (bk < kc && j0 + bs + 8 * u < m) ? bv[u] : 0.0;
            }
        }
        __syncthreads();
        if (k0 + kKgK < K)
            kg_load_chunk<WITH_F, INTERIOR>(av, bv, Phi, ldp, row0, offA, wave, K, k0 + kKgK, xi, ldxi, m, j0, bs, bk);
        if constexpr (WITH_F) {
            const int nkq = (kc + 3) / 4;
#pragma unroll
            for (int kq = 0; kq < kKgK / 4; ++kq) {
                if (kq < nkq) {
                    const double b = L.A[4 * kq + lk][16 * wave + li];
#pragma unroll
                    for (int t = 0; t < kKgCols / 16; ++t)
                        acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(L.B[4 * kq + lk][16 * t + li], b, acc[t], 0, 0, 0);
                }
            }
        }
    }
    if (var && j0 == 0) {
        L.V[wave][lane] = vpart;
        __syncthreads();
        if (tid < kKgRows && row0 + tid < Nt) {
            const double v = ((L.V[0][tid] + L.V[1][tid]) + L.V[2][tid]) + L.V[3][tid];
            var[row0 + tid] = first ? v : var[row0 + tid] + v;
        }
    }
    if constexpr (WITH_F) {
        // D[(lane >> 4) + 4 r][lane & 15]: sample 16 t + lk + 4 r, row 16 wave + li
        if constexpr (INTERIOR) {
            const uint32_t offF = (uint32_t(lk) * uint32_t(ldf) + uint32_t(16 * wave + li)) * 8u;
            if (!first) {
                // later mode passes add to the stored field: all reads first
#pragma unroll
                for (int t = 0; t < kKgCols / 16; ++t)
#pragma unroll
                    for (int r = 0; r < 4; ++r)
                        acc[t][r] += *at_bytes(F + int64_t(j0 + 16 * t + 4 * r) * ldf + row0, offF);
            }
#pragma unroll
            for (int t = 0; t < kKgCols / 16; ++t)
#pragma unroll
                for (int r = 0; r < 4; ++r) *at_bytes(F + int64_t(j0 + 16 * t + 4 * r) * ldf + row0, offF) = acc[t][r];
        } else {
            const int64_t row = row0 + 16 * wave + li;
            if (!first) {
                const int64_t rc = min(row, Nt - 1);
#pragma unroll
                for (int t = 0; t < kKgCols / 16; ++t)
#pragma unroll
                    for (int r = 0; r < 4; ++r)
                        acc[t][r] += F[int64_t(min(j0 + 16 * t + lk + 4 * r, m - 1)) * ldf + rc];
            }
            if (row < Nt)
#pragma unroll
                for (int t = 0; t < kKgCols / 16; ++t)
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const int j = j0 + 16 * t + lk + 4 * r;
                        if (j < m) F[int64_t(j) * ldf + row] = acc[t][r];
                    }
        }
    }
}

// One pass over K <= kKgMaxModes modes (Phi columns 0..K-1, unscaled, column-major ld ldp):
// A[x][i] = Phi[x][i] s_i / J[x];  var[x] (+)= sum_i A[x][i]^2 (workgroups of sample tile 0);
// with WITH_F, F[x][j] (+)= sum_i A[x][i] xi[i][j] for the workgroup's 64 rows x 64 samples
// (v_mfma_f64_16x16x4f64 with A operand xi^T and B operand A^T, so that the accumulators of a
// lane hold 16 consecutive rows of one sample: 128-byte stores).  first = 1 writes, 0 adds.
// narrow = ldxi and ldf are at most kKgNarrowLd.  One-dimensional grid over the tiles of F:
// workgroup b takes sample tile b % nct of row tile b / nct, so that consecutive workgroups
// stage the same rows of Phi.
template <bool WITH_F>
__global__ __launch_bounds__(256, 4) void kle_gemm_kernel(const double *__restrict__ Phi, int64_t ldp, int64_t Nt,
                                                        int K, const double *__restrict__ J, ModeScale sc,
                                                        const double *__restrict__ xi, int64_t ldxi, int m,
                                                        double *__restrict__ F, int64_t ldf,
                                                        double *__restrict__ var, int first, int narrow,
                                                        int nct) {
    __shared__ KgLds L;
    const int64_t row0 = int64_t(blockIdx.x / unsigned(nct)) * kKgRows;
    const int j0 = int(blockIdx.x % unsigned(nct)) * kKgCols;
    const bool interior = WITH_F && narrow && j0 + kKgCols <= m && row0 + kKgRows <= Nt;
    if (interior)
        kle_gemm_tile<WITH_F, true>(L, Phi, ldp, Nt, K, J, sc, xi, ldxi, m, F, ldf, var, first, row0, j0);
    else
        kle_gemm_tile<WITH_F, false>(L, Phi, ldp, Nt, K, J, sc, xi, ldxi, m, F, ldf, var, first, row0, j0);
}

}  // namespace
}  // namespace kl

using namespace kl;

extern "C" kl_status kl_kle_field(kl_problem *P, int32_t M, const double *lam, const double *evecs,
                                  int64_t ldv, int32_t m, const double *xi, int64_t ldxi, double *F,
                                  int64_t ldf, double *var, void *stream) {
    if (!P || P->host_only) { set_error("kl_kle_field: NULL or host-only handle"); return KL_EINVAL; }
    const HostSetup &hs = P->hs;
    if (M < 1 || m < 0) { set_error("kl_kle_field: need M >= 1 and m >= 0"); return KL_EINVAL; }
    if (!lam || !evecs || ldv < hs.N) { set_error("kl_kle_field: NULL eigenpairs or ldv < N"); return KL_EINVAL; }
    const bool want_f = F != nullptr && m > 0;
    if (!want_f && !var) { set_error("kl_kle_field: neither F nor var requested"); return KL_EINVAL; }
    if (want_f && (!xi || ldxi < M || ldf < hs.Nt)) {
        set_error("kl_kle_field: NULL xi, ldxi < M or ldf < Ntilde"); return KL_EINVAL;
    }
    const int64_t n_row_tiles = (hs.Nt + kKgRows - 1) / kKgRows;
    const int64_t n_col_tiles = want_f ? (int64_t(m) + kKgCols - 1) / kKgCols : 1;
    if (n_row_tiles * n_col_tiles > int64_t(INT32_MAX)) {
        set_error("kl_kle_field: ceil(Ntilde / 64) * ceil(m / 64) must be below 2^31"); return KL_EINVAL;
    }
    for (int i = 0; i < M; ++i)
        if (!(lam[i] >= 0.0) || !std::isfinite(lam[i])) {
            set_error("kl_kle_field: eigenvalues must be finite and >= 0"); return KL_EINVAL;
        }
    hipStream_t s = static_cast<hipStream_t>(stream);
    // The unscaled values of a pass's modes go to the split-partials buffer (Ntpad x K).  A
    // pass is evaluated in one forward call (every mode at once) when both Kronecker
    // intermediates of its K modes fit behind them in that buffer and the mode kernels' row
    // counts (intermediate x K) stay in 32 bits, and that takes no more passes than chunks of
    // kBW modes through the workspace's intermediates would; otherwise it runs in such chunks.
    double *Phi = static_cast<double *>(P->ws.Z5);
    const int64_t z5_elems = int64_t(P->ws.z5_bytes / sizeof(double));
    const int64_t tmax = (problem_max_intermediate(P) + 31) / 32 * 32;
    const int64_t rows_max = std::max<int64_t>(std::max<int64_t>(tmax, P->Ntpad), hs.N);
    const int64_t wide = std::min<int64_t>(std::min<int64_t>(kKgMaxModes, z5_elems / (P->Ntpad + 2 * tmax)),
                                           (int64_t(INT32_MAX) - 1) / rows_max);
    const int chunked_pass =
        int(std::min<int64_t>(kKgMaxModes, std::max<int64_t>(kBW, z5_elems / P->Ntpad / kBW * kBW)));
    const bool one_call = wide >= std::min(M, chunked_pass);
    const int per_pass = one_call ? int(wide) : chunked_pass;
    const int chunk = one_call ? per_pass : kBW;
    for (int p0 = 0; p0 < M; p0 += per_pass) {
        const int K = std::min(per_pass, M - p0);
        double *T0 = one_call ? Phi + int64_t(per_pass) * P->Ntpad : P->ws.T0;
        double *T1 = one_call ? T0 + int64_t(per_pass) * tmax : P->ws.T1;
        for (int c0 = 0; c0 < K; c0 += chunk) {
            const int nb = std::min(chunk, K - c0);
            // the trial functions at the Greville points, patch by patch on the patch's rows
            const bool fuse = fused_directions(P, nb);
            for (int pi = 0; pi < patch_count(P); ++pi) {
                const kl_problem *Q = patch_of(P, pi);
                forward_patch(Q, Q->dE, Q->dET, fuse, 0, nb, evecs + int64_t(p0 + c0) * ldv + patch_noff(P, pi), ldv,
                              Phi + int64_t(c0) * P->Ntpad + patch_toff(P, pi), nullptr, P->Ntpad, nullptr, T0, T1,
                              s);
            }
        }
        ModeScale sc{};
        for (int i = 0; i < K; ++i) sc.v[i] = std::sqrt(lam[p0 + i]);
        const int first = p0 == 0 ? 1 : 0;
        const int narrow = (ldxi <= kKgNarrowLd && ldf <= kKgNarrowLd) ? 1 : 0;
        if (want_f) {
            hipLaunchKernelGGL(kle_gemm_kernel<true>, dim3(unsigned(n_row_tiles * n_col_tiles)), dim3(256), 0, s, Phi,
                               P->Ntpad, hs.Nt, K, P->dJ, sc, xi + p0, ldxi, m, F, ldf, var, first, narrow,
                               int(n_col_tiles));
        } else {
            hipLaunchKernelGGL(kle_gemm_kernel<false>, dim3(unsigned(n_row_tiles)), dim3(256), 0, s, Phi, P->Ntpad,
                               hs.Nt, K, P->dJ, sc, nullptr, ldxi, 0, nullptr, ldf, var, first, 0, 1);
        }
    }
    if (hipGetLastError() != hipSuccess) { set_error("kl_kle_field: kernel launch failed"); return KL_EHIP; }
    return KL_OK;
}
