// Truncated KL expansion at the interpolation Greville points (Sec. 3.2): zero-mean field
// samples sum_i sqrt(lambda_i) phi_i(x) xi_i and the variance sum_i lambda_i phi_i(x)^2, with
// phi_i = (sum_j v_j B_j) / sqrt(det DF) (Sec. 3.4) and v = L^{-T} v' (Sec. 4.1).
//
// Per chunk of up to 32 eigenvectors: the Kronecker product of the factors E_k = B_k(g) L_k^{-T}
// (one per-direction launch each, the forward-stage kernel with E_k in place of C_k) gives
// the unscaled values in the stage-5 output buffer; one more launch scales row x by 1 / J(x)
// and column i by sqrt(lambda_i), adds the squares to the variance and accumulates the
// chunk's part of the samples (a contraction of at most 32 terms per output: FP64 FMAs in
// registers, bound by writing F).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>

#include "kl_internal.h"

namespace kl {
namespace {

struct ColScale {
    double v[kBW];
};

// One chunk of nb <= 32 eigenfunctions, Phi[row][i] unscaled (column-major, ld ldp).  The
// thread of row x runs over i, forming phi_i(x) sqrt(lambda_i) = Phi[x][i] sqrt(lambda_i) / J[x]
// one at a time: the workgroups of column group 0 add its square to the variance, and with
// WITH_F every workgroup adds its products with xi[i][j] to kCols columns of F (F[x][j] (+)=
// sum_i phi_i(x) sqrt(lambda_i) xi[i][j]), which stay in registers.  Rows run along the
// threads, so the Phi reads and the F accesses are coalesced; sqrt(lambda_i) and the group's
// xi entries sit in LDS (every lane reads the same word: a broadcast).
constexpr int kCols = 16;

template <bool WITH_F>
__global__ __launch_bounds__(256) void kle_field_kernel(const double *__restrict__ Phi, int64_t ldp, int64_t Nt,
                                                         int nb, const double *__restrict__ J, ColScale cs,
                                                         const double *__restrict__ xi, int64_t ldxi, int m,
                                                         double *__restrict__ F, int64_t ldf,
                                                         double *__restrict__ var, int first) {
    __shared__ double ssl[kBW];
    __shared__ double sxi[kBW][kCols];
    const int64_t row = int64_t(blockIdx.x) * 256 + threadIdx.x;
    const bool live = row < Nt;
    const int64_t r = live ? row : Nt - 1;                  // clamped: dead rows store nothing
    const int j0 = int(blockIdx.y) * kCols;
    if (threadIdx.x < kBW) ssl[threadIdx.x] = cs.v[threadIdx.x];
    if constexpr (WITH_F) {
        for (int e = threadIdx.x; e < kCols * kBW; e += 256) {
            const int c = e % kCols, i = e / kCols;
            sxi[i][c] = (j0 + c < m && i < nb) ? xi[int64_t(j0 + c) * ldxi + i] : 0.0;
        }
    }
    const int nc = min(kCols, m - j0);
    double acc[kCols];
#pragma unroll
    for (int c = 0; c < kCols; ++c)
        acc[c] = (WITH_F && !first && live && c < nc) ? F[int64_t(j0 + c) * ldf + row] : 0.0;
    const double inv = 1.0 / J[r];
    __syncthreads();
    double vs = 0.0;
#pragma unroll 4
    for (int i = 0; i < nb; ++i) {
        const double v = Phi[int64_t(i) * ldp + r] * inv * ssl[i];
        vs = fma(v, v, vs);
        if constexpr (WITH_F)
#pragma unroll
            for (int c = 0; c < kCols; ++c) acc[c] = fma(v, sxi[i][c], acc[c]);
    }
    if (!live) return;
    if (var && blockIdx.y == 0) var[row] = first ? vs : var[row] + vs;
    if constexpr (WITH_F)
#pragma unroll
        for (int c = 0; c < kCols; ++c)
            if (c < nc) F[int64_t(j0 + c) * ldf + row] = acc[c];
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
    if (want_f && (int64_t(m) + kCols - 1) / kCols > 65535) {
        set_error("kl_kle_field: more than 1048560 samples per call"); return KL_EINVAL;
    }
    for (int i = 0; i < M; ++i)
        if (!(lam[i] >= 0.0) || !std::isfinite(lam[i])) {
            set_error("kl_kle_field: eigenvalues must be finite and >= 0"); return KL_EINVAL;
        }
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int d = hs.d;
    double *Phi = static_cast<double *>(P->ws.Zf);        // Ntpad x kBW, column-major
    for (int c0 = 0; c0 < M; c0 += kBW) {
        const int nb = std::min(kBW, M - c0);
        // the trial functions at the Greville points, patch by patch on the patch's rows
        for (int pi = 0; pi < patch_count(P); ++pi) {
            const kl_problem *Q = patch_of(P, pi);
            const HostSetup &qs = Q->hs;
            const void *cur = evecs + int64_t(c0) * ldv + patch_noff(P, pi);
            int64_t cur_ld = ldv, A = 1;
            for (int k = 0; k < d; ++k) {
                ModeSpec ms;
                ms.D = Q->dE[k];
                ms.DT = Q->dET[k];
                ms.in = cur;
                ms.in_ldj = cur_ld;
                ms.A = A;
                ms.nin = qs.n[k];
                ms.nout = qs.nt[k];
                ms.Clo = 1;
                for (int j = k + 1; j < d; ++j) ms.Clo *= qs.n[j];
                ms.nvec = nb;
                if (k == d - 1) {
                    ms.out = Phi + patch_toff(P, pi);
                    ms.out_ldj = P->Ntpad;
                } else {
                    ms.out = (cur == P->ws.T0) ? P->ws.T1 : P->ws.T0;
                    ms.out_ldj = A * qs.nt[k] * ms.Clo;
                }
                launch_mode(ms, s);
                A *= qs.nt[k];
                cur = ms.out;
                cur_ld = ms.out_ldj;
            }
        }
        ColScale cs{};
        for (int i = 0; i < nb; ++i) cs.v[i] = std::sqrt(lam[c0 + i]);
        const unsigned groups = want_f ? unsigned((m + kCols - 1) / kCols) : 1u;
        const dim3 grid(unsigned((hs.Nt + 255) / 256), groups);
        if (want_f)
            hipLaunchKernelGGL(kle_field_kernel<true>, grid, dim3(256), 0, s, Phi, P->Ntpad, hs.Nt, nb, P->dJ, cs,
                               xi + c0, ldxi, m, F, ldf, var, c0 == 0 ? 1 : 0);
        else
            hipLaunchKernelGGL(kle_field_kernel<false>, grid, dim3(256), 0, s, Phi, P->Ntpad, hs.Nt, nb, P->dJ, cs,
                               nullptr, ldxi, 0, nullptr, ldf, var, c0 == 0 ? 1 : 0);
    }
    if (hipGetLastError() != hipSuccess) { set_error("kl_kle_field: kernel launch failed"); return KL_EHIP; }
    return KL_OK;
}
