// Truncated KL expansion at the interpolation Greville points (Sec. 3.2): zero-mean field
// samples sum_i sqrt(lambda_i) phi_i(x) xi_i and the variance sum_i lambda_i phi_i(x)^2, with
// phi_i = (sum_j v_j B_j) / sqrt(det DF) (Sec. 3.4) and v = L^{-T} v' (Sec. 4.1).
//
// Per chunk of up to 32 eigenvectors: the Kronecker product of the factors E_k = B_k(g) L_k^{-T}
// (one per-direction launch each, the forward-stage kernel with E_k in place of C_k) gives
// the unscaled values in the stage-5 output buffer; one pass scales row x by 1 / J(x) and
// column i by sqrt(lambda_i) and adds the squares to the variance; the samples are then one
// tall-skinny product with the chunk's rows of xi (the eigensolver's FP64 matrix-core GEMM),
// accumulated over chunks.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>

#include "kl_internal.h"

namespace kl {
namespace {

struct ColScale {
    double v[kBW];
};

// Phi[row][i] *= sqrt(lambda_i) / J[row]; var[row] (+)= sum_i Phi[row][i]^2.  One thread per
// row; the columns are read row-contiguously (coalesced).
__global__ __launch_bounds__(256) void kle_scale_kernel(double *__restrict__ Phi, int64_t ldp, int64_t Nt,
                                                         int nb, const double *__restrict__ J, ColScale cs,
                                                         double *__restrict__ var, int first) {
    const int64_t row = int64_t(blockIdx.x) * 256 + threadIdx.x;
    if (row >= Nt) return;
    const double inv = 1.0 / J[row];
    double acc = 0.0;
    for (int i = 0; i < nb; ++i) {
        const double v = Phi[int64_t(i) * ldp + row] * inv * cs.v[i];
        Phi[int64_t(i) * ldp + row] = v;
        acc = fma(v, v, acc);
    }
    if (var) var[row] = first ? acc : var[row] + acc;
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
    for (int i = 0; i < M; ++i)
        if (!(lam[i] >= 0.0) || !std::isfinite(lam[i])) {
            set_error("kl_kle_field: eigenvalues must be finite and >= 0"); return KL_EINVAL;
        }
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int d = hs.d;
    double *Phi = static_cast<double *>(P->ws.Zf);        // Ntpad x kBW, column-major
    for (int c0 = 0; c0 < M; c0 += kBW) {
        const int nb = std::min(kBW, M - c0);
        const void *cur = evecs + int64_t(c0) * ldv;
        int64_t cur_ld = ldv, A = 1;
        for (int k = 0; k < d; ++k) {
            ModeSpec ms;
            ms.D = P->dE[k];
            ms.DT = P->dET[k];
            ms.in = cur;
            ms.in_ldj = cur_ld;
            ms.A = A;
            ms.nin = hs.n[k];
            ms.nout = hs.nt[k];
            ms.Clo = 1;
            for (int j = k + 1; j < d; ++j) ms.Clo *= hs.n[j];
            ms.nvec = nb;
            if (k == d - 1) {
                ms.out = Phi;
                ms.out_ldj = P->Ntpad;
            } else {
                ms.out = (cur == P->ws.T0) ? P->ws.T1 : P->ws.T0;
                ms.out_ldj = A * hs.nt[k] * ms.Clo;
            }
            launch_mode(ms, s);
            A *= hs.nt[k];
            cur = ms.out;
            cur_ld = ms.out_ldj;
        }
        ColScale cs{};
        for (int i = 0; i < nb; ++i) cs.v[i] = std::sqrt(lam[c0 + i]);
        hipLaunchKernelGGL(kle_scale_kernel, dim3(unsigned((hs.Nt + 255) / 256)), dim3(256), 0, s, Phi,
                           P->Ntpad, hs.Nt, nb, P->dJ, cs, var, c0 == 0 ? 1 : 0);
        if (want_f)
            launch_gemm_nn(Phi, P->Ntpad, nb, xi + c0, ldxi, m, hs.Nt, 1.0, c0 == 0 ? 0.0 : 1.0, F, ldf, s);
    }
    if (hipGetLastError() != hipSuccess) { set_error("kl_kle_field: kernel launch failed"); return KL_EHIP; }
    return KL_OK;
}
