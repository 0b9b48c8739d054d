// Internal declarations of the KL library (not part of the C ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/kl.h"

namespace kl {

// Stage 5 processes blocks of this many columns per pass.
constexpr int kBW = 32;
// Greville grids are padded to a multiple of this many points (zero rows/columns).
constexpr int kPad = 256;

void set_error(const std::string &msg);

// Host-side setup data, built in FP64 (Sec. 3.5, 4.1-4.3).
struct HostSetup {
    int d = 0;
    int p[3] = {1, 1, 1}, ne[3] = {1, 1, 1}, pt[3] = {1, 1, 1}, net[3] = {1, 1, 1};
    int n[3] = {1, 1, 1}, nt[3] = {1, 1, 1};
    int64_t N = 0, Nt = 0;
    std::vector<double> C[3];   // composed factor C_k (nt_k x n_k, row-major)
    std::vector<double> X;      // Nt x d, physical Greville points, vec order
    std::vector<double> J;      // Nt, sqrt(det DF)
};

// Dense symmetric eigensolver (row-major A, descending w, column-major Z); false if the
// QR iteration fails to converge.
bool sym_eig(int n, const double *A, double *w, double *Z);

// Fills `hs` from the description; returns KL_OK or an error (message set).
kl_status build_host_setup(const kl_desc &desc, HostSetup &hs);

struct Workspace {
    double *T0 = nullptr, *T1 = nullptr;   // FP64 Kronecker ping-pong buffers
    size_t t_elems = 0;                    // elements per buffer (max intermediate x kBW)
    void *Y5 = nullptr;                    // stage-5 input block, kernel layout
    size_t y5_bytes = 0;
    void *Z5 = nullptr;                    // stage-5 split partial sums
    size_t z5_bytes = 0;
    int max_split = 1;
};

}  // namespace kl

struct kl_problem {
    kl::HostSetup hs;
    int cov_kind = 0;
    double sigma2 = 1.0;
    double ell[3] = {1, 1, 1};
    int64_t Ntpad = 0;
    // device data
    double *dX64 = nullptr;   // [d][Ntpad], coordinates scaled for the FP64 kernel
    float *dX32 = nullptr;    // [d][Ntpad], coordinates scaled for the exp2-based kernels
    double *dJ = nullptr;     // [Ntpad], sqrt(det DF); zero in the padding
    double *dC[3] = {nullptr, nullptr, nullptr};    // C_k, nt_k x n_k row-major
    double *dCT[3] = {nullptr, nullptr, nullptr};   // C_k^T, n_k x nt_k row-major
    kl::Workspace ws;
    int n_cu = 256;
    bool host_only = false;   // built by kl_setup_host: no device data
    // optional stage-5 timing with HIP events (kl_profile_enable / kl_profile_read)
    bool prof_on = false;
    std::vector<hipEvent_t> prof_ev;      // pool: 2 events per timed launch
    std::vector<int> prof_prec;           // precision of each recorded launch
    size_t prof_used = 0;
    int64_t prof_count[4] = {0, 0, 0, 0};
    double prof_ms[4] = {0, 0, 0, 0};
};

namespace kl {

// ---- kernels (launch wrappers; all asynchronous on `s`) ---------------------------
// Mode-k contraction on column-major FP64 tensors:
//   out[a + A*(o + nout*c)] = sum_i D[o*nin + i] * in[a + A*(i + nin*c)],
//   a < A, o < nout, c < Cn (Cn includes the column index).
void launch_mode_contract(const double *D, const double *in, double *out, int64_t A, int nin,
                          int nout, int64_t Cn, hipStream_t s);
// Forward epilogue: Y5[p, j] = J[p] * T[p + ldt*j] in stage-5 precision and layout
// (J may be NULL: no scaling), zero for p >= Nt or j >= nvec.
void launch_to_stage5(int precision, const double *T, int64_t Nt, int64_t ldt, int nvec,
                      const double *J, int64_t Ntpad, void *Y5, hipStream_t s);
// Backward prologue: T[p + Nt*j] = scale * w[p] * sum_s Z5[s][p][j].
void launch_from_stage5(int precision, const void *Z5, int nsplit, int64_t Ntpad, int64_t Nt,
                        int nvec, const double *w, double scale, double *T, int64_t ldt,
                        hipStream_t s);
// Copies a strided column block (FP64) into / out of a packed one.
void launch_copy_cols(const double *src, int64_t lds, double *dst, int64_t ldd, int64_t rows,
                      int cols, hipStream_t s);

// Number of l-splits of stage 5 for a padded grid; *lchunk receives the l-range length.
int stage5_splits(int64_t Ntpad, int n_cu, int64_t *lchunk);
// Stage 5: Z5[s][k][j] = sum_{l in split s} Gamma(x_k, x_l) Y5[l][j] for all k < Ntpad.
// Returns the number of splits used.
int launch_stage5(const kl_problem *P, int precision, const void *Y5, void *Z5, hipStream_t s);

}  // namespace kl
