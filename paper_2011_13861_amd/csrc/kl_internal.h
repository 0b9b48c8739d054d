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
    void *Y5d = nullptr;                   // stage-5 input, FP64 (column-major, ld Ntpad)
    void *Y5f = nullptr;                   // stage-5 input, FP32; padding rows stay zero
    void *Y5b = nullptr;                   // stage-5 input, BF16 hi then lo part
    size_t y5_bytes = 0;
    void *Z5 = nullptr;                    // stage-5 split partial sums (scratch)
    size_t z5_bytes = 0;
    void *Zf = nullptr;                    // stage-5 output (column-major, ld Ntpad)
    int max_split = 1;
};

// Device buffers, stream and rocBLAS handle of the block eigensolver, kept with the
// problem between kl_eigs calls (grown on demand, freed by kl_destroy).
struct SolverCache;
void free_solver_cache(SolverCache *c);

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
    kl::SolverCache *solver = nullptr;
    int n_cu = 256;
    bool host_only = false;   // built by kl_setup_host: no device data
    // stage-5 tuning per kl_precision: 32-row blocks per wave (2 or 4) and forced split
    // count (0 = automatic); set by kl_stage5_config
    int s5_rb[4] = {2, 2, 2, 2};
    int s5_split[4] = {0, 0, 0, 0};
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
// One direction of a Kronecker product (see kernels_kron.hip for the index layout):
//   OUT[a + A(o + nout c) + out_ldj j] = out_w[p] * sum_i D[o][i] IN'[a + A(i + nin c)]
//   IN'[q] = in_scale * in_w[q] * sum_{s < nsplit} in[q + in_ldj j + s in_split]
struct ModeSpec {
    const double *D = nullptr;      // nout x nin, row-major, FP64
    const double *DT = nullptr;     // the same factor transposed (nin x nout)
    const void *in = nullptr;
    void *out = nullptr;
    int64_t A = 1;
    int nin = 1, nout = 1;
    int64_t Clo = 1;
    int nvec = 1;
    int64_t in_ldj = 0, out_ldj = 0;
    int nsplit = 1;
    int64_t in_split = 0;
    const double *in_w = nullptr;
    double in_scale = 1.0;
    const double *out_w = nullptr;
    void *out_lo = nullptr;         // BF16 output: low parts (hi/lo split), or NULL
    bool in_f32 = false, out_f32 = false, out_bf16 = false;
};
// true if a factor (nout x nin) fits the LDS-staged MFMA kernel
bool mode_fits(int nin, int nout);
void launch_mode(const ModeSpec &m, hipStream_t s);
// Copies a strided column block (FP64).
void launch_copy_cols(const double *src, int64_t lds, double *dst, int64_t ldd, int64_t rows,
                      int cols, hipStream_t s);
// Stage-5 input from an FP64 block (no scaling): Y5[j*Ntpad + p] = y[p + ldy j], p < Nt.
void launch_pack_stage5(int precision, const double *y, int64_t ldy, int64_t Nt, int nvec,
                        int64_t Ntpad, void *Y5, hipStream_t s);
// Stage-5 output to FP64: z[p + ldz j] = scale * sum_s Z5[s][j*Ntpad + p].
void launch_unpack_stage5(int precision, const void *Z5, int nsplit, int64_t Ntpad, int64_t Nt,
                          int nvec, double scale, double *z, int64_t ldz, hipStream_t s);
// C (m x c, column-major, ld m) = A^T B for tall-skinny FP64 blocks; `part` holds
// 64 * m * c doubles of row-range partials.
int gram_splits(int64_t N, int m, int c, int n_cu);
void launch_gram(const double *A, int64_t lda, int m, const double *B, int64_t ldb, int c,
                 int64_t N, double *part, double *C, int n_cu, hipStream_t s);

// Stage-5 launch geometry: rows per workgroup, and the number of l-splits (forced > 0
// overrides the automatic choice); *lchunk receives the l-range length of one split.
int64_t stage5_rows_per_wg(int precision, int rb);
int stage5_splits(int64_t Ntpad, int64_t rows_wg, int n_cu, int max_split, int forced,
                  int64_t *lchunk);
// Stage 5: Z5[s][k][j] = sum_{l in split s} Gamma(x_k, x_l) Y5[l][j] for all k < Ntpad.
// Returns the number of splits used.
// Stage 5: Zf[j][k] = sum_l Gamma(x_k, x_l) Y5[j][l]; Z5 holds split partials (scratch).
int launch_stage5(const kl_problem *P, int precision, const void *Y5, void *Z5, void *Zf,
                  hipStream_t s);

}  // namespace kl
