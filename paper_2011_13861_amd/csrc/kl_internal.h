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
    std::vector<double> E[3];   // B_k(Greville points of the interpolation space) L_k^{-T} (nt_k x n_k)
    std::vector<double> LT[3];  // L_k^{-T} (n_k x n_k, row-major, upper triangular)
    std::vector<double> X;      // Nt x d, physical Greville points, vec order
    std::vector<double> J;      // Nt, sqrt(det DF)
};

// Dense symmetric eigensolver (row-major A, descending w, column-major Z); false if the
// QR iteration fails to converge.
bool sym_eig(int n, const double *A, double *w, double *Z);
// All eigenvalues (descending) and the eigenvectors of the nv largest (Z: n x nv).
bool sym_eig_partial(int n, const double *A, double *w, double *Z, int nv);
// The nv largest eigenvalues only (w[0..nv-1], descending) and their eigenvectors (Z, n x nv),
// parts of the work on the host thread team when use_team is set (same results).
bool sym_eig_top(int n, const double *A, int nv, double *w, double *Z, bool use_team = true);
// T = R^{-1} with G = R^T R (host; false on a pivot <= rel_tol max diag(G)).  min_sine
// (optional) receives min_j R_jj / sqrt(G_jj): the smallest sine of the angle between a
// column and the span of the columns before it (1 for orthogonal columns).
bool chol_orth_transform(int n, const double *G, double *T, double rel_tol, double *min_sine = nullptr);

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
    // symmetric FP64 stage 5 (allocated by kl_stage5_symmetric): forward partials per (row
    // tile, column block), owned partials per work item, and the plan on the device
    // (SymItem[sym_items] followed by int o_first[sym_NB + 1])
    double *symF = nullptr, *symO = nullptr;
    void *symTab = nullptr;
    int sym_items = 0, sym_NB = 0, sym_grid = 0, sym_chunk = 0;
};

// Work item of the symmetric FP64 stage 5: column block J (256 points) against row tiles
// [t0, t1) (64 points each, t1 <= 4 J + 4); its owned partial goes to slot oslot.
struct SymItem {
    int J, t0, t1, oslot;
};
struct SymPlan {
    int NB = 0, chunk = 0, n_items = 0, n_oslots = 0;
    int64_t f_slots = 0;               // forward partial slots: (t, J) for t < 4 J
    std::vector<SymItem> items;        // longest first
    std::vector<int> o_first;          // NB + 1: the owned slots of block J are o_first[J] ..
};

// Device buffers and stream of the block eigensolver, kept with the
// problem between kl_eigs calls (grown on demand, freed by kl_destroy).
struct SolverCache;
void free_solver_cache(SolverCache *c);

}  // namespace kl

struct kl_batch;

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
    double *dE[3] = {nullptr, nullptr, nullptr};    // E_k, nt_k x n_k row-major (kl_kle_field)
    double *dET[3] = {nullptr, nullptr, nullptr};   // E_k^T
    double *dLT[3] = {nullptr, nullptr, nullptr};   // L_k^{-T}, n_k x n_k row-major (coefficients)
    double *dL1[3] = {nullptr, nullptr, nullptr};   // L_k^{-1} (its transpose)
    double t_setup = 0.0;                           // seconds spent in kl_setup
    kl::Workspace ws;
    kl::SolverCache *solver = nullptr;
    int n_cu = 256;
    bool host_only = false;   // built by kl_setup_host: no device data
    // stage-5 tuning per kl_precision: 32-row blocks per wave (2 or 4) and forced split
    // count (0 = automatic); set by kl_stage5_config
    int s5_rb[4] = {2, 2, 2, 2};
    bool fuse_dirs = true;                 // first two directions of each side in one launch
    int s5_split[4] = {0, 0, 0, 0};
    bool s5_sym[4] = {false, false, false, false};   // symmetric stage 5 per precision (kl_stage5_symmetric)
    // optional stage-5 timing with HIP events (kl_profile_enable / kl_profile_read)
    bool prof_on = false;
    std::vector<hipEvent_t> prof_ev;      // pool: 2 events per timed launch
    std::vector<int> prof_prec;           // precision of each recorded launch
    size_t prof_used = 0;
    int64_t prof_count[4] = {0, 0, 0, 0};
    double prof_ms[4] = {0, 0, 0, 0};
    // Several patches (kl_setup_patches): one kl_problem per patch holds that patch's
    // factors (no workspace); this problem holds the points, J, stage-5 buffers and the
    // workspace of the union, and hs carries the totals.  Empty for a single patch.
    std::vector<kl_problem *> patches;
    std::vector<int64_t> noff, toff;      // offsets of each patch's dofs and points
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
// Kernel-side form of a ModeSpec (kernels_kron.hip).
struct ModeArgs {
    const double *D;          // nout x nin row-major
    const double *DT;         // nin x nout row-major (D transposed)
    const void *in;           // TIN
    void *out;                // TOUT
    int64_t A;                // product of the sizes before the direction (1 = first)
    int nin, nout;
    int64_t Clo;              // product of the sizes after the direction
    int nvec;
    int64_t in_ldj, out_ldj;  // distance between vectors
    int nsplit;               // unused (1)
    int64_t in_split;
    const double *in_w;       // optional per-point input scale (times in_scale)
    double in_scale;
    const double *out_w;      // optional per-point output scale
    void *out_lo;             // BF16 output only: low part v - bf16(v), or NULL
};
// Kernel arguments of the fused pair of directions 1 and 2 over 2-D slabs
// (kernels_kron.hip): D1 nout1 x nin1 and D2 nout2 x nin2 row-major FP64; slabs
// s = c + Clo j (c < Clo, j < nvec); input = sum of nsplit partials (stride in_split),
// optionally scaled by in_scale in_w[point]; output optionally scaled by out_w[point].
struct Mode2Args {
    const double *D1, *D2;
    const double *D1T, *D2T;  // the same factors transposed (nin x nout row-major)
    const void *in;
    void *out;
    void *out_lo;             // BF16 output only: low part v - bf16(v), or NULL
    int nin1, nin2, nout1, nout2;
    int Clo, nvec;
    int64_t in_ldj, out_ldj;
    int nsplit;
    int64_t in_split;
    const double *in_w;
    double in_scale;
    const double *out_w;
};
constexpr int kMode2MaxLds = 96 * 1024;
// Whether the fused kernel takes these sizes (LDS, grid limits).
bool mode2_fits(int nin1, int nin2, int nout1, int nout2, int64_t slabs);
// out_kind: 0 FP64, 1 FP32, 2 BF16 output (FP64 input); in_f32: FP32 input, FP64 output.
void launch_mode2(const Mode2Args &a, bool in_f32, int out_kind, hipStream_t s);
ModeArgs mode_args(const ModeSpec &m);
// Workgroups of one launch_mode (4 waves of one 16 x 16 tile each).
int64_t mode_workgroups(const ModeSpec &m);
// One direction for all problems of a batch: args[p] per problem (device), wg_prefix
// (device, nprob + 1 entries) the prefix sums of mode_workgroups; `kind` selects the
// kernel variant (first direction, FP32 input, FP32 / BF16 output) shared by all.
void launch_mode_batch(const ModeSpec &kind, const ModeArgs *args, const int64_t *wg_prefix, int nprob,
                       int64_t total_wgs, const int *active, hipStream_t s);
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
// gram_part_elems(N, m, c) doubles of row-range partials (it grows with m and c).
int gram_splits(int64_t N, int m, int c, int n_cu);
int64_t gram_part_elems(int64_t N, int m, int c);
void launch_gram(const double *A, int64_t lda, int m, const double *B, int64_t ldb, int c,
                 int64_t N, double *part, double *C, int n_cu, hipStream_t s);

// Out (N x c) = alpha A (N x m) S (m x c) + beta Out, FP64 column-major (beta = 0: Out is
// not read).
void launch_gemm_nn(const double *A, int64_t lda, int m, const double *S, int64_t lds, int c, int64_t N,
                    double alpha, double beta, double *Out, int64_t ldo, hipStream_t s);
// R[:, j] = AX[:, j] - theta_j X[:, j] (R may be NULL) and norms[j] = ||R[:, j]||_2 for
// j < kk (device arrays, ld ld); `part` holds residual_chunks(N) * kk doubles.
int residual_chunks(int64_t N);
void launch_residual(const double *X, const double *AX, const double *theta, int64_t N, int64_t ld, int kk,
                     double *R, double *part, double *norms, hipStream_t s);

// Stage-5 launch geometry: rows per workgroup, and the number of l-splits (forced > 0
// overrides the automatic choice); *lchunk receives the l-range length of one split.
int64_t stage5_rows_per_wg(int precision, int rb);
int stage5_splits(int64_t Ntpad, int64_t rows_wg, int n_cu, int max_split, int forced,
                  int64_t *lchunk);
// Stage 5: Zf[j][k] = w_k sum_l Gamma(x_k, x_l) Y5[j][l] with w_k = scale wrow[k] (1 if
// wrow is NULL); Z5 holds split partials (scratch).  Returns the number of splits used.
// Non-NULL ev_start / ev_stop are recorded right before and right after the covariance
// kernel (the split sums that follow are outside).  With defer_reduce and more than one
// split, the split sums are left to the consumer: Z5 then holds the unscaled partials
// (split q of column j at Z5 + (q kBW + j) Ntpad) and Zf is not written.
// max_split caps the split count (the partials buffer Z5 holds that many; 0 = the
// problem's own workspace cap).
int launch_stage5(const kl_problem *P, int precision, const void *Y5, void *Z5, void *Zf,
                  const double *wrow, double scale, hipStream_t s, hipEvent_t ev_start = nullptr,
                  hipEvent_t ev_stop = nullptr, bool defer_reduce = false, int max_split = 0);
// Symmetric stage 5 (KL_F64, KL_BF16, KL_BF16X3) into ws.Zf (same result as launch_stage5
// with one split): the plan of a padded grid (chunk = row tiles per item, 0 = automatic),
// the sizes of its partial buffers (FP64; the BF16 forms use them for FP32 partials), and
// the launch (covariance kernel and ordered reduction, both inside the events).
SymPlan sym_plan(int64_t Ntpad, int n_cu, int chunk);
size_t sym_f_bytes(const SymPlan &pl);
size_t sym_o_bytes(const SymPlan &pl);
void launch_stage5_sym(const kl_problem *P, int precision, const Workspace &ws, const void *Y5,
                       const double *wrow, double scale, hipStream_t s, hipEvent_t ev_start = nullptr,
                       hipEvent_t ev_stop = nullptr);

// kl_setup with or without the single-problem apply workspace (T0/T1, stage-5 buffers);
// problems of a batch use the batch's arenas instead.  Uploads on `s`, then waits for it.
kl_status setup_problem(const kl_desc *desc, bool workspace, hipStream_t s, kl_problem **out);
// kl_setup_patches: one factor-only problem per patch and the union's buffers.
kl_status setup_patches(int npatch, const kl_desc *descs, hipStream_t s, kl_problem **out);
// Standard-form vectors to B-spline coefficients, v = L^{-T} v' (Sec. 4.1), in place on
// nvec columns of x (ld >= N), using `tmp` (N x nvec, ld N) as the ping-pong buffer.
void launch_to_coefficients(const kl_problem *P, double *x, int64_t ldx, int nvec, double *tmp, hipStream_t s);
void destroy_problem(kl_problem *P);
int64_t max_intermediate(const HostSetup &hs);
// Patch i of a problem (the problem itself when it has a single patch), with the offsets
// of its dofs and points in the problem's vectors; the largest Kronecker intermediate
// over the patches.
inline int patch_count(const kl_problem *P) { return P->patches.empty() ? 1 : int(P->patches.size()); }
inline const kl_problem *patch_of(const kl_problem *P, int i) { return P->patches.empty() ? P : P->patches[i]; }
inline int64_t patch_noff(const kl_problem *P, int i) { return P->patches.empty() ? 0 : P->noff[i]; }
inline int64_t patch_toff(const kl_problem *P, int i) { return P->patches.empty() ? 0 : P->toff[i]; }
int64_t problem_max_intermediate(const kl_problem *P);
// Whether the first two directions of each side run as one launch (mode2_kernel) for nb
// columns: for every patch or for none.
bool fused_directions(const kl_problem *P, int nb);
// Forward Kronecker stages of one patch Q with the factors D[k] (nt_k x n_k, row-major) and
// their transposes DT[k]: x (Q's N x nb, ld ldx) -> out (Q's Ntilde rows, ld ldout), FP64
// (y5_kind 0), FP32 (1), BF16 (2) or BF16 pairs (3, low parts to out_lo), times J unless J
// is NULL; T0 and T1 hold the intermediates.
void forward_patch(const kl_problem *Q, const double *const *D, const double *const *DT, bool fuse, int y5_kind,
                   int nb, const double *x, int64_t ldx, void *out, void *out_lo, int64_t ldout, const double *J,
                   double *T0, double *T1, hipStream_t s);
// One chunk (<= kBW columns) of the single-problem apply, on the problem's workspace or
// on `ws` (same layout; its padding rows of the stage-5 inputs must be zero).
kl_status apply_chunk(kl_problem *P, int precision, int nb, const double *x, int64_t ldx, double *y,
                      int64_t ldy, hipStream_t s, const Workspace *ws = nullptr);

// ---- batches of problems (batch.hip) ---------------------------------------------------
int batch_size(const kl_batch *B);
kl_problem *batch_problem(kl_batch *B, int i);
hipStream_t batch_stream(kl_batch *B);
// A~'_i applied to nvec[i] <= kBW columns of each problem i (0 = skip), one graph replay.
kl_status batch_apply(kl_batch *B, int precision, const int *nvec, const double *const *x, const int64_t *ldx,
                      double *const *y, const int64_t *ldy, hipStream_t s);

// ---- batched stage 5 (kernels_stage5.hip) -------------------------------------------
// One problem of a batch: points (FP32 and FP64 scaled copies, [d][Ntpad]), its
// stage-5 input, split partials and output (layouts as for one problem), l-range per
// split and the covariance kind.
struct S5Prob {
    const float *X32;
    const double *X64;
    const void *Y5;
    void *Z5;
    void *Zf;
    int64_t Ntpad, lchunk;
    int nsplit, kind;
    const double *wrow;      // output rows scaled by scale * wrow[row] (sigma^2 J)
    double scale;
};
// One work item: the workgroup-sized row tile `rowtile` of problem `prob` against split
// `split` of its l-range.
struct S5Item {
    int prob, rowtile, split, pad;
};
// Split sum of one problem: Zf[4 e4 + t] = w sum_s Zpart[s stride + 4 e4 + t], e4 < n4,
// w = scale wrow[(4 e4 + t) mod Ntpad]; base4 = sum of n4 over the preceding entries.
struct RedProb {
    const void *Zpart;
    void *Zf;
    int64_t n4, stride, base4, Ntpad;
    int nsplit, prob;
    const double *wrow;
    double scale;
};
// Persistent grid size (workgroups resident at once) of the batched stage-5 kernel.
int stage5_batch_grid(int precision, int d, int rb, int n_cu);
// Resets `counter` and launches the persistent kernel over n_items queue entries.
void launch_stage5_batch(int precision, int d, int rb, const S5Prob *probs, const S5Item *items, int n_items,
                         int *counter, const int *active, int grid, hipStream_t s);
void launch_split_reduce_batch(int precision, const RedProb *probs, int nprob, int64_t total4, const int *active,
                               hipStream_t s);

}  // namespace kl
