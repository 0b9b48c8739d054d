// Internal declarations of the warm-start network kernels (not part of the C ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>

namespace kl {
namespace mlp {

enum Epilogue { EPI_NONE = 0, EPI_BIAS = 1, EPI_BIAS_TANH = 2, EPI_DTANH = 3, EPI_ADAM = 4 };

// Adam step with bias correction c1 = 1 - b1^t, c2 = 1 - b2^t, applied through their
// reciprocals ic1 = 1 / c1, ic2 = 1 / c2 (rounded from FP64 on the host).
struct AdamArgs {
    float lr, b1, b2, eps, ic1, ic2;
};

// C = op(A) op(B) with an epilogue; logical A is M x K, logical B is K x N:
//   A(i, k) = TA ? A[k lda + i] : A[i lda + k],  B(k, j) = TB ? B[j ldb + k] : B[k ldb + j].
// Epilogues: EPI_BIAS  C = AB + bias[j];  EPI_BIAS_TANH  C = tanh(AB + bias[j]);
// EPI_DTANH  C = AB * (1 - aux[i][j]^2).
// EPI_ADAM (float4 form with one K range only, see adam_fusable in the network code): AB
// is the gradient of the parameters at C, whose Adam moments sit at am and av with the
// same layout (leading dimension ldc); the three are updated in place and no gradient is
// stored.
struct GemmArgs {
    const float *A = nullptr;
    int64_t lda = 0;
    const float *B = nullptr;
    int64_t ldb = 0;
    float *C = nullptr;
    int64_t ldc = 0;
    int M = 0, N = 0, K = 0;
    int kchunk = 0;                 // K range of one split (multiple of the K chunk)
    const float *bias = nullptr;
    const float *aux = nullptr;
    int64_t ldaux = 0;
    int epi = EPI_NONE;
    float *part = nullptr;          // splits x M x N partials when split over K
    float *am = nullptr, *av = nullptr;   // Adam moments (EPI_ADAM)
    AdamArgs adam{};
    // float4 form with TA, not TB and one K range only: the column sums of B (the bias
    // gradient of a weight-gradient product) go to colsum[N], or with EPI_ADAM take the Adam
    // step of the parameters at colsum (moments bm, bv)
    float *colsum = nullptr, *bm = nullptr, *bv = nullptr;
};

// Parameter ranges [off[r], off[r] + len) of one Adam launch, given as off[] and the
// running ends end[r] = len_0 + ... + len_r.  A range that starts where the previous one
// ends extends it.  Capacity: two ranges (weights and biases) for each of at most 16 layers.
constexpr int kAdamRanges = 32;
struct AdamRanges {
    int n = 0;
    int64_t off[kAdamRanges] = {};
    int64_t end[kAdamRanges] = {};
    void add(int64_t o, int64_t len) {
        if (n > 0 && off[n - 1] + (end[n - 1] - (n > 1 ? end[n - 2] : 0)) == o) {
            end[n - 1] += len;
            return;
        }
        off[n] = o;
        end[n] = (n ? end[n - 1] : 0) + len;
        ++n;
    }
};

// Whether the float4 form of the product applies: A and B 16-byte aligned, lda and ldb
// multiples of 4, and the contiguous extent of each operand (K or M for A, N or K for B)
// a multiple of 4.
bool gemm_vec_ok(bool ta, bool tb, const GemmArgs &g);
// Whether a product goes to the one-thread-per-output kernel instead of matrix tiles: fan-in
// K <= kDirectK and at most kDirectOut outputs (never for EPI_ADAM).
constexpr int kDirectK = 8;
constexpr int64_t kDirectOut = 65536;
bool gemm_direct_ok(const GemmArgs &g);
void launch_gemm_direct(bool ta, bool tb, const GemmArgs &g, hipStream_t s);
// Number of K splits for a launch (partials limited to part_cap floats); *kchunk
// receives the K range of one split (a multiple of the form's K chunk: 64 for the float4
// form, 32 otherwise).
int gemm_splits(int M, int N, int K, int n_cu, int64_t part_cap, bool vec, int *kchunk);
void launch_gemm(bool ta, bool tb, bool vec, GemmArgs g, int splits, hipStream_t s);
void launch_loss(const float *y, int64_t ldy, const float *t, int64_t ldt, const int *rows, int batch,
                 int n_out, int group, int signed_, float *dy, int64_t lddy, double *loss_part,
                 hipStream_t s);
// Subspace term of the warm-start loss (after launch_loss on the same stream): adds
// weight inv_b (I - P) y_g to dy and 0.5 weight ||(I - P) y_g||^2 to loss_part, P the
// projector onto the sample's target groups; n_out / group <= kMaxSubGroups.  `scratch`
// holds subspace_scratch(batch, n_out, group) doubles (partial sums and coefficients).
constexpr int kMaxSubGroups = 32;
int64_t subspace_scratch(int batch, int n_out, int group);
void launch_subspace(const float *y, int64_t ldy, const float *t, int64_t ldt, const int *rows, int batch,
                     int n_out, int group, float weight, float *dy, int64_t lddy, double *loss_part,
                     double *scratch, hipStream_t s);
void launch_colsum(const float *D, int64_t ldd, int M, int N, float *out, hipStream_t s);
void launch_adam(float *p, const float *g, float *m, float *v, int64_t n, const AdamArgs &a, hipStream_t s);
void launch_adam_ranges(float *p, const float *g, float *m, float *v, const AdamRanges &r, const AdamArgs &a,
                        hipStream_t s);
void launch_gather(const float *src, int64_t lds, const int *rows, int nrows, int ncols, float *dst,
                   hipStream_t s);

}  // namespace mlp
}  // namespace kl
