// FP64 block kernels of the eigensolver: C = A^T B for tall-skinny A (N x m) and
// B (N x c), N >> m, c (the Gram matrices of the Rayleigh-Ritz projection and of the
// Gram-Schmidt reorthogonalisation), and Out = alpha A S + beta Out for a tall-skinny A
// and a small S (Ritz vectors, projections).
//
// Gram products: the N rows are split into G <= 256 ranges of at least two slabs, so that short
// products still spread over the chip.  A workgroup owns one (64 x 64 tile of C, row
// range) pair: it stages 32-row slabs of the 64 columns of A and of B in LDS (loads
// coalesced along the rows, the next slab prefetched into registers while the current
// one is used) and accumulates 16 entries per thread with FP64 FMAs.  The partials are
// stored output-major, part[e][g], so that the reduction is one wave per output entry:
// coalesced loads of G values and a cross-lane sum, in a fixed order.
#include <algorithm>

#include "kl_internal.h"

namespace kl {
namespace {

constexpr int kT = 64;         // C tile edge
constexpr int kSlab = 32;      // rows per LDS slab
constexpr int kThreads = 256;  // 16 x 16 threads, 4 x 4 entries each
constexpr int kG = 256;        // maximum number of row ranges

__global__ __launch_bounds__(kThreads) void gram_partial_kernel(
    const double *__restrict__ A, int64_t lda, int m, const double *__restrict__ B, int64_t ldb,
    int c, int64_t N, int64_t rows_per_range, double *__restrict__ part) {
    __shared__ double sA[kSlab][kT + 1];
    __shared__ double sB[kSlab][kT + 1];
    const int i0 = blockIdx.x * kT, j0 = blockIdx.y * kT;
    const int g = blockIdx.z;
    const int64_t n0 = int64_t(g) * rows_per_range;
    const int64_t n1 = min(N, n0 + rows_per_range);
    const int ti = threadIdx.x % 16, tj = threadIdx.x / 16;
    double acc[4][4];
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int v = 0; v < 4; ++v) acc[u][v] = 0.0;
    constexpr int kPer = (kSlab * kT) / kThreads;       // 8 elements of A and of B per thread
    double pa[kPer], pb[kPer];
    auto load = [&](int64_t ns) {
#pragma unroll
        for (int q = 0; q < kPer; ++q) {
            const int e = threadIdx.x + q * kThreads;
            const int r = e % kSlab, col = e / kSlab;
            const int64_t n = ns + r;
            pa[q] = (n < n1 && i0 + col < m) ? A[(i0 + col) * lda + n] : 0.0;
            pb[q] = (n < n1 && j0 + col < c) ? B[(j0 + col) * ldb + n] : 0.0;
        }
    };
    if (n0 < n1) load(n0);
    for (int64_t ns = n0; ns < n1; ns += kSlab) {
        __syncthreads();
#pragma unroll
        for (int q = 0; q < kPer; ++q) {
            const int e = threadIdx.x + q * kThreads;
            const int r = e % kSlab, col = e / kSlab;
            sA[r][col] = pa[q];
            sB[r][col] = pb[q];
        }
        __syncthreads();
        if (ns + kSlab < n1) load(ns + kSlab);
#pragma unroll 4
        for (int r = 0; r < kSlab; ++r) {
            double a[4], b[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) a[u] = sA[r][ti + 16 * u];
#pragma unroll
            for (int v = 0; v < 4; ++v) b[v] = sB[r][tj + 16 * v];
#pragma unroll
            for (int u = 0; u < 4; ++u)
#pragma unroll
                for (int v = 0; v < 4; ++v) acc[u][v] = fma(a[u], b[v], acc[u][v]);
        }
    }
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int i = i0 + ti + 16 * u, j = j0 + tj + 16 * v;
            if (i < m && j < c) part[(int64_t(j) * m + i) * gridDim.z + g] = acc[u][v];
        }
}

// One wave per entry of C: sums part[e][0..G-1] across lanes.
__global__ __launch_bounds__(kThreads) void gram_reduce_kernel(const double *__restrict__ part,
                                                               int G, int64_t mc,
                                                               double *__restrict__ C) {
    const int lane = threadIdx.x & 63;
    const int64_t e = int64_t(blockIdx.x) * (kThreads / 64) + (threadIdx.x >> 6);
    if (e >= mc) return;
    double v = 0.0;
    for (int g = lane; g < G; g += 64) v += part[e * G + g];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    if (lane == 0) C[e] = v;
}

// Out (N x c) = alpha A (N x m) S (m x c) + beta Out, column-major, on
// v_mfma_f64_16x16x4_f64 in the transposed form Out^T = S^T A^T: A operand S^T[j][k] in
// lane j + 16 k, B operand A^T[k][i] = A[i + lda k] in lane i + 16 k (16 consecutive
// rows of one column: coalesced), accumulator r of lane L = Out^T[(L >> 4) + 4 r][L & 15].
// A workgroup owns 16 rows of Out and NT tiles of 16 columns (all of c up to 128, so
// that A is read once); its 4 waves split the contraction (wave w takes the 4-wide
// k-steps s = w mod 4), with the operands of the next batch of steps in flight while the
// current one runs on the matrix cores.  The four partial tiles are added in LDS in
// wave order and stored with alpha and beta (beta = 0 does not read Out).
typedef double doublex4 __attribute__((ext_vector_type(4)));
constexpr int kNNBatch = 2;      // k-steps per wave per batch of loads
constexpr int kNNMaxTiles = 8;   // column tiles per workgroup

template <int NT>
__global__ __launch_bounds__(kThreads) void gemm_nn_kernel(const double *__restrict__ A, int64_t lda, int m,
                                                           const double *__restrict__ S, int64_t lds, int c,
                                                           int64_t N, double alpha, double beta,
                                                           double *__restrict__ Out, int64_t ldo) {
    extern __shared__ double red_nn[];                     // [4][16][16 NT + 1]
    constexpr int ldr = 16 * NT + 1;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int li = lane & 15, lk = lane >> 4;
    const int64_t row0 = int64_t(blockIdx.x) * 16;
    const int j0 = blockIdx.y * 16 * NT;
    const int64_t rowc = min(row0 + li, N - 1);            // clamped: rows past N are not stored
    const int steps = (m + 3) / 4;
    doublex4 acc[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) acc[t] = doublex4{0.0, 0.0, 0.0, 0.0};
    // batch q of this wave: steps w + 4 (kNNBatch q + u), u < kNNBatch
    auto load = [&](int q, double (&a)[kNNBatch], double (&b)[kNNBatch][NT]) {
#pragma unroll
        for (int u = 0; u < kNNBatch; ++u) {
            const int k = 4 * (w + 4 * (kNNBatch * q + u)) + lk;
            const bool kok = k < m;
            const int kc = kok ? k : m - 1;
            const double va = A[rowc + lda * kc];
            a[u] = kok ? va : 0.0;
#pragma unroll
            for (int t = 0; t < NT; ++t) {
                const int j = j0 + 16 * t + li;
                const double vs = S[kc + lds * min(j, c - 1)];
                b[u][t] = (kok && j < c) ? vs : 0.0;
            }
        }
    };
    auto mma = [&](const double (&a)[kNNBatch], const double (&b)[kNNBatch][NT]) {
#pragma unroll
        for (int u = 0; u < kNNBatch; ++u)
#pragma unroll
            for (int t = 0; t < NT; ++t) acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(b[u][t], a[u], acc[t], 0, 0, 0);
    };
    const int nbatch = (steps + 4 * kNNBatch - 1) / (4 * kNNBatch);
    double a0[kNNBatch], b0[kNNBatch][NT], a1[kNNBatch], b1[kNNBatch][NT];
    if (nbatch > 0) load(0, a0, b0);                       // m = 0: no loads, Out = beta Out
    for (int q = 0; q < nbatch; q += 2) {
        if (q + 1 < nbatch) load(q + 1, a1, b1);
        mma(a0, b0);
        if (q + 1 >= nbatch) break;
        if (q + 2 < nbatch) load(q + 2, a0, b0);
        mma(a1, b1);
    }
    // partial tiles -> LDS: acc[t][r] of lane L = Out[row0 + (L & 15)][j0 + 16 t + (L >> 4) + 4 r]
#pragma unroll
    for (int t = 0; t < NT; ++t)
#pragma unroll
        for (int r = 0; r < 4; ++r) red_nn[(w * 16 + li) * ldr + 16 * t + lk + 4 * r] = acc[t][r];
    __syncthreads();
    for (int e = threadIdx.x; e < 16 * 16 * NT; e += kThreads) {
        const int i = e & 15, jj = e >> 4;
        const int64_t row = row0 + i;
        const int j = j0 + jj;
        if (row < N && j < c) {
            double v = red_nn[i * ldr + jj];
#pragma unroll
            for (int ww = 1; ww < 4; ++ww) v += red_nn[(ww * 16 + i) * ldr + jj];
            double *o = Out + row + ldo * j;
            *o = beta == 0.0 ? alpha * v : alpha * v + beta * *o;
        }
    }
}

template <int NT>
void launch_gemm_nn_t(const double *A, int64_t lda, int m, const double *S, int64_t lds, int c, int64_t N,
                      double alpha, double beta, double *Out, int64_t ldo, hipStream_t s) {
    const size_t lds_bytes = size_t(4) * 16 * (16 * NT + 1) * sizeof(double);
    // once per process (thread-safe initialisation of a function-local static)
    static const bool attr = [lds_bytes] {
        (void)hipFuncSetAttribute(reinterpret_cast<const void *>(&gemm_nn_kernel<NT>),
                                  hipFuncAttributeMaxDynamicSharedMemorySize, int(lds_bytes));
        return true;
    }();
    (void)attr;
    const dim3 grid(unsigned((N + 15) / 16), unsigned((c + 16 * NT - 1) / (16 * NT)));
    hipLaunchKernelGGL((gemm_nn_kernel<NT>), grid, dim3(kThreads), lds_bytes, s, A, lda, m, S, lds, c, N, alpha,
                       beta, Out, ldo);
}

}  // namespace

int gram_splits(int64_t N, int m, int c, int n_cu) {
    (void)m; (void)c; (void)n_cu;
    int64_t g = (N + 2 * kSlab - 1) / (2 * kSlab);     // at least two slabs per range
    if (g > kG) g = kG;
    if (g < 1) g = 1;
    return int(g);
}

// C (m x c, column-major, ld m) = A^T B with A: N x m (ld lda), B: N x c (ld ldb).
// `part` needs gram_splits(N, ...) * m * c doubles (at most 256 m c).
void launch_gram(const double *A, int64_t lda, int m, const double *B, int64_t ldb, int c,
                 int64_t N, double *part, double *C, int n_cu, hipStream_t s) {
    const int G0 = gram_splits(N, m, c, n_cu);
    int64_t rows = (N + G0 - 1) / G0;
    rows = (rows + kSlab - 1) / kSlab * kSlab;
    const int G = int((N + rows - 1) / rows);
    dim3 grid((m + kT - 1) / kT, (c + kT - 1) / kT, G);
    hipLaunchKernelGGL(gram_partial_kernel, grid, dim3(kThreads), 0, s, A, lda, m, B, ldb, c, N, rows,
                       part);
    const int64_t mc = int64_t(m) * c;
    hipLaunchKernelGGL(gram_reduce_kernel, dim3(unsigned((mc + 3) / 4)), dim3(kThreads), 0, s, part,
                       G, mc, C);
}

void launch_gemm_nn(const double *A, int64_t lda, int m, const double *S, int64_t lds, int c, int64_t N,
                    double alpha, double beta, double *Out, int64_t ldo, hipStream_t s) {
    if (N < 1 || c < 1) return;
    if (m < 1) {                        // empty contraction: Out = beta Out
        if (beta != 1.0) launch_gemm_nn_t<1>(A, lda, 0, S, lds, c, N, alpha, beta, Out, ldo, s);
        return;
    }
    switch (std::min(kNNMaxTiles, (c + 15) / 16)) {
    case 1: launch_gemm_nn_t<1>(A, lda, m, S, lds, c, N, alpha, beta, Out, ldo, s); break;
    case 2: launch_gemm_nn_t<2>(A, lda, m, S, lds, c, N, alpha, beta, Out, ldo, s); break;
    case 3: launch_gemm_nn_t<3>(A, lda, m, S, lds, c, N, alpha, beta, Out, ldo, s); break;
    case 4: launch_gemm_nn_t<4>(A, lda, m, S, lds, c, N, alpha, beta, Out, ldo, s); break;
    case 5: launch_gemm_nn_t<5>(A, lda, m, S, lds, c, N, alpha, beta, Out, ldo, s); break;
    case 6: launch_gemm_nn_t<6>(A, lda, m, S, lds, c, N, alpha, beta, Out, ldo, s); break;
    case 7: launch_gemm_nn_t<7>(A, lda, m, S, lds, c, N, alpha, beta, Out, ldo, s); break;
    default: launch_gemm_nn_t<8>(A, lda, m, S, lds, c, N, alpha, beta, Out, ldo, s); break;
    }
}

}  // namespace kl
