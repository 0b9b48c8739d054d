// FP64 block kernels of the eigensolver: C = A^T B for tall-skinny A (N x m) and
// B (N x c), N >> m, c (the Gram matrices of the Rayleigh-Ritz projection and of the
// Gram-Schmidt reorthogonalisation), and Out = alpha A S + beta Out for a tall-skinny A
// and a small S (Ritz vectors, projections).  Both read A once from HBM and are bound by
// it; both run on v_mfma_f64_16x16x4_f64 (accumulator r of lane L holds
// D[(L >> 4) + 4 r][L & 15]; A operand X[i][k] and B operand Y[k][j] in lane (i or j) + 16 k).
//
// Gram products: the N rows are split into G <= 256 ranges of at least 128 rows.  A
// workgroup owns one (64 rows of C, row range) pair and all c <= 128 columns of C: per
// 32-row slab it stages the slab of its 64 columns of A and of all columns of B in LDS
// (loads coalesced along the rows, the next slab in registers while the current one is
// used), and wave w accumulates the 16 rows 16 w.. of C against every 16-column tile.
// Each workgroup stores its accumulators as they sit in the registers (contiguous,
// coalesced); a second kernel adds the G partials of every slot in a fixed order and
// writes the entry of C the slot holds.
#include <algorithm>
#include <string>

#include "kl_internal.h"

namespace kl {
namespace {

typedef double doublex4 __attribute__((ext_vector_type(4)));

constexpr int kThreads = 256;
constexpr int kG = 256;          // maximum number of row ranges
constexpr int kSlab = 32;        // rows per LDS slab
constexpr int kGramRows = 64;    // rows of C per workgroup (4 waves x 16)
constexpr int kMaxCT = 8;        // 16-column tiles of C per workgroup (c <= 128)
constexpr int kRangeRows = 128;  // minimum rows per range

template <int CT>
__global__ __launch_bounds__(kThreads) void gram_mfma_kernel(
    const double *__restrict__ A, int64_t lda, int m, const double *__restrict__ B, int64_t ldb,
    int c, int64_t N, int64_t rows_per_range, double *__restrict__ part) {
    __shared__ double sA[kSlab][kGramRows + 2];
    __shared__ double sB[kSlab][16 * CT + 2];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int li = lane & 15, lk = lane >> 4;
    const int i0 = blockIdx.x * kGramRows;
    const int g = blockIdx.y;
    const int64_t n0 = int64_t(g) * rows_per_range;
    const int64_t n1 = min(N, n0 + rows_per_range);
    doublex4 acc[CT];
#pragma unroll
    for (int t = 0; t < CT; ++t) acc[t] = doublex4{0.0, 0.0, 0.0, 0.0};
    // slab loads: element e of a slab is (row r = e % 32, column e / 32): 32 consecutive
    // rows of one column per 32 threads
    constexpr int kPA = (kSlab * kGramRows) / kThreads;       // 8 elements of A per thread
    constexpr int kPB = (kSlab * 16 * CT + kThreads - 1) / kThreads;
    double pa[kPA], pb[kPB];
    auto load = [&](int64_t ns) {
#pragma unroll
        for (int q = 0; q < kPA; ++q) {
            const int e = threadIdx.x + q * kThreads;
            const int r = e % kSlab, col = i0 + e / kSlab;
            const int64_t n = ns + r;
            const bool ok = n < n1 && col < m;
            const double v = A[int64_t(ok ? col : 0) * lda + (ok ? n : 0)];
            pa[q] = ok ? v : 0.0;
        }
#pragma unroll
        for (int q = 0; q < kPB; ++q) {
            const int e = threadIdx.x + q * kThreads;
            const int r = e % kSlab, col = e / kSlab;
            const int64_t n = ns + r;
            const bool ok = n < n1 && col < c && e < kSlab * 16 * CT;
            const double v = B[int64_t(ok ? col : 0) * ldb + (ok ? n : 0)];
            pb[q] = ok ? v : 0.0;
        }
    };
    if (n0 < n1) load(n0);
    for (int64_t ns = n0; ns < n1; ns += kSlab) {
        __syncthreads();
#pragma unroll
        for (int q = 0; q < kPA; ++q) {
            const int e = threadIdx.x + q * kThreads;
            sA[e % kSlab][e / kSlab] = pa[q];
        }
#pragma unroll
        for (int q = 0; q < kPB; ++q) {
            const int e = threadIdx.x + q * kThreads;
            if (e < kSlab * 16 * CT) sB[e % kSlab][e / kSlab] = pb[q];
        }
        __syncthreads();
        if (ns + kSlab < n1) load(ns + kSlab);
        // C[16 w + i][16 t + j] += sum_n A[n][16 w + i] B[n][16 t + j]: A operand = A^T
        // (lane i + 16 k: sA[4 s + k][16 w + i]), B operand = B (lane j + 16 k)
#pragma unroll
        for (int st = 0; st < kSlab / 4; ++st) {
            const double a = sA[4 * st + lk][16 * w + li];
#pragma unroll
            for (int t = 0; t < CT; ++t) {
                const double b = sB[4 * st + lk][16 * t + li];
                acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[t], 0, 0, 0);
            }
        }
    }
    // slot (t, r, thread) of workgroup (row block, range g) at
    // part[((g nblk + blockIdx.x) 4 CT + 4 t + r) 256 + thread]
    double *dst = part + (int64_t(g) * gridDim.x + blockIdx.x) * (4 * CT * kThreads);
#pragma unroll
    for (int t = 0; t < CT; ++t)
#pragma unroll
        for (int r = 0; r < 4; ++r) dst[(4 * t + r) * kThreads + threadIdx.x] = acc[t][r];
}

// Sum of the G range partials of every accumulator slot.  A workgroup takes 64 slots;
// wave w adds the ranges [w G / 4, (w + 1) G / 4) of its lane's slot in range order (four
// loads in flight), and the four wave sums are added in wave order, so the result does
// not depend on scheduling.  The slot's entry of C (column-major, ld m) is stored.
template <int CT>
__global__ __launch_bounds__(kThreads) void gram_reduce_kernel(const double *__restrict__ part, int G, int nblk,
                                                               int m, int c, double *__restrict__ C) {
    constexpr int kSlots = 4 * CT * kThreads;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int64_t e = int64_t(blockIdx.x) * 64 + lane;     // slot over all row blocks
    const int64_t total = int64_t(nblk) * kSlots;
    __shared__ double red[4][64];
    double v = 0.0;
    if (e < total) {
        const int g0 = int(int64_t(G) * wv / 4), g1 = int(int64_t(G) * (wv + 1) / 4);
        const double *p = part + e;
        int g = g0;
        for (; g + 4 <= g1; g += 4) {
            const double a0 = p[int64_t(g) * total], a1 = p[int64_t(g + 1) * total];
            const double a2 = p[int64_t(g + 2) * total], a3 = p[int64_t(g + 3) * total];
            v += a0; v += a1; v += a2; v += a3;
        }
        for (; g < g1; ++g) v += p[int64_t(g) * total];
    }
    red[wv][lane] = v;
    __syncthreads();
    if (wv != 0 || e >= total) return;
    const int blk = int(e / kSlots), rem = int(e % kSlots);
    const int tr = rem / kThreads, th = rem % kThreads;
    const int t = tr >> 2, r = tr & 3;
    const int w = th >> 6, ln = th & 63;
    const int i = blk * kGramRows + 16 * w + (ln >> 4) + 4 * r, j = 16 * t + (ln & 15);
    if (i >= m || j >= c) return;
    C[int64_t(j) * m + i] = ((red[0][lane] + red[1][lane]) + red[2][lane]) + red[3][lane];
}

// Out (N x c) = alpha A (N x m) S (m x c) + beta Out, column-major, in the transposed form
// Out^T = S^T A^T: A operand S^T[j][k] (lane j + 16 k) from S staged in LDS, B operand
// A^T[k][i] = A[i + lda k] (lane i + 16 k: 16 consecutive rows of one column, coalesced)
// straight from memory, the next chunk in flight while the current one runs.  A workgroup
// owns 32 rows of Out; wave w takes rows 16 (w & 1).. and the 16-column tiles of group
// w >> 1 (at most 4 tiles per wave), so no partial tiles are added across waves.  S is
// staged 32 rows (k) at a time with loads coalesced along k.  beta = 0 does not read Out.
constexpr int kNNChunk = 32;     // k per LDS chunk of S
constexpr int kNNMaxTiles = 8;   // column tiles per workgroup (c <= 128)

template <int TPW, int NG>
__global__ __launch_bounds__(128 * NG) void gemm_nn_kernel(const double *__restrict__ A, int64_t lda, int m,
                                                           const double *__restrict__ S, int64_t lds, int c,
                                                           int64_t N, double alpha, double beta,
                                                           double *__restrict__ Out, int64_t ldo) {
    // NG tile groups of TPW tiles; 2 NG waves
    constexpr int kW = 2 * NG, kT = 64 * kW;
    constexpr int kC = 16 * TPW * NG;                     // columns covered
    __shared__ double sS[kNNChunk][kC + 2];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int li = lane & 15, lk = lane >> 4;
    const int64_t row0 = int64_t(blockIdx.x) * 32 + 16 * (w & 1);
    const int tg = w >> 1;
    const int64_t rowc = min(row0 + li, N - 1);            // clamped: rows past N are not stored
    doublex4 acc[TPW];
#pragma unroll
    for (int t = 0; t < TPW; ++t) acc[t] = doublex4{0.0, 0.0, 0.0, 0.0};
    constexpr int kPS = (kNNChunk * kC + kT - 1) / kT;    // S elements per thread per chunk
    double ps[kPS], pa[kNNChunk / 4];
    auto load = [&](int k0) {
#pragma unroll
        for (int q = 0; q < kPS; ++q) {
            const int e = threadIdx.x + q * kT;
            const int kk = e % kNNChunk, j = e / kNNChunk;
            const bool ok = e < kNNChunk * kC && k0 + kk < m && j < c;
            const double v = S[(ok ? k0 + kk : 0) + lds * (ok ? j : 0)];
            ps[q] = ok ? v : 0.0;
        }
#pragma unroll
        for (int st = 0; st < kNNChunk / 4; ++st) {
            const int k = k0 + 4 * st + lk;
            const bool ok = k < m;
            const double v = A[rowc + lda * (ok ? k : 0)];
            pa[st] = ok ? v : 0.0;
        }
    };
    if (m > 0) load(0);
    for (int k0 = 0; k0 < m; k0 += kNNChunk) {
        __syncthreads();
#pragma unroll
        for (int q = 0; q < kPS; ++q) {
            const int e = threadIdx.x + q * kT;
            if (e < kNNChunk * kC) sS[e % kNNChunk][e / kNNChunk] = ps[q];
        }
        __syncthreads();
        double a[kNNChunk / 4];
#pragma unroll
        for (int st = 0; st < kNNChunk / 4; ++st) a[st] = pa[st];
        if (k0 + kNNChunk < m) load(k0 + kNNChunk);
#pragma unroll
        for (int st = 0; st < kNNChunk / 4; ++st)
#pragma unroll
            for (int t = 0; t < TPW; ++t) {
                const double sv = sS[4 * st + lk][16 * (TPW * tg + t) + li];
                acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(sv, a[st], acc[t], 0, 0, 0);
            }
    }
    // acc[t][r] of lane L = Out[row0 + (L & 15)][16 (TPW tg + t) + (L >> 4) + 4 r]
    const int64_t row = row0 + li;
    if (row < N)
#pragma unroll
        for (int t = 0; t < TPW; ++t)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int j = 16 * (TPW * tg + t) + lk + 4 * r;
                if (j < c) {
                    double *o = Out + row + ldo * j;
                    *o = beta == 0.0 ? alpha * acc[t][r] : alpha * acc[t][r] + beta * *o;
                }
            }
}

// The same product for wide S (c > 32) and tall A (N >= kNN2MinRows): a wave owns 16 rows of
// Out and all TPW <= 8 column tiles, so that A is read once (the kernel above re-reads it in
// each group of column tiles), and a workgroup of 4 waves owns 64 rows.  S is staged through
// LDS in chunks of 64 k (the next chunk in registers while the current one is used) and the
// A operands of a chunk (16 steps, one double per lane each) are loaded one chunk ahead.
// The k steps of every tile run in the same order as in the kernel above (the same results).
constexpr int kNN2Chunk = 64;
constexpr int64_t kNN2MinRows = 16384;   // one 64-row workgroup per compute unit at least

template <int TPW>
__global__ __launch_bounds__(256) void gemm_nn_wide_kernel(const double *__restrict__ A, int64_t lda, int m,
                                                           const double *__restrict__ S, int64_t lds, int c,
                                                           int64_t N, double alpha, double beta,
                                                           double *__restrict__ Out, int64_t ldo) {
    constexpr int kC = 16 * TPW;
    __shared__ double sS[kNN2Chunk][kC + 1];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int li = lane & 15, lk = lane >> 4;
    const int64_t row0 = int64_t(blockIdx.x) * 64 + 16 * w;
    const int64_t rowc = min(row0 + li, N - 1);            // clamped: rows past N are not stored
    doublex4 acc[TPW];
#pragma unroll
    for (int t = 0; t < TPW; ++t) acc[t] = doublex4{0.0, 0.0, 0.0, 0.0};
    constexpr int kSteps = kNN2Chunk / 4;
    constexpr int kPS = (kNN2Chunk * kC) / 256;              // S elements per thread per chunk
    double ps[kPS], pa[kSteps];
    // loads clamped into S and A (m >= 1 here); the values past m or c are zeroed in use
    auto load = [&](int k0) __attribute__((always_inline)) {
#pragma unroll
        for (int q = 0; q < kPS; ++q) {
            const int e = threadIdx.x + q * 256;
            const int kk = e % kNN2Chunk, j = e / kNN2Chunk;
            ps[q] = S[min(k0 + kk, m - 1) + lds * min(j, c - 1)];
        }
#pragma unroll
        for (int st = 0; st < kSteps; ++st) pa[st] = A[rowc + lda * min(k0 + 4 * st + lk, m - 1)];
    };
    if (m > 0) load(0);
    for (int k0 = 0; k0 < m; k0 += kNN2Chunk) {
        __syncthreads();
#pragma unroll
        for (int q = 0; q < kPS; ++q) {
            const int e = threadIdx.x + q * 256;
            const int kk = e % kNN2Chunk, j = e / kNN2Chunk;
            sS[kk][j] = (k0 + kk < m && j < c) ? ps[q] : 0.0;
        }
        __syncthreads();
        double a[kSteps];
#pragma unroll
        for (int st = 0; st < kSteps; ++st) a[st] = (k0 + 4 * st + lk < m) ? pa[st] : 0.0;
        if (k0 + kNN2Chunk < m) load(k0 + kNN2Chunk);
        const int nst = min(kSteps, (m - k0 + 3) / 4);
#pragma unroll
        for (int st = 0; st < kSteps; ++st)
            if (st < nst)
#pragma unroll
                for (int t = 0; t < TPW; ++t)
                    acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(sS[4 * st + lk][16 * t + li], a[st], acc[t], 0, 0, 0);
    }
    // acc[t][r] of lane L = Out[row0 + (L & 15)][16 t + (L >> 4) + 4 r]
    const int64_t row = row0 + li;
    if (row < N)
#pragma unroll
        for (int t = 0; t < TPW; ++t)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int j = 16 * t + lk + 4 * r;
                if (j < c) {
                    double *o = Out + row + ldo * j;
                    *o = beta == 0.0 ? alpha * acc[t][r] : alpha * acc[t][r] + beta * *o;
                }
            }
}

template <int TPW>
void launch_gemm_nn_wide_t(const double *A, int64_t lda, int m, const double *S, int64_t lds, int c, int64_t N,
                           double alpha, double beta, double *Out, int64_t ldo, hipStream_t s) {
    hipLaunchKernelGGL((gemm_nn_wide_kernel<TPW>), dim3(unsigned((N + 63) / 64)), dim3(256), 0, s, A, lda, m, S, lds,
                       c, N, alpha, beta, Out, ldo);
}

template <int TPW, int NG>
void launch_gemm_nn_t(const double *A, int64_t lda, int m, const double *S, int64_t lds, int c, int64_t N,
                      double alpha, double beta, double *Out, int64_t ldo, hipStream_t s) {
    const dim3 grid(unsigned((N + 31) / 32));
    hipLaunchKernelGGL((gemm_nn_kernel<TPW, NG>), grid, dim3(128 * NG), 0, s, A, lda, m, S, lds, c, N, alpha,
                       beta, Out, ldo);
}

// R[:, j] = AX[:, j] - theta_j X[:, j] (if R) and the partial sums of r^2 over the row
// chunk g (blockIdx.y): part[g kk + j].  One workgroup per (column, row chunk).
__global__ __launch_bounds__(kThreads) void residual_partial_kernel(
    const double *__restrict__ X, const double *__restrict__ AX, const double *__restrict__ theta, int64_t N,
    int64_t ld, int64_t rows_per_chunk, int kk, double *__restrict__ R, double *__restrict__ part) {
    const int j = blockIdx.x, g = blockIdx.y;
    const double t = theta[j];
    const int64_t r0 = int64_t(g) * rows_per_chunk, r1 = min(N, r0 + rows_per_chunk);
    double s = 0.0;
    for (int64_t i = r0 + threadIdx.x; i < r1; i += kThreads) {
        const double r = AX[i + ld * j] - t * X[i + ld * j];
        if (R) R[i + ld * j] = r;
        s = fma(r, r, s);
    }
    __shared__ double red[kThreads / 64];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) part[int64_t(g) * kk + j] = red[0] + red[1] + red[2] + red[3];
}

// norms[j] = sqrt(sum_g part[g kk + j]) in chunk order.
__global__ __launch_bounds__(kThreads) void residual_norm_kernel(const double *__restrict__ part, int G, int kk,
                                                                 double *__restrict__ norms) {
    const int j = blockIdx.x * kThreads + threadIdx.x;
    if (j >= kk) return;
    double v = 0.0;
    for (int g = 0; g < G; ++g) v += part[int64_t(g) * kk + j];
    norms[j] = sqrt(v);
}

}  // namespace

int gram_splits(int64_t N, int m, int c, int n_cu) {
    (void)m; (void)c; (void)n_cu;
    int64_t g = (N + kRangeRows - 1) / kRangeRows;       // at least 128 rows per range
    if (g > kG) g = kG;
    if (g < 1) g = 1;
    return int(g);
}

int64_t gram_part_elems(int64_t N, int m, int c) {
    const int64_t nblk = (m + kGramRows - 1) / kGramRows;
    const int64_t tiles = std::min<int64_t>(kMaxCT, (c + 15) / 16);
    return int64_t(gram_splits(N, m, c, 0)) * nblk * 4 * tiles * kThreads;
}

// C (m x c, column-major, ld m) = A^T B with A: N x m (ld lda), B: N x c (ld ldb), c <= 128
// per launch (wider products are done in column blocks of 128).
// `part` needs gram_part_elems(N, m, c) doubles.
void launch_gram(const double *A, int64_t lda, int m, const double *B, int64_t ldb, int c,
                 int64_t N, double *part, double *C, int n_cu, hipStream_t s) {
    if (m < 1 || c < 1) return;
    const int G0 = gram_splits(N, m, c, n_cu);
    int64_t rows = (N + G0 - 1) / G0;
    rows = (rows + kSlab - 1) / kSlab * kSlab;
    const int G = int(std::max<int64_t>(1, (N + rows - 1) / rows));
    for (int j0 = 0; j0 < c; j0 += 16 * kMaxCT) {
        const int cb = std::min(16 * kMaxCT, c - j0);
        const int nblk = (m + kGramRows - 1) / kGramRows;
        const dim3 grid{unsigned(nblk), unsigned(G), 1u};
        const double *Bj = B + int64_t(j0) * ldb;
        double *Cj = C + int64_t(j0) * m;
#define KL_GRAM(CT)                                                                                        \
    do {                                                                                                   \
        hipLaunchKernelGGL((gram_mfma_kernel<CT>), grid, dim3(kThreads), 0, s, A, lda, m, Bj, ldb, cb, N,     \
                           rows, part);                                                                    \
        const int64_t slots = int64_t(nblk) * 4 * CT * kThreads;                                           \
        hipLaunchKernelGGL((gram_reduce_kernel<CT>), dim3(unsigned((slots + 63) / 64)),                      \
                           dim3(kThreads), 0, s, part, G, nblk, m, cb, Cj);                                \
    } while (0)
        switch ((cb + 15) / 16) {
        case 1: KL_GRAM(1); break;
        case 2: KL_GRAM(2); break;
        case 3: KL_GRAM(3); break;
        case 4: KL_GRAM(4); break;
        case 5: KL_GRAM(5); break;
        case 6: KL_GRAM(6); break;
        case 7: KL_GRAM(7); break;
        default: KL_GRAM(8); break;
        }
#undef KL_GRAM
    }
}

void launch_gemm_nn(const double *A, int64_t lda, int m, const double *S, int64_t lds, int c, int64_t N,
                    double alpha, double beta, double *Out, int64_t ldo, hipStream_t s) {
    if (N < 1 || c < 1) return;
    const int mm = std::max(m, 0);       // m = 0: empty contraction, Out = beta Out
    for (int j0 = 0; j0 < c; j0 += 16 * kNNMaxTiles) {
        const int cb = std::min(16 * kNNMaxTiles, c - j0);
        const double *Sj = S + int64_t(j0) * lds;
        double *Oj = Out + int64_t(j0) * ldo;
        if (cb > 32 && N >= kNN2MinRows) {
            switch ((cb + 15) / 16) {
            case 3: launch_gemm_nn_wide_t<3>(A, lda, mm, Sj, lds, cb, N, alpha, beta, Oj, ldo, s); break;
            case 4: launch_gemm_nn_wide_t<4>(A, lda, mm, Sj, lds, cb, N, alpha, beta, Oj, ldo, s); break;
            case 5: launch_gemm_nn_wide_t<5>(A, lda, mm, Sj, lds, cb, N, alpha, beta, Oj, ldo, s); break;
            case 6: launch_gemm_nn_wide_t<6>(A, lda, mm, Sj, lds, cb, N, alpha, beta, Oj, ldo, s); break;
            case 7: launch_gemm_nn_wide_t<7>(A, lda, mm, Sj, lds, cb, N, alpha, beta, Oj, ldo, s); break;
            default: launch_gemm_nn_wide_t<8>(A, lda, mm, Sj, lds, cb, N, alpha, beta, Oj, ldo, s); break;
            }
            continue;
        }
        switch ((cb + 15) / 16) {
        case 1: launch_gemm_nn_t<1, 1>(A, lda, mm, Sj, lds, cb, N, alpha, beta, Oj, ldo, s); break;
        case 2: launch_gemm_nn_t<1, 2>(A, lda, mm, Sj, lds, cb, N, alpha, beta, Oj, ldo, s); break;
        case 3: launch_gemm_nn_t<1, 3>(A, lda, mm, Sj, lds, cb, N, alpha, beta, Oj, ldo, s); break;
        case 4: launch_gemm_nn_t<2, 2>(A, lda, mm, Sj, lds, cb, N, alpha, beta, Oj, ldo, s); break;
        case 5:
        case 6: launch_gemm_nn_t<2, 3>(A, lda, mm, Sj, lds, cb, N, alpha, beta, Oj, ldo, s); break;
        default: launch_gemm_nn_t<2, 4>(A, lda, mm, Sj, lds, cb, N, alpha, beta, Oj, ldo, s); break;
        }
    }
}

int residual_chunks(int64_t N) {
    return int(std::max<int64_t>(1, std::min<int64_t>(64, (N + 2047) / 2048)));
}

void launch_residual(const double *X, const double *AX, const double *theta, int64_t N, int64_t ld, int kk,
                     double *R, double *part, double *norms, hipStream_t s) {
    if (kk < 1) return;
    const int G = residual_chunks(N);
    const int64_t rows = (N + G - 1) / G;
    hipLaunchKernelGGL(residual_partial_kernel, dim3(unsigned(kk), unsigned(G)), dim3(kThreads), 0, s, X, AX, theta,
                       N, ld, rows, kk, R, part);
    hipLaunchKernelGGL(residual_norm_kernel, dim3(unsigned((kk + kThreads - 1) / kThreads)), dim3(kThreads), 0, s,
                       part, G, kk, norms);
}

}  // namespace kl

// Tall-skinny product on the device through the C ABI (see include/kl.h).
extern "C" kl_status kl_gemm_tall(int64_t N, int32_t m, int32_t c, const double *A, int64_t lda, const double *S,
                                  int64_t lds, double alpha, double beta, double *Out, int64_t ldo, void *stream) {
    using namespace kl;
    if (N < 0 || m < 0 || c < 0) { set_error("kl_gemm_tall: negative size"); return KL_EINVAL; }
    if (N == 0 || c == 0) return KL_OK;
    if (N > (int64_t(1) << 36)) { set_error("kl_gemm_tall: more than 2^36 rows"); return KL_EINVAL; }
    if (!Out || ldo < N || (m > 0 && (!A || !S || lda < N || lds < m))) {
        set_error("kl_gemm_tall: NULL pointer or leading dimension too small");
        return KL_EINVAL;
    }
    (void)hipGetLastError();
    launch_gemm_nn(A, lda, m, S, lds, c, N, alpha, beta, Out, ldo, static_cast<hipStream_t>(stream));
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) { set_error(std::string("kl_gemm_tall: ") + hipGetErrorString(e)); return KL_EHIP; }
    return KL_OK;
}

// Gram product on the device through the C ABI (see include/kl.h).
extern "C" int64_t kl_gram_tall_workspace(int64_t N, int32_t m, int32_t c) {
    if (N < 1 || m < 1 || c < 1) return 0;
    return kl::gram_part_elems(N, m, c);
}

extern "C" kl_status kl_gram_tall(int64_t N, int32_t m, int32_t c, const double *A, int64_t lda, const double *B,
                                  int64_t ldb, double *C, double *work, int64_t work_elems, void *stream) {
    using namespace kl;
    if (N < 0 || m < 0 || c < 0) { set_error("kl_gram_tall: negative size"); return KL_EINVAL; }
    if (m == 0 || c == 0) return KL_OK;
    if (!C) { set_error("kl_gram_tall: NULL C"); return KL_EINVAL; }
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (N == 0) {                                        // empty sums: C = 0
        if (hipMemsetAsync(C, 0, size_t(m) * size_t(c) * sizeof(double), s) != hipSuccess) {
            set_error("kl_gram_tall: clearing C failed");
            return KL_EHIP;
        }
        return KL_OK;
    }
    if (N > (int64_t(1) << 36)) { set_error("kl_gram_tall: more than 2^36 rows"); return KL_EINVAL; }
    if (!A || !B || lda < N || ldb < N) {
        set_error("kl_gram_tall: NULL pointer or leading dimension too small");
        return KL_EINVAL;
    }
    if (!work || work_elems < gram_part_elems(N, m, c)) {
        set_error("kl_gram_tall: workspace smaller than kl_gram_tall_workspace(N, m, c)");
        return KL_EINVAL;
    }
    int dev = 0, ncu = 256;
    (void)hipGetDevice(&dev);
    (void)hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
    (void)hipGetLastError();
    launch_gram(A, lda, m, B, ldb, c, N, work, C, ncu, s);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) { set_error(std::string("kl_gram_tall: ") + hipGetErrorString(e)); return KL_EHIP; }
    return KL_OK;
}
