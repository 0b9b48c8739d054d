// FP64 block kernels of the eigensolver: C = A^T B for tall-skinny A (N x m) and
// B (N x c), N >> m, c (the Gram matrices of the Rayleigh-Ritz projection and of the
// Gram-Schmidt reorthogonalisation).
//
// The N rows are split into G ranges.  A workgroup owns one (64 x 64 tile of C, row
// range) pair: it stages 32-row slabs of the 64 columns of A and of B in LDS (loads
// coalesced along the rows) and accumulates 16 entries per thread with FP64 FMAs.  The
// partials are stored output-major, part[e][g], so that the reduction is one wave per
// output entry: 64 coalesced loads and a cross-lane sum, in a fixed order.
#include "kl_internal.h"

namespace kl {
namespace {

constexpr int kT = 64;         // C tile edge
constexpr int kSlab = 32;      // rows per LDS slab
constexpr int kThreads = 256;  // 16 x 16 threads, 4 x 4 entries each
constexpr int kG = 64;         // maximum number of row ranges

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
    for (int64_t ns = n0; ns < n1; ns += kSlab) {
#pragma unroll
        for (int q = 0; q < (kSlab * kT) / kThreads; ++q) {
            const int e = threadIdx.x + q * kThreads;
            const int r = e % kSlab, col = e / kSlab;
            const int64_t n = ns + r;
            sA[r][col] = (n < n1 && i0 + col < m) ? A[(i0 + col) * lda + n] : 0.0;
            sB[r][col] = (n < n1 && j0 + col < c) ? B[(j0 + col) * ldb + n] : 0.0;
        }
        __syncthreads();
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
        __syncthreads();
    }
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int i = i0 + ti + 16 * u, j = j0 + tj + 16 * v;
            if (i < m && j < c) part[(int64_t(j) * m + i) * kG + g] = acc[u][v];
        }
}

// One wave per entry of C: sums part[e][0..G-1] across lanes.
__global__ __launch_bounds__(kThreads) void gram_reduce_kernel(const double *__restrict__ part,
                                                               int G, int64_t mc,
                                                               double *__restrict__ C) {
    const int lane = threadIdx.x & 63;
    const int64_t e = int64_t(blockIdx.x) * (kThreads / 64) + (threadIdx.x >> 6);
    if (e >= mc) return;
    double v = lane < G ? part[e * kG + lane] : 0.0;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    if (lane == 0) C[e] = v;
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
// `part` needs 64 * m * c doubles.
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

}  // namespace kl
