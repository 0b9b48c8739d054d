// Kernels of the warm-start network: FP32 GEMM on the matrix cores with fused
// bias / tanh / tanh-derivative epilogues, the sign-invariant loss, column sums for the
// bias gradients, Adam, and a row gather for minibatches.
//
// The network maps covariance parameters to a block of leading eigenvector coefficients
// (an addition to the method: the paper starts its Lanczos iteration from a generic
// vector).  All matrices are row-major FP32.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "mlp_internal.h"

namespace kl {
namespace mlp {

namespace {

typedef float floatx16 __attribute__((ext_vector_type(16)));

constexpr int kTM = 64, kTN = 64, kTK = 32, kThreads = 256;
constexpr int kPadL = 4;   // LDS row padding (floats)

__device__ __forceinline__ float epilogue(const GemmArgs &g, int row, int col, float v) {
    switch (g.epi) {
    case EPI_BIAS: return v + g.bias[col];
    case EPI_BIAS_TANH: return tanhf(v + g.bias[col]);
    case EPI_DTANH: {
        const float h = g.aux[int64_t(row) * g.ldaux + col];
        return v * (1.0f - h * h);
    }
    default: return v;
    }
}

// C (M x N) = op(A) (M x K) * op(B) (K x N), one 64 x 64 tile per workgroup, four waves
// of 32 x 32 on v_mfma_f32_32x32x2f32.  blockIdx.z selects a K range; with more than one
// range the raw sums go to part[z][M][N] and splitk_reduce applies the epilogue.
// Operand tiles are staged k-major in LDS (sA[k][i], sB[k][j]) from coalesced global
// loads along whichever index is contiguous; the next tile is prefetched into registers
// while the current one is consumed.
template <bool TA, bool TB>
__global__ __launch_bounds__(kThreads) void gemm_f32_kernel(GemmArgs g) {
    __shared__ float sA[kTK][kTM + kPadL];
    __shared__ float sB[kTK][kTN + kPadL];
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    const int i0 = blockIdx.y * kTM, j0 = blockIdx.x * kTN;
    const int kb = blockIdx.z * g.kchunk;
    const int ke = min(g.K, kb + g.kchunk);
    const int wi = (w >> 1) * 32, wj = (w & 1) * 32;
    floatx16 acc;
    for (int r = 0; r < 16; ++r) acc[r] = 0.0f;
    float ra[8], rb[8];
    auto a_index = [&](int e, int &ii, int &kk) {
        if (TA) { ii = e & (kTM - 1); kk = e >> 6; } else { kk = e & (kTK - 1); ii = e >> 5; }
    };
    auto b_index = [&](int e, int &jj, int &kk) {
        if (TB) { kk = e & (kTK - 1); jj = e >> 5; } else { jj = e & (kTN - 1); kk = e >> 6; }
    };
    auto load = [&](int k0) {
#pragma unroll
        for (int r = 0; r < 8; ++r) {
            const int e = r * kThreads + t;
            int ii, jj, ka, kbb;
            a_index(e, ii, ka);
            b_index(e, jj, kbb);
            const int gi = i0 + ii, gka = k0 + ka;
            const int gj = j0 + jj, gkb = k0 + kbb;
            ra[r] = (gi < g.M && gka < ke)
                        ? (TA ? g.A[int64_t(gka) * g.lda + gi] : g.A[int64_t(gi) * g.lda + gka])
                        : 0.0f;
            rb[r] = (gj < g.N && gkb < ke)
                        ? (TB ? g.B[int64_t(gj) * g.ldb + gkb] : g.B[int64_t(gkb) * g.ldb + gj])
                        : 0.0f;
        }
    };
    if (kb < ke) load(kb);
    for (int k0 = kb; k0 < ke; k0 += kTK) {
        __syncthreads();
#pragma unroll
        for (int r = 0; r < 8; ++r) {
            const int e = r * kThreads + t;
            int ii, jj, ka, kbb;
            a_index(e, ii, ka);
            b_index(e, jj, kbb);
            sA[ka][ii] = ra[r];
            sB[kbb][jj] = rb[r];
        }
        __syncthreads();
        if (k0 + kTK < ke) load(k0 + kTK);
#pragma unroll
        for (int kk = 0; kk < kTK; kk += 2) {
            const float a = sA[kk + (lane >> 5)][wi + (lane & 31)];
            const float b = sB[kk + (lane >> 5)][wj + (lane & 31)];
            acc = __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, acc, 0, 0, 0);
        }
    }
    // accumulator r of lane L: row (r & 3) + 4 (L >> 5) + 8 (r >> 2), column L & 31
    const int col = j0 + wj + (lane & 31);
    if (col >= g.N) return;
#pragma unroll
    for (int r = 0; r < 16; ++r) {
        const int row = i0 + wi + (r & 3) + 4 * (lane >> 5) + 8 * (r >> 2);
        if (row >= g.M) continue;
        if (gridDim.z > 1)
            g.part[(int64_t(blockIdx.z) * g.M + row) * g.N + col] = acc[r];
        else
            g.C[int64_t(row) * g.ldc + col] = epilogue(g, row, col, acc[r]);
    }
}

// Sum of the K-range partials in a fixed order, then the epilogue.
__global__ __launch_bounds__(kThreads) void splitk_reduce_kernel(GemmArgs g, int splits) {
    const int64_t total = int64_t(g.M) * g.N;
    for (int64_t e = int64_t(blockIdx.x) * kThreads + threadIdx.x; e < total;
         e += int64_t(gridDim.x) * kThreads) {
        float v = 0.0f;
        for (int s = 0; s < splits; ++s) v += g.part[int64_t(s) * total + e];
        const int row = int(e / g.N), col = int(e % g.N);
        g.C[int64_t(row) * g.ldc + col] = epilogue(g, row, col, v);
    }
}

// Sign-invariant loss, one workgroup per (group, sample): with y_g and t_g the group's
// output and target, s = +1 if <y_g, t_g> >= 0 else -1 (dot accumulated in FP64);
// dy_g = (y_g - s t_g) * inv_b and loss_part = 0.5 ||y_g - s t_g||^2 (FP64).
// signed_ == 0 keeps s = +1 (plain squared error).
__global__ __launch_bounds__(kThreads) void loss_kernel(const float *__restrict__ y, int64_t ldy,
                                                        const float *__restrict__ tgt, int64_t ldt,
                                                        const int *__restrict__ rows, int group,
                                                        int signed_, float inv_b, float *__restrict__ dy,
                                                        int64_t lddy, double *__restrict__ loss_part) {
    const int gi = blockIdx.x, s = blockIdx.y;
    const float *yr = y + int64_t(s) * ldy + int64_t(gi) * group;
    const int trow = rows ? rows[s] : s;
    const float *tr = tgt + int64_t(trow) * ldt + int64_t(gi) * group;
    __shared__ double red[kThreads];
    __shared__ double sgn_sh;
    double dot = 0.0;
    if (signed_) {
        for (int i = threadIdx.x; i < group; i += kThreads) dot += double(yr[i]) * double(tr[i]);
        red[threadIdx.x] = dot;
        __syncthreads();
        for (int w = kThreads / 2; w > 0; w >>= 1) {
            if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
            __syncthreads();
        }
        if (threadIdx.x == 0) sgn_sh = red[0] >= 0.0 ? 1.0 : -1.0;
        __syncthreads();
    }
    const float sg = signed_ ? float(sgn_sh) : 1.0f;
    float *dr = dy + int64_t(s) * lddy + int64_t(gi) * group;
    double l2 = 0.0;
    for (int i = threadIdx.x; i < group; i += kThreads) {
        const float e = yr[i] - sg * tr[i];
        dr[i] = e * inv_b;
        l2 += double(e) * double(e);
    }
    __syncthreads();
    red[threadIdx.x] = l2;
    __syncthreads();
    for (int w = kThreads / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) loss_part[int64_t(s) * gridDim.x + gi] = 0.5 * red[0];
}

// Sum of a double over the workgroup in a fixed order (lanes by butterfly within each
// wave, then the waves in order); every thread gets the result.  `red` holds kThreads / 64.
__device__ __forceinline__ double block_sum(double v, double *red) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    double t = 0.0;
#pragma unroll
    for (int w = 0; w < kThreads / 64; ++w) t += red[w];
    return t;
}

// Subspace term of the loss, one workgroup per (group, sample), after loss_kernel on the
// same stream: with y the group's output and t_j the sample's ng target groups,
// c_j = <t_j, y>, n_j = <t_j, t_j> (FP64), r = y - sum_j t_j c_j / n_j (the part of y
// outside the span of orthogonal targets); dy += w inv_b r and loss_part += 0.5 w ||r||^2.
__global__ __launch_bounds__(kThreads) void subspace_kernel(const float *__restrict__ y, int64_t ldy,
                                                            const float *__restrict__ tgt, int64_t ldt,
                                                            const int *__restrict__ rows, int group, int ng, float w,
                                                            float inv_b, float *__restrict__ dy, int64_t lddy,
                                                            double *__restrict__ loss_part) {
    const int gi = blockIdx.x, s = blockIdx.y;
    const float *yr = y + int64_t(s) * ldy + int64_t(gi) * group;
    const int trow = rows ? rows[s] : s;
    const float *tr = tgt + int64_t(trow) * ldt;
    __shared__ double red[kThreads / 64];
    __shared__ double coef[kMaxSubGroups];
    for (int j0 = 0; j0 < ng; j0 += 8) {
        double c[8], n[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) c[q] = n[q] = 0.0;
        for (int i = threadIdx.x; i < group; i += kThreads) {
            const double yv = yr[i];
#pragma unroll
            for (int q = 0; q < 8; ++q)
                if (j0 + q < ng) {
                    const double t = tr[int64_t(j0 + q) * group + i];
                    c[q] += t * yv;
                    n[q] += t * t;
                }
        }
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            if (j0 + q >= ng) break;
            const double cs = block_sum(c[q], red);
            const double ns = block_sum(n[q], red);
            if (threadIdx.x == 0) coef[j0 + q] = ns > 0.0 ? cs / ns : 0.0;
        }
    }
    __syncthreads();
    float *dr = dy + int64_t(s) * lddy + int64_t(gi) * group;
    const float sc = w * inv_b;
    double l2 = 0.0;
    for (int i = threadIdx.x; i < group; i += kThreads) {
        double r = yr[i];
        for (int j = 0; j < ng; ++j) r -= double(tr[int64_t(j) * group + i]) * coef[j];
        dr[i] += sc * float(r);
        l2 += r * r;
    }
    const double tot = block_sum(l2, red);
    if (threadIdx.x == 0) loss_part[int64_t(s) * gridDim.x + gi] += 0.5 * double(w) * tot;
}

// db[j] = sum_i D[i][j] over M rows (one thread per column, fixed row order).
__global__ __launch_bounds__(kThreads) void colsum_kernel(const float *__restrict__ D, int64_t ldd, int M,
                                                          int N, float *__restrict__ out) {
    const int j = blockIdx.x * kThreads + threadIdx.x;
    if (j >= N) return;
    float s = 0.0f;
    for (int i = 0; i < M; ++i) s += D[int64_t(i) * ldd + j];
    out[j] = s;
}

// Adam with bias correction: m = b1 m + (1 - b1) g, v = b2 v + (1 - b2) g^2,
// p -= lr (m / c1) / (sqrt(v / c2) + eps), c1 = 1 - b1^t, c2 = 1 - b2^t.
__global__ __launch_bounds__(kThreads) void adam_kernel(float *__restrict__ p, const float *__restrict__ g,
                                                        float *__restrict__ m, float *__restrict__ v,
                                                        int64_t n, AdamArgs a) {
    for (int64_t i = int64_t(blockIdx.x) * kThreads + threadIdx.x; i < n; i += int64_t(gridDim.x) * kThreads) {
        const float gi = g[i];
        const float mi = a.b1 * m[i] + (1.0f - a.b1) * gi;
        const float vi = a.b2 * v[i] + (1.0f - a.b2) * gi * gi;
        m[i] = mi;
        v[i] = vi;
        p[i] -= a.lr * (mi / a.c1) / (sqrtf(vi / a.c2) + a.eps);
    }
}

// dst[s][c] = src[rows[s]][c]
__global__ __launch_bounds__(kThreads) void gather_kernel(const float *__restrict__ src, int64_t lds,
                                                          const int *__restrict__ rows, int nrows, int ncols,
                                                          float *__restrict__ dst) {
    const int64_t total = int64_t(nrows) * ncols;
    for (int64_t e = int64_t(blockIdx.x) * kThreads + threadIdx.x; e < total;
         e += int64_t(gridDim.x) * kThreads) {
        const int s = int(e / ncols), c = int(e % ncols);
        dst[e] = src[int64_t(rows[s]) * lds + c];
    }
}

int grid_for(int64_t n, int cap) { return int(std::max<int64_t>(1, std::min<int64_t>(cap, (n + kThreads - 1) / kThreads))); }

}  // namespace

int gemm_splits(int M, int N, int K, int n_cu, int64_t part_cap, int *kchunk) {
    const int64_t tiles = int64_t((M + kTM - 1) / kTM) * ((N + kTN - 1) / kTN);
    const int ksteps = std::max(1, (K + kTK - 1) / kTK);
    int splits = 1;
    const int64_t want = 2 * int64_t(n_cu);
    if (tiles < want) splits = int(std::min<int64_t>(ksteps, (want + tiles - 1) / tiles));
    while (splits > 1 && int64_t(splits) * M * N > part_cap) --splits;
    const int steps_per = (ksteps + splits - 1) / splits;
    *kchunk = steps_per * kTK;
    return (ksteps + steps_per - 1) / steps_per;
}

void launch_gemm(bool ta, bool tb, GemmArgs g, int splits, hipStream_t s) {
    const dim3 grid((g.N + kTN - 1) / kTN, (g.M + kTM - 1) / kTM, splits);
    if (ta && tb) hipLaunchKernelGGL((gemm_f32_kernel<true, true>), grid, dim3(kThreads), 0, s, g);
    else if (ta) hipLaunchKernelGGL((gemm_f32_kernel<true, false>), grid, dim3(kThreads), 0, s, g);
    else if (tb) hipLaunchKernelGGL((gemm_f32_kernel<false, true>), grid, dim3(kThreads), 0, s, g);
    else hipLaunchKernelGGL((gemm_f32_kernel<false, false>), grid, dim3(kThreads), 0, s, g);
    if (splits > 1)
        hipLaunchKernelGGL(splitk_reduce_kernel, dim3(grid_for(int64_t(g.M) * g.N, 2048)), dim3(kThreads), 0, s,
                           g, splits);
}

void launch_loss(const float *y, int64_t ldy, const float *t, int64_t ldt, const int *rows, int batch,
                 int n_out, int group, int signed_, float *dy, int64_t lddy, double *loss_part,
                 hipStream_t s) {
    const int ng = n_out / group;
    hipLaunchKernelGGL(loss_kernel, dim3(ng, batch), dim3(kThreads), 0, s, y, ldy, t, ldt, rows, group, signed_,
                       1.0f / float(batch), dy, lddy, loss_part);
}

void launch_subspace(const float *y, int64_t ldy, const float *t, int64_t ldt, const int *rows, int batch,
                     int n_out, int group, float weight, float *dy, int64_t lddy, double *loss_part, hipStream_t s) {
    const int ng = n_out / group;
    hipLaunchKernelGGL(subspace_kernel, dim3(ng, batch), dim3(kThreads), 0, s, y, ldy, t, ldt, rows, group, ng,
                       weight, 1.0f / float(batch), dy, lddy, loss_part);
}

void launch_colsum(const float *D, int64_t ldd, int M, int N, float *out, hipStream_t s) {
    hipLaunchKernelGGL(colsum_kernel, dim3((N + kThreads - 1) / kThreads), dim3(kThreads), 0, s, D, ldd, M, N, out);
}

void launch_adam(float *p, const float *g, float *m, float *v, int64_t n, const AdamArgs &a, hipStream_t s) {
    hipLaunchKernelGGL(adam_kernel, dim3(grid_for(n, 4096)), dim3(kThreads), 0, s, p, g, m, v, n, a);
}

void launch_gather(const float *src, int64_t lds, const int *rows, int nrows, int ncols, float *dst,
                   hipStream_t s) {
    hipLaunchKernelGGL(gather_kernel, dim3(grid_for(int64_t(nrows) * ncols, 1024)), dim3(kThreads), 0, s, src,
                       lds, rows, nrows, ncols, dst);
}

}  // namespace mlp
}  // namespace kl
