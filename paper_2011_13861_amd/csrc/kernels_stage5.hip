// Stage 5 of Algorithm 1 on MFMA: Z'_k = sum_l Gamma(x_k, x_l) Y'_l.
// Y and the split partials Z are column-major blocks of kBW columns, ld = padded grid.
//
// Sec. 4.4.2: the dense Ntilde x Ntilde covariance matrix is never stored; its entries
// are evaluated on the fly and contracted with the block of vectors.  Here the
// contraction runs on the matrix cores: each lane evaluates the kernel entry that is
// its A-operand element of one MFMA (a Gamma tile), the B operand is a tile of the
// block of vectors staged in LDS, and the accumulators hold a tile of Z'.  Work is
// split over row tiles (grid.x) and, for small problems, over ranges of l (grid.y);
// the split partial sums are added by the backward prologue.
//
// Coordinates are pre-scaled on the host: by 1/ell for the FP64 kernels (Gamma =
// exp(-rho) or exp(-rho^2)) and by log2(e)/ell or sqrt(log2 e)/ell for the FP32 kernels,
// which then use the hardware base-2 exponential.  sigma^2 is applied after the split
// reduction.  Grids are padded with zero points and zero vectors, which add nothing.
#include "kl_internal.h"

namespace kl {
namespace {

typedef float floatx16 __attribute__((ext_vector_type(16)));
typedef double doublex4 __attribute__((ext_vector_type(4)));

template <int KIND, int D>
__device__ __forceinline__ float gamma_f32(const float *xk, const float *xl) {
    if constexpr (KIND == KL_COV_EXP) {
        float r2 = 0.f;
#pragma unroll
        for (int k = 0; k < D; ++k) { float t = xk[k] - xl[k]; r2 = fmaf(t, t, r2); }
        return __builtin_amdgcn_exp2f(-__builtin_amdgcn_sqrtf(r2));
    } else if constexpr (KIND == KL_COV_SQEXP) {
        float r2 = 0.f;
#pragma unroll
        for (int k = 0; k < D; ++k) { float t = xk[k] - xl[k]; r2 = fmaf(t, t, r2); }
        return __builtin_amdgcn_exp2f(-r2);
    } else if constexpr (KIND == KL_COV_EXP_L1) {
        float s = 0.f;
#pragma unroll
        for (int k = 0; k < D; ++k) s += fabsf(xk[k] - xl[k]);
        return __builtin_amdgcn_exp2f(-s);
    } else if constexpr (KIND == KL_COV_CONST) {
        return 1.f;
    } else {
        float s = 1.f;
#pragma unroll
        for (int k = 0; k < D; ++k) s = fmaf(xk[k], xl[k], s);
        return s;
    }
}

template <int KIND, int D>
__device__ __forceinline__ double gamma_f64(const double *xk, const double *xl) {
    if constexpr (KIND == KL_COV_EXP) {
        double r2 = 0.0;
#pragma unroll
        for (int k = 0; k < D; ++k) { double t = xk[k] - xl[k]; r2 = fma(t, t, r2); }
        return exp(-sqrt(r2));
    } else if constexpr (KIND == KL_COV_SQEXP) {
        double r2 = 0.0;
#pragma unroll
        for (int k = 0; k < D; ++k) { double t = xk[k] - xl[k]; r2 = fma(t, t, r2); }
        return exp(-r2);
    } else if constexpr (KIND == KL_COV_EXP_L1) {
        double s = 0.0;
#pragma unroll
        for (int k = 0; k < D; ++k) s += fabs(xk[k] - xl[k]);
        return exp(-s);
    } else if constexpr (KIND == KL_COV_CONST) {
        return 1.0;
    } else {
        double s = 1.0;
#pragma unroll
        for (int k = 0; k < D; ++k) s = fma(xk[k], xl[k], s);
        return s;
    }
}

constexpr int kWaves = 4;
constexpr int kThreads = 64 * kWaves;

// ---- FP32: v_mfma_f32_32x32x2_f32; A = Gamma[32 rows][2 l], B = Y[2 l][32 cols] -----
// Lane layout: A[i][k] and B[k][j] sit in lane (i or j) + 32 k; accumulator element r of
// lane L holds C[(r & 3) + 4 (L >> 5) + 8 (r >> 2)][L & 31].
constexpr int kTL32 = 64;   // l-points per LDS tile

template <int KIND, int D, int RB>
__global__ __launch_bounds__(kThreads) void stage5_f32_kernel(
    const float *__restrict__ X, const float *__restrict__ Y, float *__restrict__ Z,
    int64_t Ntpad, int64_t lchunk) {
    __shared__ float sX[D][kTL32];
    __shared__ float sY[kTL32][kBW + 1];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int i = lane & 31, kh = lane >> 5;
    const int64_t row0 = int64_t(blockIdx.x) * (kWaves * 32 * RB) + int64_t(wave) * 32 * RB;
    const int64_t l0 = int64_t(blockIdx.y) * lchunk;
    const int64_t l1 = min(l0 + lchunk, Ntpad);
    float xk[RB][D];
#pragma unroll
    for (int rb = 0; rb < RB; ++rb)
#pragma unroll
        for (int k = 0; k < D; ++k) xk[rb][k] = X[k * Ntpad + row0 + rb * 32 + i];
    floatx16 acc[RB];
#pragma unroll
    for (int rb = 0; rb < RB; ++rb)
#pragma unroll
        for (int r = 0; r < 16; ++r) acc[rb][r] = 0.f;

    for (int64_t lt = l0; lt < l1; lt += kTL32) {
        __syncthreads();
        // Y is column-major (ld Ntpad): coalesced along l, transposed into LDS
#pragma unroll
        for (int q = 0; q < (kTL32 * kBW) / kThreads; ++q) {
            const int e = threadIdx.x + q * kThreads;
            const int l = e % kTL32, j = e / kTL32;
            sY[l][j] = Y[int64_t(j) * Ntpad + lt + l];
        }
        if (threadIdx.x < D * kTL32) {
            const int k = threadIdx.x / kTL32, l = threadIdx.x % kTL32;
            sX[k][l] = X[k * Ntpad + lt + l];
        }
        __syncthreads();
#pragma unroll 8
        for (int ll = 0; ll < kTL32; ll += 2) {
            float xl[D];
#pragma unroll
            for (int k = 0; k < D; ++k) xl[k] = sX[k][ll + kh];
            const float b = sY[ll + kh][i];
#pragma unroll
            for (int rb = 0; rb < RB; ++rb) {
                const float g = gamma_f32<KIND, D>(xk[rb], xl);
                acc[rb] = __builtin_amdgcn_mfma_f32_32x32x2f32(g, b, acc[rb], 0, 0, 0);
            }
        }
    }
    // Z is column-major (ld Ntpad); accumulator registers 4m..4m+3 of a lane hold four
    // consecutive rows of one column, stored as one 16-byte vector
    float *Zs = Z + int64_t(blockIdx.y) * Ntpad * kBW + int64_t(i) * Ntpad;
#pragma unroll
    for (int rb = 0; rb < RB; ++rb)
#pragma unroll
        for (int m = 0; m < 4; ++m) {
            const int64_t row = row0 + rb * 32 + 4 * kh + 8 * m;
            float4 v = {acc[rb][4 * m], acc[rb][4 * m + 1], acc[rb][4 * m + 2], acc[rb][4 * m + 3]};
            *reinterpret_cast<float4 *>(Zs + row) = v;
        }
}

// ---- FP64: v_mfma_f64_16x16x4_f64; A = Gamma[16 rows][4 l], B = Y[4 l][16 cols] -----
// Lane layout: A[i][k] and B[k][j] sit in lane (i or j) + 16 k; accumulator element r of
// lane L holds C[(L >> 4) + 4 r][L & 15] (measured on gfx950; this differs from the
// FP32 16x16x4 layout).  Two MFMAs cover the 32 columns.
constexpr int kTL64 = 32;

template <int KIND, int D, int RB>
__global__ __launch_bounds__(kThreads) void stage5_f64_kernel(
    const double *__restrict__ X, const double *__restrict__ Y, double *__restrict__ Z,
    int64_t Ntpad, int64_t lchunk) {
    __shared__ double sX[D][kTL64];
    __shared__ double sY[kTL64][kBW + 1];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int i = lane & 15, kq = lane >> 4;
    const int64_t row0 = int64_t(blockIdx.x) * (kWaves * 16 * RB) + int64_t(wave) * 16 * RB;
    const int64_t l0 = int64_t(blockIdx.y) * lchunk;
    const int64_t l1 = min(l0 + lchunk, Ntpad);
    double xk[RB][D];
#pragma unroll
    for (int rb = 0; rb < RB; ++rb)
#pragma unroll
        for (int k = 0; k < D; ++k) xk[rb][k] = X[k * Ntpad + row0 + rb * 16 + i];
    doublex4 acc[RB][2];
#pragma unroll
    for (int rb = 0; rb < RB; ++rb)
#pragma unroll
        for (int r = 0; r < 4; ++r) { acc[rb][0][r] = 0.0; acc[rb][1][r] = 0.0; }

    for (int64_t lt = l0; lt < l1; lt += kTL64) {
        __syncthreads();
#pragma unroll
        for (int q = 0; q < (kTL64 * kBW) / kThreads; ++q) {
            const int e = threadIdx.x + q * kThreads;
            const int l = e % kTL64, j = e / kTL64;
            sY[l][j] = Y[int64_t(j) * Ntpad + lt + l];
        }
        if (threadIdx.x < D * kTL64) {
            const int k = threadIdx.x / kTL64, l = threadIdx.x % kTL64;
            sX[k][l] = X[k * Ntpad + lt + l];
        }
        __syncthreads();
#pragma unroll 2
        for (int ll = 0; ll < kTL64; ll += 4) {
            double xl[D];
#pragma unroll
            for (int k = 0; k < D; ++k) xl[k] = sX[k][ll + kq];
            const double b0 = sY[ll + kq][i];
            const double b1 = sY[ll + kq][16 + i];
#pragma unroll
            for (int rb = 0; rb < RB; ++rb) {
                const double g = gamma_f64<KIND, D>(xk[rb], xl);
                acc[rb][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(g, b0, acc[rb][0], 0, 0, 0);
                acc[rb][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(g, b1, acc[rb][1], 0, 0, 0);
            }
        }
    }
    // Z is column-major (ld Ntpad): for each register, lanes with the same column
    // write four consecutive rows
    double *Zs = Z + int64_t(blockIdx.y) * Ntpad * kBW;
#pragma unroll
    for (int rb = 0; rb < RB; ++rb)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int64_t row = row0 + rb * 16 + kq + 4 * r;
            Zs[int64_t(i) * Ntpad + row] = acc[rb][0][r];
            Zs[int64_t(16 + i) * Ntpad + row] = acc[rb][1][r];
        }
}


// ---- BF16: v_mfma_f32_32x32x16_bf16; A = Gamma[32 rows][16 l], B = Y[16 l][32 cols] ---
// Lane layout (measured on gfx950): A[i][k] in lane i + 32 (k / 8), element k % 8;
// B[k][j] in lane j + 32 (k / 8), element k % 8; accumulators as for the FP32 32x32x2.
// The kernel is evaluated in FP32 and rounded to BF16 (round to nearest even).  With
// X3 both operands are split into hi + lo BF16 parts and three products are
// accumulated (hi hi + hi lo + lo hi), about 16 significant bits per operand.
constexpr int kTLB = 64;   // l-points per LDS tile (4 MFMA k-steps)
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

template <int KIND, int D, int RB, bool X3>
__global__ __launch_bounds__(kThreads) void stage5_bf16_kernel(
    const float *__restrict__ X, const __bf16 *__restrict__ Yh, const __bf16 *__restrict__ Yl,
    float *__restrict__ Z, int64_t Ntpad, int64_t lchunk) {
    __shared__ float sX[D][kTLB];
    __shared__ __attribute__((aligned(16))) __bf16 sYh[kBW][kTLB + 8];
    __shared__ __attribute__((aligned(16))) __bf16 sYl[X3 ? kBW : 1][kTLB + 8];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int i = lane & 31, kh = lane >> 5;
    const int64_t row0 = int64_t(blockIdx.x) * (kWaves * 32 * RB) + int64_t(wave) * 32 * RB;
    const int64_t l0 = int64_t(blockIdx.y) * lchunk;
    const int64_t l1 = min(l0 + lchunk, Ntpad);
    float xk[RB][D];
#pragma unroll
    for (int rb = 0; rb < RB; ++rb)
#pragma unroll
        for (int k = 0; k < D; ++k) xk[rb][k] = X[k * Ntpad + row0 + rb * 32 + i];
    floatx16 acc[RB];
#pragma unroll
    for (int rb = 0; rb < RB; ++rb)
#pragma unroll
        for (int r = 0; r < 16; ++r) acc[rb][r] = 0.f;

    for (int64_t lt = l0; lt < l1; lt += kTLB) {
        __syncthreads();
        // Y (column-major bf16, ld Ntpad): 8 consecutive l of one column per 16-byte load
        {
            const int j = threadIdx.x >> 3, seg = threadIdx.x & 7;   // 32 columns x 8 segments
            const int4 vh = *reinterpret_cast<const int4 *>(Yh + int64_t(j) * Ntpad + lt + 8 * seg);
            *reinterpret_cast<int4 *>(&sYh[j][8 * seg]) = vh;
            if constexpr (X3) {
                const int4 vl = *reinterpret_cast<const int4 *>(Yl + int64_t(j) * Ntpad + lt + 8 * seg);
                *reinterpret_cast<int4 *>(&sYl[j][8 * seg]) = vl;
            }
        }
        if (threadIdx.x < D * kTLB) {
            const int k = threadIdx.x / kTLB, l = threadIdx.x % kTLB;
            sX[k][l] = X[k * Ntpad + lt + l];
        }
        __syncthreads();
#pragma unroll
        for (int ll = 0; ll < kTLB; ll += 16) {
            const int lb = ll + 8 * kh;
            float xl[8][D];
#pragma unroll
            for (int e = 0; e < 8; ++e)
#pragma unroll
                for (int k = 0; k < D; ++k) xl[e][k] = sX[k][lb + e];
            const bf16x8 bh = *reinterpret_cast<const bf16x8 *>(&sYh[i][lb]);
            bf16x8 bl;
            if constexpr (X3) bl = *reinterpret_cast<const bf16x8 *>(&sYl[i][lb]);
#pragma unroll
            for (int rb = 0; rb < RB; ++rb) {
                bf16x8 ah, al;
#pragma unroll
                for (int e = 0; e < 8; ++e) {
                    const float g = gamma_f32<KIND, D>(xk[rb], xl[e]);
                    ah[e] = __bf16(g);
                    if constexpr (X3) al[e] = __bf16(g - float(ah[e]));
                }
                acc[rb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, bh, acc[rb], 0, 0, 0);
                if constexpr (X3) {
                    acc[rb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, bl, acc[rb], 0, 0, 0);
                    acc[rb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al, bh, acc[rb], 0, 0, 0);
                }
            }
        }
    }
    float *Zs = Z + int64_t(blockIdx.y) * Ntpad * kBW + int64_t(i) * Ntpad;
#pragma unroll
    for (int rb = 0; rb < RB; ++rb)
#pragma unroll
        for (int m = 0; m < 4; ++m) {
            const int64_t row = row0 + rb * 32 + 4 * kh + 8 * m;
            float4 v = {acc[rb][4 * m], acc[rb][4 * m + 1], acc[rb][4 * m + 2], acc[rb][4 * m + 3]};
            *reinterpret_cast<float4 *>(Zs + row) = v;
        }
}

constexpr int kRB32 = 2;   // rows per FP32 workgroup: 4 waves x 2 x 32 = 256
constexpr int kRB64 = 4;   // rows per FP64 workgroup: 4 waves x 4 x 16 = 256
constexpr int kRowsPerWG = 256;

template <int KIND, int D>
void launch_kind(int precision, const kl_problem *P, const void *Y5, void *Z5, int nsplit,
                 int64_t lchunk, hipStream_t s) {
    dim3 grid(unsigned(P->Ntpad / kRowsPerWG), unsigned(nsplit));
    if (precision == KL_F64) {
        hipLaunchKernelGGL((stage5_f64_kernel<KIND, D, kRB64>), grid, dim3(kThreads), 0, s,
                           P->dX64, static_cast<const double *>(Y5), static_cast<double *>(Z5),
                           P->Ntpad, lchunk);
    } else if (precision == KL_F32) {
        hipLaunchKernelGGL((stage5_f32_kernel<KIND, D, kRB32>), grid, dim3(kThreads), 0, s,
                           P->dX32, static_cast<const float *>(Y5), static_cast<float *>(Z5),
                           P->Ntpad, lchunk);
    } else {
        // BF16 operands: hi part at Y5, lo part right after it (Ntpad x kBW each)
        const __bf16 *yh = static_cast<const __bf16 *>(Y5);
        const __bf16 *yl = yh + P->Ntpad * kBW;
        if (precision == KL_BF16)
            hipLaunchKernelGGL((stage5_bf16_kernel<KIND, D, kRB32, false>), grid, dim3(kThreads), 0, s,
                               P->dX32, yh, yl, static_cast<float *>(Z5), P->Ntpad, lchunk);
        else
            hipLaunchKernelGGL((stage5_bf16_kernel<KIND, D, kRB32, true>), grid, dim3(kThreads), 0, s,
                               P->dX32, yh, yl, static_cast<float *>(Z5), P->Ntpad, lchunk);
    }
}

template <int D>
void launch_dim(int precision, const kl_problem *P, const void *Y5, void *Z5, int nsplit,
                int64_t lchunk, hipStream_t s) {
    switch (P->cov_kind) {
    case KL_COV_EXP: launch_kind<KL_COV_EXP, D>(precision, P, Y5, Z5, nsplit, lchunk, s); break;
    case KL_COV_SQEXP: launch_kind<KL_COV_SQEXP, D>(precision, P, Y5, Z5, nsplit, lchunk, s); break;
    case KL_COV_EXP_L1: launch_kind<KL_COV_EXP_L1, D>(precision, P, Y5, Z5, nsplit, lchunk, s); break;
    case KL_COV_CONST: launch_kind<KL_COV_CONST, D>(precision, P, Y5, Z5, nsplit, lchunk, s); break;
    default: launch_kind<KL_COV_LIN, D>(precision, P, Y5, Z5, nsplit, lchunk, s); break;
    }
}

}  // namespace

// Number of l-splits: enough workgroups to fill the chip twice over, each split a
// whole number of LDS tiles.
int stage5_splits(int64_t Ntpad, int n_cu, int64_t *lchunk_out) {
    const int64_t row_tiles = Ntpad / kRowsPerWG;
    const int64_t tile = 64;   // common multiple of both LDS tile lengths
    int64_t want = (2 * int64_t(n_cu) + row_tiles - 1) / row_tiles;
    const int64_t max_split = Ntpad / tile;
    if (want > max_split) want = max_split;
    if (want > 64) want = 64;
    if (want < 1) want = 1;
    int64_t lchunk = ((Ntpad + want - 1) / want + tile - 1) / tile * tile;
    int64_t nsplit = (Ntpad + lchunk - 1) / lchunk;
    if (lchunk_out) *lchunk_out = lchunk;
    return int(nsplit);
}

int launch_stage5(const kl_problem *P, int precision, const void *Y5, void *Z5, hipStream_t s) {
    int64_t lchunk;
    const int nsplit = stage5_splits(P->Ntpad, P->n_cu, &lchunk);
    switch (P->hs.d) {
    case 1: launch_dim<1>(precision, P, Y5, Z5, nsplit, lchunk, s); break;
    case 2: launch_dim<2>(precision, P, Y5, Z5, nsplit, lchunk, s); break;
    default: launch_dim<3>(precision, P, Y5, Z5, nsplit, lchunk, s); break;
    }
    return nsplit;
}

}  // namespace kl
