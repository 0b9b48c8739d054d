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
// Coordinates are pre-scaled on the host by log2(e)/ell (exponential kernels) or
// sqrt(log2 e)/ell (squared exponential), so that every kernel evaluates a base-2
// exponential: the hardware one in the FP32 kernels, a polynomial one in FP64.  sigma^2 is applied after the split
// reduction.  Grids are padded with zero points and zero vectors, which add nothing.
#include <algorithm>

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

// FP64 base-2 exponential and square root for the arguments of the covariance kernels only
// (2^x of a finite x <= 0, sqrt of a normal a > 0), without the range and special-value
// handling of the general library functions.  The coordinates of the FP64 kernels are
// scaled on the host by log2(e) / ell (sqrt(log2 e) / ell for the squared exponential), so
// that Gamma = 2^(-rho') with rho' the scaled distance (squared distance).
//  * exp2: x = n + f with n = rint(x) and f = x - n in [-1/2, 1/2] (exact); 2^f as the
//    square of 2^(f/2), which a polynomial of degree 9 in f gives (below; one FMA fewer
//    than a degree-11 polynomial for 2^f itself, at about 1.6 ulp); scaling by 2^n.
//  * sqrt: Goldschmidt iteration from the hardware reciprocal square root y: s = a y and
//    h = y / 2 approximate sqrt(a) and 1 / (2 sqrt(a)); one step s (1 + e), e = 1/2 - s h,
//    squares the relative error of s (to about 2^-44), and a Newton correction
//    s + h (a - s^2) squares it again, below the rounding of s: the correction term is
//    already of relative size 2^-44, so h needs no refinement of its own.  The callers
//    start the squared distance at 1e-300, so that a coincident pair gives
//    sqrt(1e-300) = 1e-150 and 2^(-1e-150) = 1 without a special case (1e-300 is far below
//    the rounding of any non-zero squared distance).
__device__ __forceinline__ double exp2_nonpos(double x) {
    const double n = __builtin_rint(x);
    const double f = x - n;
    // degree-9 interpolant of 2^(f/2) at the 10 Chebyshev nodes of [-1/2, 1/2]
    // (coefficients solved in exact rational arithmetic from 80-digit values, then
    // rounded; interpolation error below 1e-17; squared, the Horner evaluation stays below
    // 3.6e-16 relative); exp_poly.py beside this file regenerates them
    double p = 1.9892645214512514e-10;
    p = fma(p, f, 5.166607104479313e-09);
    p = fma(p, f, 1.1916195315468524e-07);
    p = fma(p, f, 2.4068006815705036e-06);
    p = fma(p, f, 4.166736921023986e-05);
    p = fma(p, f, 0.0006011330693109269);
    p = fma(p, f, 0.006938013583102615);
    p = fma(p, f, 0.06005662673977255);
    p = fma(p, f, 0.34657359027997264);
    p = fma(p, f, 1.0);
    return __builtin_ldexp(p * p, int(n));
}

__device__ __forceinline__ double sqrt_pos(double a) {
    const double y = __builtin_amdgcn_rsq(a);
    double s = a * y;
    const double h = 0.5 * y;
    const double e = fma(-s, h, 0.5);
    s = fma(s, e, s);
    const double d = fma(-s, s, a);
    return fma(d, h, s);
}

template <int KIND, int D>
__device__ __forceinline__ double gamma_f64(const double *xk, const double *xl) {
    if constexpr (KIND == KL_COV_EXP) {
        double r2 = 1e-300;
#pragma unroll
        for (int k = 0; k < D; ++k) { double t = xk[k] - xl[k]; r2 = fma(t, t, r2); }
        return exp2_nonpos(-sqrt_pos(r2));
    } else if constexpr (KIND == KL_COV_SQEXP) {
        double r2 = 0.0;
#pragma unroll
        for (int k = 0; k < D; ++k) { double t = xk[k] - xl[k]; r2 = fma(t, t, r2); }
        return exp2_nonpos(-r2);
    } else if constexpr (KIND == KL_COV_EXP_L1) {
        double s = 0.0;
#pragma unroll
        for (int k = 0; k < D; ++k) s += fabs(xk[k] - xl[k]);
        return exp2_nonpos(-s);
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
constexpr int kRows = 64;                  // rows per FP64 workgroup (shared by its 4 waves)
constexpr int kSub = 64;                   // l-points per wave per step
constexpr int kStep = kWaves * kSub;       // l-points per workgroup step


// End of a workgroup: add the four waves' 32-row blocks (LDS `red`,
// [wave][32 rows][kBW + 1]) and store the block: the final result with one split,
// otherwise the split's partial (added in split order by split_reduce_kernel or by the
// consumer: the fused backward Kronecker launch).
template <typename T, int W = kWaves>
__device__ __forceinline__ void finish_block(const T *red, T *__restrict__ Zpart, T *__restrict__ Zf,
                                             int split, int nsplit, int64_t Ntpad, int64_t row0,
                                             const double *__restrict__ wrow, double scale) {
    constexpr int kPer = (32 * kBW) / (64 * W);          // entries per thread
    T *dst = nsplit == 1 ? Zf : Zpart + int64_t(split) * Ntpad * kBW;
#pragma unroll
    for (int q = 0; q < kPer; ++q) {
        const int e = threadIdx.x + q * (64 * W);
        const int row = e % 32, j = e / 32;
        T acc = T(0);
#pragma unroll
        for (int w = 0; w < W; ++w) acc += red[(w * 32 + row) * (kBW + 1) + j];
        if (nsplit == 1 && wrow) acc = T(double(acc) * scale * wrow[row0 + row]);
        dst[int64_t(j) * Ntpad + row0 + row] = acc;
    }
}

// Zf[e] = w(row) sum_{s < nsplit} Zpart[s][e] in split order (w = scale wrow[row], or 1
// without wrow; row = e mod Ntpad); each thread owns 4 consecutive entries (one column)
// and issues up to 8 splits' 16-byte loads before adding.
template <typename T>
__global__ __launch_bounds__(kThreads) void split_reduce_kernel(const T *__restrict__ Zpart,
                                                                T *__restrict__ Zf, int nsplit,
                                                                int64_t n4, int64_t stride, int64_t Ntpad,
                                                                const double *__restrict__ wrow, double scale) {
    const int64_t e4 = int64_t(blockIdx.x) * kThreads + threadIdx.x;
    if (e4 >= n4) return;
    T acc[4] = {T(0), T(0), T(0), T(0)};
    for (int s0 = 0; s0 < nsplit; s0 += 8) {
        T v[8][4];
#pragma unroll
        for (int u = 0; u < 8; ++u)
            if (s0 + u < nsplit) {
                const T *src = Zpart + int64_t(s0 + u) * stride + 4 * e4;
#pragma unroll
                for (int t = 0; t < 4; ++t) v[u][t] = src[t];
            }
#pragma unroll
        for (int u = 0; u < 8; ++u)
            if (s0 + u < nsplit)
#pragma unroll
                for (int t = 0; t < 4; ++t) acc[t] += v[u][t];
    }
    const int64_t row = (4 * e4) % Ntpad;
#pragma unroll
    for (int t = 0; t < 4; ++t) Zf[4 * e4 + t] = wrow ? T(double(acc[t]) * scale * wrow[row + t]) : acc[t];
}

// Work of one workgroup: rows [row0, row0 + rows_wg) against the l-range [l0, l1) of
// split `split` (of nsplit) of a problem with Ntpad padded points.
struct S5Tile {
    int64_t Ntpad, row0, l0, l1;
    int split, nsplit;
    const double *wrow;     // final rows scaled by scale * wrow[row] (NULL: unscaled)
    double scale;
};

// Workgroup -> (row tile, split).  Workgroups are dispatched to the 8 XCDs of the chip in
// turn (linear id g, x fastest, goes to XCD g mod 8), each XCD with its own L2.  With a
// split count that is a multiple of 8, the workgroups of split s are all placed on XCD
// s mod 8 (slot q = g / 8 of that XCD covers split s = xcd + 8 (q / R), row tile q mod R),
// so each XCD reads only its splits' columns of the stage-5 input instead of all of them.
__device__ __forceinline__ S5Tile grid_tile(int64_t rows_wg, int64_t Ntpad, int64_t lchunk,
                                             const double *wrow, double scale) {
    S5Tile t;
    t.wrow = wrow;
    t.scale = scale;
    t.Ntpad = Ntpad;
    const int64_t R = gridDim.x, S = gridDim.y;
    int64_t rowtile = blockIdx.x, split = blockIdx.y;
    if ((S & 7) == 0) {
        const int64_t g = int64_t(blockIdx.x) + R * int64_t(blockIdx.y);
        const int64_t q = g >> 3;
        rowtile = q % R;
        split = (g & 7) + 8 * (q / R);
    }
    t.row0 = rowtile * rows_wg;
    t.l0 = split * lchunk;
    t.l1 = min(t.l0 + lchunk, Ntpad);
    t.split = int(split);
    t.nsplit = int(S);
    return t;
}

// Skeleton shared by all precisions.  The workgroup owns rows [row0, row0 + 64) and the
// l-range [l0, l1) of its split; each step stages 256 points (and the matching rows of
// the stage-5 input block) in LDS and wave w contracts the 64-point sub-tile w.  At the
// end the four waves' 64 x 32 accumulator tiles are added in LDS and the workgroup writes
// one partial tile, column-major.
//
// FP32: v_mfma_f32_32x32x2_f32, A = Gamma[32 rows][2 l], B = Y[2 l][32 cols]; A[i][k] and
// B[k][j] sit in lane (i or j) + 32 k; accumulator r of lane L holds
// C[(r & 3) + 4 (L >> 5) + 8 (r >> 2)][L & 31].
// LDS of the FP32 skeleton: points [D][kStep] and the block tile [l][kBW + 1] (reused
// for the reduction).
constexpr int kLdsF32Y = kStep * (kBW + 1);

template <int KIND, int D, int RB, int W = kWaves>
__device__ __forceinline__ void stage5_f32_body(const float *__restrict__ X, const float *__restrict__ Y,
                                                float *__restrict__ Z, float *__restrict__ Zf, const S5Tile &t,
                                                float (*sX)[kStep], float *sY) {
    // W waves share the 256-point step: wave w contracts the sub-tile of kStep / W points
    constexpr int kNT = 64 * W, kSubW = kStep / W;
    constexpr int kLd4 = (kStep * kBW / 4) / kNT;        // float4 loads per thread per step
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int i = lane & 31, kh = lane >> 5;
    const int64_t Ntpad = t.Ntpad, row0 = t.row0, l0 = t.l0, l1 = t.l1;
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
    // prefetch registers: the next step's Y rows (16-byte loads) and points.  l1 - l0 is a
    // multiple of 64 (Ntpad and lchunk are), so a wave whose first point is below l1 has all
    // kSubW of its points below l1 and the other waves skip the step: staged points at or
    // past l1 are never read, and their loads are clamped into the split (no zero fill).
    static_assert(64 % kSubW == 0, "a wave sub-tile divides the 64-point granule of the splits");
    float4 py[kLd4];
    float px[D];
    auto prefetch = [&](int64_t lt) {
#pragma unroll
        for (int q = 0; q < kLd4; ++q) {
            const int e = threadIdx.x + q * kNT;
            const int l4 = e % (kStep / 4), j = e / (kStep / 4);
            const int64_t lg = min(lt + 4 * l4, l1 - 4);
            py[q] = *reinterpret_cast<const float4 *>(Y + int64_t(j) * Ntpad + lg);
        }
        const int64_t lg = min(lt + int64_t(threadIdx.x), l1 - 1);
#pragma unroll
        for (int k = 0; k < D; ++k) px[k] = threadIdx.x < kStep ? X[k * Ntpad + lg] : 0.f;
    };
    prefetch(l0);
    for (int64_t lt = l0; lt < l1; lt += kStep) {
        __syncthreads();
#pragma unroll
        for (int q = 0; q < kLd4; ++q) {
            const int e = threadIdx.x + q * kNT;
            const int l4 = e % (kStep / 4), j = e / (kStep / 4);
            sY[(4 * l4 + 0) * (kBW + 1) + j] = py[q].x;
            sY[(4 * l4 + 1) * (kBW + 1) + j] = py[q].y;
            sY[(4 * l4 + 2) * (kBW + 1) + j] = py[q].z;
            sY[(4 * l4 + 3) * (kBW + 1) + j] = py[q].w;
        }
        if (threadIdx.x < kStep)
#pragma unroll
            for (int k = 0; k < D; ++k) sX[k][threadIdx.x] = px[k];
        __syncthreads();
        if (lt + kStep < l1) prefetch(lt + kStep);       // lands while this step computes
        if (lt + wave * kSubW < l1) {
            const int base = wave * kSubW;
#pragma unroll 8
            for (int ll = 0; ll < kSubW; ll += 2) {
                float xl[D];
#pragma unroll
                for (int k = 0; k < D; ++k) xl[k] = sX[k][base + ll + kh];
                const float b = sY[(base + ll + kh) * (kBW + 1) + i];
#pragma unroll
                for (int rb = 0; rb < RB; ++rb) {
                    const float g = gamma_f32<KIND, D>(xk[rb], xl);
                    acc[rb] = __builtin_amdgcn_mfma_f32_32x32x2f32(g, b, acc[rb], 0, 0, 0);
                }
            }
        }
    }
    // ---- reduce the four waves (one 32-row block at a time) and write ------------------
#pragma unroll
    for (int rb = 0; rb < RB; ++rb) {
        __syncthreads();
        float *red = sY;                                  // [wave][32 rows][kBW + 1]
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const int row = (r & 3) + 4 * kh + 8 * (r >> 2);
            red[(wave * 32 + row) * (kBW + 1) + i] = acc[rb][r];
        }
        __syncthreads();
        finish_block<float, W>(red, Z, Zf, t.split, t.nsplit, Ntpad, row0 + rb * 32, t.wrow, t.scale);
    }
}

template <int KIND, int D, int RB, int W = kWaves>
__global__ __launch_bounds__(64 * W) void stage5_f32_kernel(
    const float *__restrict__ X, const float *__restrict__ Y, float *__restrict__ Z,
    float *__restrict__ Zf, int64_t Ntpad, int64_t lchunk, const double *__restrict__ wrow, double scale) {
    __shared__ float sX[D][kStep];
    __shared__ float sY[kLdsF32Y];
    stage5_f32_body<KIND, D, RB, W>(X, Y, Z, Zf, grid_tile(32 * RB, Ntpad, lchunk, wrow, scale), sX, sY);
}

// FP64: v_mfma_f64_16x16x4_f64, A = Gamma[16 rows][4 l], B = Y[4 l][16 cols]; A[i][k] and
// B[k][j] sit in lane (i or j) + 16 k; accumulator r of lane L holds C[(L >> 4) + 4 r][L & 15]
// (measured on gfx950; differs from the FP32 16x16x4 layout).  Four 16-row tiles x two
// 16-column halves per wave.
template <int KIND, int D>
__device__ __forceinline__ void stage5_f64_body(const double *__restrict__ X, const double *__restrict__ Y,
                                                double *__restrict__ Z, double *__restrict__ Zf,
                                                const S5Tile &t, double *sm64) {
    double *sX = sm64;                           // [D][kStep]
    double *sY = sm64 + D * kStep;               // [l][kBW + 1]; reduction reuses it all
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int i = lane & 15, kq = lane >> 4;
    const int64_t Ntpad = t.Ntpad, row0 = t.row0, l0 = t.l0, l1 = t.l1;
    double xk[4][D];
#pragma unroll
    for (int rb = 0; rb < 4; ++rb)
#pragma unroll
        for (int k = 0; k < D; ++k) xk[rb][k] = X[k * Ntpad + row0 + rb * 16 + i];
    doublex4 acc[4][2];
#pragma unroll
    for (int rb = 0; rb < 4; ++rb)
#pragma unroll
        for (int r = 0; r < 4; ++r) { acc[rb][0][r] = 0.0; acc[rb][1][r] = 0.0; }
    for (int64_t lt = l0; lt < l1; lt += kStep) {
        __syncthreads();
        // l1 - l0 is a multiple of kSub (Ntpad and lchunk are), so a wave whose first point
        // is below l1 has all kSub of its points below l1 and the other waves skip the step:
        // staged points at or past l1 are never read.  Their loads are clamped into the split
        // (no zero fill, no branch).  Every load of a thread is at l = 2 (tid mod kStep/2).
        static_assert(kThreads % (kStep / 2) == 0, "one l per thread in the Y staging");
        static_assert(64 % kSub == 0, "a wave sub-tile divides the 64-point granule of the splits");
        const int64_t lgy = min(lt + 2 * (threadIdx.x % (kStep / 2)), l1 - 2);
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            // 16-byte loads (2 consecutive l of one column), 8 in flight per thread
            double2 v[8];
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                const int j = (threadIdx.x + (h * 8 + q) * kThreads) / (kStep / 2);
                v[q] = *reinterpret_cast<const double2 *>(Y + int64_t(j) * Ntpad + lgy);
            }
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                const int e = threadIdx.x + (h * 8 + q) * kThreads;
                const int l2 = e % (kStep / 2), j = e / (kStep / 2);
                sY[(2 * l2 + 0) * (kBW + 1) + j] = v[q].x;
                sY[(2 * l2 + 1) * (kBW + 1) + j] = v[q].y;
            }
        }
        const int64_t lgx = min(lt + int64_t(threadIdx.x), l1 - 1);
#pragma unroll
        for (int k = 0; k < D; ++k) sX[k * kStep + threadIdx.x] = X[k * Ntpad + lgx];
        __syncthreads();
        if (lt + wave * kSub < l1) {
            const int base = wave * kSub;
#pragma unroll 2
            for (int ll = 0; ll < kSub; ll += 4) {
                double xl[D];
#pragma unroll
                for (int k = 0; k < D; ++k) xl[k] = sX[k * kStep + base + ll + kq];
                const double b0 = sY[(base + ll + kq) * (kBW + 1) + i];
                const double b1 = sY[(base + ll + kq) * (kBW + 1) + 16 + i];
#pragma unroll
                for (int rb = 0; rb < 4; ++rb) {
                    const double g = gamma_f64<KIND, D>(xk[rb], xl);
                    acc[rb][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(g, b0, acc[rb][0], 0, 0, 0);
                    acc[rb][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(g, b1, acc[rb][1], 0, 0, 0);
                }
            }
        }
    }
#pragma unroll
    for (int half = 0; half < 2; ++half) {
        __syncthreads();
        double *red = sm64;                               // [wave][32 rows][kBW + 1]
#pragma unroll
        for (int rb = 2 * half; rb < 2 * half + 2; ++rb)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int row = (rb - 2 * half) * 16 + kq + 4 * r;
                red[(wave * 32 + row) * (kBW + 1) + i] = acc[rb][0][r];
                red[(wave * 32 + row) * (kBW + 1) + 16 + i] = acc[rb][1][r];
            }
        __syncthreads();
        finish_block<double>(red, Z, Zf, t.split, t.nsplit, Ntpad, row0 + 32 * half, t.wrow, t.scale);
    }
}
constexpr size_t kLds64 = size_t(3 * kStep + kStep * (kBW + 1)) * sizeof(double);

template <int KIND, int D>
__global__ __launch_bounds__(kThreads) void stage5_f64_kernel(
    const double *__restrict__ X, const double *__restrict__ Y, double *__restrict__ Z,
    double *__restrict__ Zf, int64_t Ntpad, int64_t lchunk, const double *__restrict__ wrow, double scale) {
    extern __shared__ double sm64[];
    stage5_f64_body<KIND, D>(X, Y, Z, Zf, grid_tile(kRows, Ntpad, lchunk, wrow, scale), sm64);
}

// BF16: v_mfma_f32_32x32x16_bf16, A = Gamma[32 rows][16 l], B = Y[16 l][32 cols];
// A[i][k] in lane i + 32 (k / 8), element k % 8; B[k][j] in lane j + 32 (k / 8), element
// k % 8; accumulators as for the FP32 32x32x2 (measured on gfx950).  The kernel value is
// evaluated in FP32 and rounded to BF16 (nearest even).  With X3 both operands are split
// into hi + lo BF16 parts and hi hi + hi lo + lo hi are accumulated.
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

template <int KIND, int D, int RB, bool X3>
__global__ __launch_bounds__(kThreads) void stage5_bf16_kernel(
    const float *__restrict__ X, const __bf16 *__restrict__ Yh, const __bf16 *__restrict__ Yl,
    float *__restrict__ Z, float *__restrict__ Zf, int64_t Ntpad, int64_t lchunk,
    const double *__restrict__ wrow, double scale) {
    constexpr int rows_wg = 32 * RB;
    constexpr int ldb = kStep + 8;               // bf16 row of one column (16-byte aligned)
    constexpr int kLd = (kBW * kStep / 8) / kThreads;   // 16-byte loads per thread per step
    __shared__ float sX[D][kStep];
    __shared__ __attribute__((aligned(16))) __bf16 sYh[kBW * ldb];
    __shared__ __attribute__((aligned(16))) __bf16 sYl[X3 ? kBW * ldb : 8];
    __shared__ float red[kWaves * 32 * (kBW + 1)];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int i = lane & 31, kh = lane >> 5;
    const S5Tile tile = grid_tile(rows_wg, Ntpad, lchunk, wrow, scale);
    const int64_t row0 = tile.row0, l0 = tile.l0, l1 = tile.l1;
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
    int4 ph[kLd], pl[kLd];
    float px[D];
    // Steps wholly inside [l0, l1) load without bounds checks; the last one zero-fills the
    // points past l1 (zero Y rows, so those products add exact zeros).
    auto prefetch = [&](int64_t lt) {
        if (lt + kStep <= l1) {
#pragma unroll
            for (int q = 0; q < kLd; ++q) {
                const int e = threadIdx.x + q * kThreads;
                const int j = e / (kStep / 8), seg = e % (kStep / 8);
                const int64_t lg = lt + 8 * seg;
                ph[q] = *reinterpret_cast<const int4 *>(Yh + int64_t(j) * Ntpad + lg);
                if constexpr (X3) pl[q] = *reinterpret_cast<const int4 *>(Yl + int64_t(j) * Ntpad + lg);
            }
#pragma unroll
            for (int k = 0; k < D; ++k) px[k] = X[k * Ntpad + lt + threadIdx.x];
            return;
        }
#pragma unroll
        for (int q = 0; q < kLd; ++q) {
            const int e = threadIdx.x + q * kThreads;
            const int j = e / (kStep / 8), seg = e % (kStep / 8);
            const int64_t lg = lt + 8 * seg;
            ph[q] = int4{0, 0, 0, 0};
            pl[q] = int4{0, 0, 0, 0};
            if (lg < l1) {
                ph[q] = *reinterpret_cast<const int4 *>(Yh + int64_t(j) * Ntpad + lg);
                if constexpr (X3) pl[q] = *reinterpret_cast<const int4 *>(Yl + int64_t(j) * Ntpad + lg);
            }
        }
#pragma unroll
        for (int k = 0; k < D; ++k) {
            const int64_t lg = lt + threadIdx.x;
            px[k] = lg < l1 ? X[k * Ntpad + lg] : 0.f;
        }
    };
    prefetch(l0);
    for (int64_t lt = l0; lt < l1; lt += kStep) {
        __syncthreads();
#pragma unroll
        for (int q = 0; q < kLd; ++q) {
            const int e = threadIdx.x + q * kThreads;
            const int j = e / (kStep / 8), seg = e % (kStep / 8);
            *reinterpret_cast<int4 *>(&sYh[j * ldb + 8 * seg]) = ph[q];
            if constexpr (X3) *reinterpret_cast<int4 *>(&sYl[j * ldb + 8 * seg]) = pl[q];
        }
#pragma unroll
        for (int k = 0; k < D; ++k) sX[k][threadIdx.x] = px[k];
        __syncthreads();
        if (lt + kStep < l1) prefetch(lt + kStep);
        // every wave runs the whole step: a wave past l1 multiplies zero Y rows, and without
        // a branch around the loop the accumulators stay in place across steps
        {
            const int base = wave * kSub;
#pragma unroll
            for (int ll = 0; ll < kSub; ll += 16) {
                const int lb = base + ll + 8 * kh;
                float xl[8][D];
#pragma unroll
                for (int e = 0; e < 8; ++e)
#pragma unroll
                    for (int k = 0; k < D; ++k) xl[e][k] = sX[k][lb + e];
                const bf16x8 bh = *reinterpret_cast<const bf16x8 *>(&sYh[i * ldb + lb]);
                bf16x8 bl;
                if constexpr (X3) bl = *reinterpret_cast<const bf16x8 *>(&sYl[i * ldb + lb]);
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
    }
#pragma unroll
    for (int rb = 0; rb < RB; ++rb) {
        __syncthreads();
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const int row = (r & 3) + 4 * kh + 8 * (r >> 2);
            red[(wave * 32 + row) * (kBW + 1) + i] = acc[rb][r];
        }
        __syncthreads();
        finish_block<float>(red, Z, Zf, tile.split, tile.nsplit, Ntpad, row0 + rb * 32, wrow, scale);
    }
}


// ---- symmetric FP64 stage 5 ---------------------------------------------------------------
// Gamma is symmetric, so one kernel value serves two products: z_r += Gamma(x_r, x_c) y_c and
// z_c += Gamma(x_r, x_c) y_r.  The points are cut into 256-point column blocks J and 64-point
// row tiles t; a work item is column block J with a run [t0, t1) of the row tiles t < 4 J + 4
// (the tiles of the blocks at or below J).  The workgroup has 8 waves (two per SIMD): wave
// (cs, rh) owns the 64 columns 256 J + 64 cs + [0, 64) and rows 32 rh + [0, 32) of every row
// tile.  It evaluates its 32 x 64 kernel values once and contracts them twice on the FP64
// matrix cores:
//   * transposed: O += G^T Y_t into the wave's accumulators (64 columns x kBW), kept over
//     the item; at its end the two row halves are added (rh order) and stored as the item's
//     owned partial;
//   * forward (tiles below the diagonal block only): F = G Y_J (32 rows x kBW), added over
//     the four column slabs in LDS (slab order) and stored as the partial of slot (t, J).
// The diagonal block (t >= 4 J) takes the transposed product only: over its four row tiles
// it adds every l of block J to the owned columns.  sym_reduce_kernel then adds, per row, the
// owned partials of its block (item order) and the forward partials of the blocks above it
// (block order): every sum is taken in a fixed order.
//
// Lane layouts (v_mfma_f64_16x16x4f64, A[i][k] in lane i + 16 k, B[k][j] in lane j + 16 k,
// D[(lane >> 4) + 4 r][lane & 15]): lane (i, k) evaluates G[row 16 p + 4 m + k][col 16 q + i]
// for m < 4, which is the A operand of the transposed product as it stands; the forward
// product needs G[row 16 p + i][col 16 q + 4 m + k], which the wave reads back from a
// 16 x 16 tile it has just written to LDS.
constexpr int kSymWaves = 8;
constexpr int kSymThreads = 64 * kSymWaves;
constexpr int kSymCols = 256;                         // columns of a block (4 slabs x 64)
constexpr int kSymTile = 64;                          // rows of a row tile (2 halves x 32)
constexpr int kSymLd = kBW + 1;                       // LDS row length of the [point][vec] arrays
constexpr int kSymYJ = kSymCols * kSymLd;             // LDS: Y of the owned block [col][vec]
constexpr int kSymXt = 3 * kSymTile;                  // LDS: points of the row tile [d][row]
constexpr int kSymYt = kSymTile * kSymLd;             // LDS: Y of the row tile [row][vec]
constexpr int kSymRed = 4 * kSymTile * kSymLd;        // LDS: [slab][64][vec] partials; holds the
constexpr int kSymTr = 16 * 17;                       //      waves' transposition tiles meanwhile
static_assert(kSymWaves * kSymTr <= kSymRed, "transposition tiles inside the reduction area");
constexpr int kSymXJ = 3 * kSymCols;                 // LDS: points of the owned block [d][col]
constexpr size_t kLdsSym = size_t(kSymYJ + kSymXJ + kSymXt + kSymYt + kSymRed) * sizeof(double);
static_assert(kLdsSym <= 160 * 1024, "LDS of one gfx950 workgroup");

template <int KIND, int D>
__global__ __launch_bounds__(kSymThreads) void stage5_f64_sym_kernel(
    const double *__restrict__ X, const double *__restrict__ Y, int64_t Ntpad,
    const SymItem *__restrict__ items, int n_items, double *__restrict__ Fp, double *__restrict__ Op) {
    extern __shared__ double sm64[];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int i = lane & 15, k = lane >> 4;
    const int cs = wave & 3, rh = wave >> 2;
    double *sYJ = sm64;                                   // [256 cols][kSymLd]
    double *sXJ = sYJ + kSymYJ;                           // [D][256]
    double *sXt = sXJ + kSymXJ;                           // [D][64]
    double *sYt = sXt + kSymXt;                           // [64 rows][kSymLd]
    double *red = sYt + kSymYt;                           // [slab][64][kSymLd]
    double *tr = red + wave * kSymTr;                     // this wave's [16][17], while computing
    const int G = gridDim.x, g = blockIdx.x;
    // items longest first, dealt to the workgroups in snake order
    for (int round = 0;; ++round) {
        const int idx = round * G + ((round & 1) ? G - 1 - g : g);
        if (idx >= n_items) break;
        const SymItem I = items[idx];
        const int64_t cb = int64_t(I.J) * kSymCols;                  // the block's first column
        // the row tile's points and block rows, prefetched one tile ahead: thread e < 64
        // holds the point 64 t + e, every thread 2 pairs of rows (e = tid + 512 u: vector
        // e >> 5, rows 2 (e & 31) and the next)
        double px[D];
        double2 py[2];
        auto prefetch = [&](int tt) {
            const int64_t rr0 = int64_t(tt) * kSymTile;
#pragma unroll
            for (int d = 0; d < D; ++d) px[d] = threadIdx.x < kSymTile ? X[d * Ntpad + rr0 + threadIdx.x] : 0.0;
#pragma unroll
            for (int u = 0; u < 2; ++u) {
                const int e = threadIdx.x + u * kSymThreads;
                py[u] = *reinterpret_cast<const double2 *>(Y + int64_t(e >> 5) * Ntpad + rr0 + 2 * (e & 31));
            }
        };
        prefetch(I.t0);
        // the owned block's rows of Y, [col][vec] (e = tid + 512 u: vector e >> 7, columns
        // 2 (e & 127) and the next); every wave is past the previous item's last reads
        __syncthreads();
        if (threadIdx.x < kSymCols)
#pragma unroll
            for (int d = 0; d < D; ++d) sXJ[d * kSymCols + threadIdx.x] = X[d * Ntpad + cb + threadIdx.x];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int e = threadIdx.x + u * kSymThreads;
            const int vec = e >> 7, cc = 2 * (e & 127);
            const double2 v = *reinterpret_cast<const double2 *>(Y + int64_t(vec) * Ntpad + cb + cc);
            sYJ[cc * kSymLd + vec] = v.x;
            sYJ[(cc + 1) * kSymLd + vec] = v.y;
        }
        doublex4 O[4][2];
#pragma unroll
        for (int q = 0; q < 4; ++q)
#pragma unroll
            for (int r = 0; r < 4; ++r) { O[q][0][r] = 0.0; O[q][1][r] = 0.0; }
        for (int t = I.t0; t < I.t1; ++t) {
            const bool diag = t >= 4 * I.J;
            // after an off-diagonal tile the barriers around its reduction already ordered
            // every read of the staging area before these writes
            if (t > I.t0 && t - 1 >= 4 * I.J) __syncthreads();
            if (threadIdx.x < kSymTile)
#pragma unroll
                for (int d = 0; d < D; ++d) sXt[d * kSymTile + threadIdx.x] = px[d];
#pragma unroll
            for (int u = 0; u < 2; ++u) {
                const int e = threadIdx.x + u * kSymThreads;
                const int vec = e >> 5, rr = 2 * (e & 31);
                sYt[rr * kSymLd + vec] = py[u].x;
                sYt[(rr + 1) * kSymLd + vec] = py[u].y;
            }
            __syncthreads();
            if (t + 1 < I.t1) prefetch(t + 1);               // lands while this tile computes
            doublex4 F[2][2];
#pragma unroll
            for (int pp = 0; pp < 2; ++pp)
#pragma unroll
                for (int r = 0; r < 4; ++r) { F[pp][0][r] = 0.0; F[pp][1][r] = 0.0; }
#pragma unroll
            for (int pp = 0; pp < 2; ++pp) {
                const int p = 2 * rh + pp;
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    // operands read from LDS per (p, q): few registers stay live across it
                    double xr[4][D], yr[4][2], xc[D], gv[4];
#pragma unroll
                    for (int m = 0; m < 4; ++m) {
#pragma unroll
                        for (int d = 0; d < D; ++d) xr[m][d] = sXt[d * kSymTile + 16 * p + 4 * m + k];
#pragma unroll
                        for (int h = 0; h < 2; ++h) yr[m][h] = sYt[(16 * p + 4 * m + k) * kSymLd + 16 * h + i];
                    }
#pragma unroll
                    for (int d = 0; d < D; ++d) xc[d] = sXJ[d * kSymCols + 64 * cs + 16 * q + i];
#pragma unroll
                    for (int m = 0; m < 4; ++m) gv[m] = gamma_f64<KIND, D>(xr[m], xc);
                    if (!diag) {
                        // transpose through LDS first, so that the round trip overlaps the
                        // transposed products
#pragma unroll
                        for (int m = 0; m < 4; ++m) tr[(4 * m + k) * 17 + i] = gv[m];
                        __builtin_amdgcn_wave_barrier();
                        double gt[4], yb[4][2];
#pragma unroll
                        for (int m = 0; m < 4; ++m) {
                            gt[m] = tr[i * 17 + 4 * m + k];
#pragma unroll
                            for (int h = 0; h < 2; ++h) yb[m][h] = sYJ[(64 * cs + 16 * q + 4 * m + k) * kSymLd + 16 * h + i];
                        }
                        __builtin_amdgcn_wave_barrier();
#pragma unroll
                        for (int m = 0; m < 4; ++m) {
                            O[q][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(gv[m], yr[m][0], O[q][0], 0, 0, 0);
                            O[q][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(gv[m], yr[m][1], O[q][1], 0, 0, 0);
                        }
#pragma unroll
                        for (int m = 0; m < 4; ++m) {
                            F[pp][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(gt[m], yb[m][0], F[pp][0], 0, 0, 0);
                            F[pp][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(gt[m], yb[m][1], F[pp][1], 0, 0, 0);
                        }
                    } else {
#pragma unroll
                        for (int m = 0; m < 4; ++m) {
                            O[q][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(gv[m], yr[m][0], O[q][0], 0, 0, 0);
                            O[q][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(gv[m], yr[m][1], O[q][1], 0, 0, 0);
                        }
                    }
                }
            }
            if (!diag) {
                __syncthreads();                              // every wave done with its tile
#pragma unroll
                for (int pp = 0; pp < 2; ++pp)
#pragma unroll
                    for (int h = 0; h < 2; ++h)
#pragma unroll
                        for (int r = 0; r < 4; ++r)
                            red[(cs * kSymTile + 16 * (2 * rh + pp) + k + 4 * r) * kSymLd + 16 * h + i] = F[pp][h][r];
                __syncthreads();
                double *dst = Fp + (int64_t(2) * I.J * (I.J - 1) + t) * (kSymTile * kBW);
#pragma unroll
                for (int u = 0; u < (kSymTile * kBW) / kSymThreads; ++u) {
                    const int e = threadIdx.x + u * kSymThreads;
                    const int row = e >> 5, vec = e & 31;
                    double acc = 0.0;
#pragma unroll
                    for (int w = 0; w < 4; ++w) acc += red[(w * kSymTile + row) * kSymLd + vec];
                    dst[e] = acc;                             // [row][vec]
                }
            }
        }
        // the owned partial of the item, [column of the block][vec]: row half 0 plus row half 1
        __syncthreads();
        if (rh == 1)
#pragma unroll
            for (int q = 0; q < 4; ++q)
#pragma unroll
                for (int h = 0; h < 2; ++h)
#pragma unroll
                    for (int r = 0; r < 4; ++r)
                        red[(cs * 64 + 16 * q + k + 4 * r) * kSymLd + 16 * h + i] = O[q][h][r];
        __syncthreads();
        if (rh == 0) {
            double *dst = Op + int64_t(I.oslot) * (kSymCols * kBW);
#pragma unroll
            for (int q = 0; q < 4; ++q)
#pragma unroll
                for (int h = 0; h < 2; ++h)
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const int col = 16 * q + k + 4 * r;
                        dst[(cs * 64 + col) * kBW + 16 * h + i] = O[q][h][r] + red[(cs * 64 + col) * kSymLd + 16 * h + i];
                    }
        }
    }
}

// Symmetric BF16 / BF16x3 stage 5: the same work items and partial-sum slots as the FP64
// form, with FP32 partial sums.  Wave w of the 8 owns the 32 columns 256 J + 32 w + [0, 32)
// and takes both 32-row halves of every row tile.  Lane (c, kh) (c = lane & 31, kh = lane >>
// 5) evaluates G[row 16 m + 8 kh + e][col c] for m < 2, e < 8 of a half: eight consecutive
// rows of its own column, which is the A operand of the transposed product
// (v_mfma_f32_32x32x16_bf16, A[i][k] = element k % 8 of lane i + 32 (k / 8)) as it stands;
// the forward product needs G[row i][cols 16 m + 8 kh + e], read back (16-byte loads) from a
// 32 x 32 tile the wave has just written to LDS.  With X3 the kernel values and both blocks
// are split into BF16 hi + lo parts and hi hi + hi lo + lo hi are accumulated, in each product.
constexpr int kSbLdJ = kSymCols + 8;                  // bf16 row of the owned block, [vec][col]
constexpr int kSbLdT = kSymTile + 8;                  // bf16 row of the row tile, [vec][row]
constexpr int kSbLdTr = 32 + 8;                       // bf16 row of a transposition tile
constexpr int kSbRedLd = kBW + 1;                     // FP32 forward partials [wave][row][vec]

template <bool X3>
struct SymBf16Lds {
    __bf16 yj[X3 ? 2 : 1][kBW * kSbLdJ];              // owned block of vectors (hi, lo)
    __bf16 yt[X3 ? 2 : 1][kBW * kSbLdT];              // row tile of vectors (hi, lo)
    __bf16 tr[kSymWaves][X3 ? 2 : 1][32 * kSbLdTr];   // the waves' transposition tiles
    float xj[3][kSymCols];                            // points of the owned block [d][col]
    float xt[3][kSymTile];                            // points of the row tile [d][row]
    float red[kSymWaves * kSymTile * kSbRedLd];       // forward partials [wave][row][vec]
};

template <int KIND, int D, bool X3>
__global__ __launch_bounds__(kSymThreads) void stage5_bf16_sym_kernel(
    const float *__restrict__ X, const __bf16 *__restrict__ Yh, const __bf16 *__restrict__ Yl, int64_t Ntpad,
    const SymItem *__restrict__ items, int n_items, float *__restrict__ Fp, float *__restrict__ Op) {
    constexpr int NP = X3 ? 2 : 1;                    // parts of a BF16 operand
    extern __shared__ __attribute__((aligned(16))) char smb[];
    SymBf16Lds<X3> &L = *reinterpret_cast<SymBf16Lds<X3> *>(smb);
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int c = lane & 31, kh = lane >> 5;
    const __bf16 *Ysrc[2] = {Yh, Yl};
    __bf16 *tr = L.tr[wave][0];
    const int G = gridDim.x, g = blockIdx.x;
    for (int round = 0;; ++round) {
        const int idx = round * G + ((round & 1) ? G - 1 - g : g);
        if (idx >= n_items) break;
        const SymItem I = items[idx];
        const int64_t cb = int64_t(I.J) * kSymCols;
        // the row tile's points and vectors, prefetched one tile ahead: thread e < 64 holds
        // the point 64 t + e; the vectors as 16-byte pieces (8 rows of one vector): 32 x 8
        // pieces per part, thread e < 256 takes vector e >> 3, rows 8 (e & 7)
        float px[D];
        int4 pyh = int4{0, 0, 0, 0}, pyl = int4{0, 0, 0, 0};
        auto prefetch = [&](int tt) {
            const int64_t rr0 = int64_t(tt) * kSymTile;
#pragma unroll
            for (int d = 0; d < D; ++d) px[d] = threadIdx.x < kSymTile ? X[d * Ntpad + rr0 + threadIdx.x] : 0.f;
            if (threadIdx.x < kBW * 8) {
                const int64_t off = int64_t(threadIdx.x >> 3) * Ntpad + rr0 + 8 * (threadIdx.x & 7);
                pyh = *reinterpret_cast<const int4 *>(Yh + off);
                if constexpr (X3) pyl = *reinterpret_cast<const int4 *>(Yl + off);
            }
        };
        prefetch(I.t0);
        __syncthreads();                                  // every wave is past the last item
        // owned block: points, and vectors [vec][col] (32 x 32 pieces of 8 columns per part)
        if (threadIdx.x < kSymCols)
#pragma unroll
            for (int d = 0; d < D; ++d) L.xj[d][threadIdx.x] = X[d * Ntpad + cb + threadIdx.x];
#pragma unroll
        for (int u = 0; u < 2; ++u) {
            const int e = threadIdx.x + u * kSymThreads;      // 1024 pieces
            const int vec = e >> 5, c8 = 8 * (e & 31);
#pragma unroll
            for (int pp = 0; pp < NP; ++pp)
                *reinterpret_cast<int4 *>(&L.yj[pp][vec * kSbLdJ + c8]) =
                    *reinterpret_cast<const int4 *>(Ysrc[pp] + int64_t(vec) * Ntpad + cb + c8);
        }
        __syncthreads();
        // per item: the lane's column point and the forward B operands of its 32 columns,
        // B[k = col 16 m + 8 kh + e][j = vec c]
        float xc[D];
#pragma unroll
        for (int d = 0; d < D; ++d) xc[d] = L.xj[d][32 * wave + c];
        bf16x8 bj[2][NP];
#pragma unroll
        for (int m = 0; m < 2; ++m)
#pragma unroll
            for (int pp = 0; pp < NP; ++pp)
                bj[m][pp] = *reinterpret_cast<const bf16x8 *>(&L.yj[pp][c * kSbLdJ + 32 * wave + 16 * m + 8 * kh]);
        floatx16 O;
#pragma unroll
        for (int r = 0; r < 16; ++r) O[r] = 0.f;
        for (int t = I.t0; t < I.t1; ++t) {
            const bool diag = t >= 4 * I.J;
            if (t > I.t0 && t - 1 >= 4 * I.J) __syncthreads();
            if (threadIdx.x < kSymTile)
#pragma unroll
                for (int d = 0; d < D; ++d) L.xt[d][threadIdx.x] = px[d];
            if (threadIdx.x < kBW * 8) {
                const int o = (threadIdx.x >> 3) * kSbLdT + 8 * (threadIdx.x & 7);
                *reinterpret_cast<int4 *>(&L.yt[0][o]) = pyh;
                if constexpr (X3) *reinterpret_cast<int4 *>(&L.yt[NP - 1][o]) = pyl;
            }
            __syncthreads();
            if (t + 1 < I.t1) prefetch(t + 1);
            floatx16 F[2];
#pragma unroll
            for (int h2 = 0; h2 < 2; ++h2) {
#pragma unroll
                for (int r = 0; r < 16; ++r) F[h2][r] = 0.f;
#pragma unroll
                for (int m = 0; m < 2; ++m) {
                    const int rb = 32 * h2 + 16 * m + 8 * kh;     // the lane's 8 rows
                    float xr[8][D];
#pragma unroll
                    for (int e = 0; e < 8; ++e)
#pragma unroll
                        for (int d = 0; d < D; ++d) xr[e][d] = L.xt[d][rb + e];
                    bf16x8 ah, al;
#pragma unroll
                    for (int e = 0; e < 8; ++e) {
                        const float gv = gamma_f32<KIND, D>(xc, xr[e]);
                        ah[e] = __bf16(gv);
                        if constexpr (X3) al[e] = __bf16(gv - float(ah[e]));
                    }
                    const bf16x8 bh = *reinterpret_cast<const bf16x8 *>(&L.yt[0][c * kSbLdT + rb]);
                    O = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, bh, O, 0, 0, 0);
                    if constexpr (X3) {
                        const bf16x8 bl = *reinterpret_cast<const bf16x8 *>(&L.yt[1][c * kSbLdT + rb]);
                        O = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, bl, O, 0, 0, 0);
                        O = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al, bh, O, 0, 0, 0);
                    }
                    if (!diag) {
                        // G[row 16 m + 8 kh + e][col c] of the half into the tile
#pragma unroll
                        for (int e = 0; e < 8; ++e) {
                            tr[(16 * m + 8 * kh + e) * kSbLdTr + c] = ah[e];
                            if constexpr (X3) tr[32 * kSbLdTr + (16 * m + 8 * kh + e) * kSbLdTr + c] = al[e];
                        }
                    }
                }
                if (!diag) {
                    __builtin_amdgcn_wave_barrier();
                    // forward: A[i = row c][k = col 16 m + 8 kh + e] from the tile
#pragma unroll
                    for (int m = 0; m < 2; ++m) {
                        const bf16x8 fh = *reinterpret_cast<const bf16x8 *>(&tr[c * kSbLdTr + 16 * m + 8 * kh]);
                        F[h2] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(fh, bj[m][0], F[h2], 0, 0, 0);
                        if constexpr (X3) {
                            const bf16x8 fl =
                                *reinterpret_cast<const bf16x8 *>(&tr[32 * kSbLdTr + c * kSbLdTr + 16 * m + 8 * kh]);
                            F[h2] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(fh, bj[m][NP - 1], F[h2], 0, 0, 0);
                            F[h2] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(fl, bj[m][0], F[h2], 0, 0, 0);
                        }
                    }
                    __builtin_amdgcn_wave_barrier();
                }
            }
            if (!diag) {
                // D[(r & 3) + 4 kh + 8 (r >> 2)][c]: row of the half, vector c
#pragma unroll
                for (int h2 = 0; h2 < 2; ++h2)
#pragma unroll
                    for (int r = 0; r < 16; ++r)
                        L.red[(wave * kSymTile + 32 * h2 + (r & 3) + 4 * kh + 8 * (r >> 2)) * kSbRedLd + c] = F[h2][r];
                __syncthreads();
                float *dst = Fp + (int64_t(2) * I.J * (I.J - 1) + t) * (kSymTile * kBW);
#pragma unroll
                for (int u = 0; u < (kSymTile * kBW) / kSymThreads; ++u) {
                    const int e = threadIdx.x + u * kSymThreads;
                    const int row = e >> 5, vec = e & 31;
                    float acc = 0.f;
#pragma unroll
                    for (int w = 0; w < kSymWaves; ++w) acc += L.red[(w * kSymTile + row) * kSbRedLd + vec];
                    dst[e] = acc;                             // [row][vec]
                }
            }
        }
        // the owned partial: D[(r & 3) + 4 kh + 8 (r >> 2)][c] = O[col of the wave][vector c]
        float *dst = Op + int64_t(I.oslot) * (kSymCols * kBW);
#pragma unroll
        for (int r = 0; r < 16; ++r) dst[(32 * wave + (r & 3) + 4 * kh + 8 * (r >> 2)) * kBW + c] = O[r];
    }
}

// Row tile t of block J = t / 4: z = sum of the owned partials of J's items (item slots
// o_first[J] .. o_first[J + 1] - 1, in order) and of the forward partials (t, J') for
// J' = J + 1 .. NB - 1 (in order); Zf[vec][row] = z scale wrow[row] (z without wrow).
template <typename T>
__global__ __launch_bounds__(kThreads) void sym_reduce_kernel(const T *__restrict__ Fp, const T *__restrict__ Op,
                                                              const int *__restrict__ o_first, int NB,
                                                              int64_t Ntpad, const double *__restrict__ wrow,
                                                              double scale, T *__restrict__ Zf) {
    constexpr int kPer = (kSymTile * kBW) / kThreads;
    __shared__ T sm[kBW][kSymTile + 1];
    const int t = blockIdx.x, J = t >> 2, rt = t & 3;
    T acc[kPer];
#pragma unroll
    for (int u = 0; u < kPer; ++u) acc[u] = T(0);
    for (int o = o_first[J]; o < o_first[J + 1]; ++o) {
        const T *src = Op + int64_t(o) * (kSymCols * kBW) + rt * (kSymTile * kBW);
#pragma unroll
        for (int u = 0; u < kPer; ++u) acc[u] += src[threadIdx.x + u * kThreads];
    }
    int J2 = J + 1;
    for (; J2 + 1 < NB; J2 += 2) {                       // two slots' loads in flight
        const T *a = Fp + (int64_t(2) * J2 * (J2 - 1) + t) * (kSymTile * kBW);
        const T *b = Fp + (int64_t(2) * (J2 + 1) * J2 + t) * (kSymTile * kBW);
        T va[kPer], vb[kPer];
#pragma unroll
        for (int u = 0; u < kPer; ++u) { va[u] = a[threadIdx.x + u * kThreads]; vb[u] = b[threadIdx.x + u * kThreads]; }
#pragma unroll
        for (int u = 0; u < kPer; ++u) acc[u] = (acc[u] + va[u]) + vb[u];
    }
    if (J2 < NB) {
        const T *a = Fp + (int64_t(2) * J2 * (J2 - 1) + t) * (kSymTile * kBW);
#pragma unroll
        for (int u = 0; u < kPer; ++u) acc[u] += a[threadIdx.x + u * kThreads];
    }
#pragma unroll
    for (int u = 0; u < kPer; ++u) {
        const int e = threadIdx.x + u * kThreads;
        sm[e & 31][e >> 5] = acc[u];
    }
    __syncthreads();
    const int64_t row0 = int64_t(t) * kSymTile;
#pragma unroll
    for (int u = 0; u < kPer; ++u) {
        const int e = threadIdx.x + u * kThreads;
        const int vec = e >> 6, row = e & 63;
        const T v = sm[vec][row];
        Zf[int64_t(vec) * Ntpad + row0 + row] = wrow ? T(double(v) * scale * wrow[row0 + row]) : v;
    }
}

// ---- batched form: many problems, one persistent launch ------------------------------
// The grid holds as many workgroups as fit on the chip at once; each repeatedly takes
// the next (problem, row tile, split) item from a queue (a device counter) and runs the
// same skeleton on it.  Items are ordered longest first on the host, so the tail of the
// launch is made of short items.  Problems whose active flag is 0 are skipped.
__device__ __forceinline__ int next_item(int *counter, int *slot) {
    __syncthreads();
    if (threadIdx.x == 0) *slot = atomicAdd(counter, 1);
    __syncthreads();
    return __builtin_amdgcn_readfirstlane(*slot);
}

__device__ __forceinline__ S5Tile item_tile(const S5Prob &P, const S5Item &I, int64_t rows_wg) {
    S5Tile t;
    t.Ntpad = P.Ntpad;
    t.row0 = int64_t(I.rowtile) * rows_wg;
    t.l0 = int64_t(I.split) * P.lchunk;
    t.l1 = min(t.l0 + P.lchunk, P.Ntpad);
    t.split = I.split;
    t.nsplit = P.nsplit;
    t.wrow = P.wrow;
    t.scale = P.scale;
    return t;
}

template <int D, int RB>
__global__ __launch_bounds__(kThreads) void stage5_f32_batch_kernel(const S5Prob *__restrict__ probs,
                                                                    const S5Item *__restrict__ items, int n_items,
                                                                    int *__restrict__ counter,
                                                                    const int *__restrict__ active) {
    __shared__ float sX[D][kStep];
    __shared__ float sY[kLdsF32Y];
    __shared__ int slot;
    for (;;) {
        const int it = next_item(counter, &slot);
        if (it >= n_items) break;
        const S5Item I = items[it];
        if (active && active[I.prob] == 0) continue;
        const S5Prob P = probs[I.prob];
        const S5Tile t = item_tile(P, I, 32 * RB);
        const float *Y = static_cast<const float *>(P.Y5);
        float *Z = static_cast<float *>(P.Z5), *Zf = static_cast<float *>(P.Zf);
        switch (P.kind) {
        case KL_COV_EXP: stage5_f32_body<KL_COV_EXP, D, RB>(P.X32, Y, Z, Zf, t, sX, sY); break;
        case KL_COV_SQEXP: stage5_f32_body<KL_COV_SQEXP, D, RB>(P.X32, Y, Z, Zf, t, sX, sY); break;
        case KL_COV_EXP_L1: stage5_f32_body<KL_COV_EXP_L1, D, RB>(P.X32, Y, Z, Zf, t, sX, sY); break;
        case KL_COV_CONST: stage5_f32_body<KL_COV_CONST, D, RB>(P.X32, Y, Z, Zf, t, sX, sY); break;
        default: stage5_f32_body<KL_COV_LIN, D, RB>(P.X32, Y, Z, Zf, t, sX, sY); break;
        }
    }
}

template <int D>
__global__ __launch_bounds__(kThreads) void stage5_f64_batch_kernel(const S5Prob *__restrict__ probs,
                                                                    const S5Item *__restrict__ items, int n_items,
                                                                    int *__restrict__ counter,
                                                                    const int *__restrict__ active) {
    extern __shared__ double sm64[];
    __shared__ int slot;
    for (;;) {
        const int it = next_item(counter, &slot);
        if (it >= n_items) break;
        const S5Item I = items[it];
        if (active && active[I.prob] == 0) continue;
        const S5Prob P = probs[I.prob];
        const S5Tile t = item_tile(P, I, kRows);
        const double *Y = static_cast<const double *>(P.Y5);
        double *Z = static_cast<double *>(P.Z5), *Zf = static_cast<double *>(P.Zf);
        switch (P.kind) {
        case KL_COV_EXP: stage5_f64_body<KL_COV_EXP, D>(P.X64, Y, Z, Zf, t, sm64); break;
        case KL_COV_SQEXP: stage5_f64_body<KL_COV_SQEXP, D>(P.X64, Y, Z, Zf, t, sm64); break;
        case KL_COV_EXP_L1: stage5_f64_body<KL_COV_EXP_L1, D>(P.X64, Y, Z, Zf, t, sm64); break;
        case KL_COV_CONST: stage5_f64_body<KL_COV_CONST, D>(P.X64, Y, Z, Zf, t, sm64); break;
        default: stage5_f64_body<KL_COV_LIN, D>(P.X64, Y, Z, Zf, t, sm64); break;
        }
    }
}

__global__ void reset_counter_kernel(int *counter) {
    if (threadIdx.x == 0) counter[0] = 0;
}

// Split sums of all problems of a batch: global 4-entry index -> problem by binary search
// over the prefix `base4` (nprob + 1 entries), then as split_reduce_kernel.
template <typename T>
__global__ __launch_bounds__(kThreads) void split_reduce_batch_kernel(const RedProb *__restrict__ probs, int nprob,
                                                                      int64_t total4, const int *__restrict__ active) {
    const int64_t g4 = int64_t(blockIdx.x) * kThreads + threadIdx.x;
    if (g4 >= total4) return;
    int lo = 0, hi = nprob;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (probs[mid].base4 <= g4) lo = mid; else hi = mid;
    }
    const RedProb P = probs[lo];
    if (active && active[P.prob] == 0) return;
    const int64_t e4 = g4 - P.base4;
    const T *Zpart = static_cast<const T *>(P.Zpart);
    T acc[4] = {T(0), T(0), T(0), T(0)};
    for (int sp = 0; sp < P.nsplit; ++sp) {
        const T *src = Zpart + int64_t(sp) * P.stride + 4 * e4;
#pragma unroll
        for (int t = 0; t < 4; ++t) acc[t] += src[t];
    }
    T *Zf = static_cast<T *>(P.Zf);
    const int64_t row = (4 * e4) % P.Ntpad;
#pragma unroll
    for (int t = 0; t < 4; ++t) Zf[4 * e4 + t] = P.wrow ? T(double(acc[t]) * P.scale * P.wrow[row + t]) : acc[t];
}

template <int KIND, int D>
void launch_kind(int precision, const kl_problem *P, const void *Y5, void *Z5, void *Zf,
                 int nsplit, int64_t lchunk, int rb, const double *wrow, double scale, hipStream_t s) {
    const int64_t rows_wg = stage5_rows_per_wg(precision, rb);
    dim3 grid(unsigned(P->Ntpad / rows_wg), unsigned(nsplit));
    if (precision == KL_F64) {
        // once per process (thread-safe initialisation of a function-local static)
        static const bool attr_set = [] {
            (void)hipFuncSetAttribute(reinterpret_cast<const void *>(&stage5_f64_kernel<KIND, D>),
                                      hipFuncAttributeMaxDynamicSharedMemorySize, int(kLds64));
            return true;
        }();
        (void)attr_set;
        hipLaunchKernelGGL((stage5_f64_kernel<KIND, D>), grid, dim3(kThreads), kLds64, s,
                           P->dX64, static_cast<const double *>(Y5), static_cast<double *>(Z5),
                           static_cast<double *>(Zf), P->Ntpad, lchunk, wrow, scale);
    } else if (precision == KL_F32) {
#define KL_F32L(RB_) hipLaunchKernelGGL((stage5_f32_kernel<KIND, D, RB_>), grid, dim3(kThreads), 0, s, P->dX32, \
                                        static_cast<const float *>(Y5), static_cast<float *>(Z5),                 \
                                        static_cast<float *>(Zf), P->Ntpad, lchunk, wrow, scale)
        if (rb == 4) KL_F32L(4);
        else if (rb == 1) KL_F32L(1);
        else if (rb == 8)
            hipLaunchKernelGGL((stage5_f32_kernel<KIND, D, 2, 8>), grid, dim3(512), 0, s, P->dX32,
                               static_cast<const float *>(Y5), static_cast<float *>(Z5),
                               static_cast<float *>(Zf), P->Ntpad, lchunk, wrow, scale);
        else KL_F32L(2);
#undef KL_F32L
    } else {
        // BF16 operands: hi part at Y5, lo part right after it (Ntpad x kBW each)
        const __bf16 *yh = static_cast<const __bf16 *>(Y5);
        const __bf16 *yl = yh + P->Ntpad * kBW;
        float *z = static_cast<float *>(Z5), *zf = static_cast<float *>(Zf);
        const bool x3 = precision == KL_BF16X3;
#define KL_BF(RB_, X3_) hipLaunchKernelGGL((stage5_bf16_kernel<KIND, D, RB_, X3_>), grid, dim3(kThreads), \
                                           0, s, P->dX32, yh, yl, z, zf, P->Ntpad, lchunk, wrow, scale)
        if (rb == 4) { if (x3) KL_BF(4, true); else KL_BF(4, false); }
        else if (rb == 1) { if (x3) KL_BF(1, true); else KL_BF(1, false); }
        else { if (x3) KL_BF(2, true); else KL_BF(2, false); }
#undef KL_BF
    }
}

template <int D>
void launch_dim(int precision, const kl_problem *P, const void *Y5, void *Z5, void *Zf,
                int nsplit, int64_t lchunk, int rb, const double *wrow, double scale, hipStream_t s) {
    switch (P->cov_kind) {
    case KL_COV_EXP: launch_kind<KL_COV_EXP, D>(precision, P, Y5, Z5, Zf, nsplit, lchunk, rb, wrow, scale, s); break;
    case KL_COV_SQEXP: launch_kind<KL_COV_SQEXP, D>(precision, P, Y5, Z5, Zf, nsplit, lchunk, rb, wrow, scale, s); break;
    case KL_COV_EXP_L1: launch_kind<KL_COV_EXP_L1, D>(precision, P, Y5, Z5, Zf, nsplit, lchunk, rb, wrow, scale, s); break;
    case KL_COV_CONST: launch_kind<KL_COV_CONST, D>(precision, P, Y5, Z5, Zf, nsplit, lchunk, rb, wrow, scale, s); break;
    default: launch_kind<KL_COV_LIN, D>(precision, P, Y5, Z5, Zf, nsplit, lchunk, rb, wrow, scale, s); break;
    }
}

}  // namespace

// Rows owned by one stage-5 workgroup: 32 rb for the FP32 and BF16 kernels (rb = 8 is the
// FP32 form with two 32-row blocks per wave and 8 waves: 64 rows; BF16 treats it as 2),
// 64 for FP64.
int64_t stage5_rows_per_wg(int precision, int rb) {
    if (precision == KL_F64 || rb == 8) return 64;
    return 32 * rb;
}

// Number of l-splits.  Each workgroup has 4 waves; a split count S gives 4 R S waves
// (R = row tiles) over the 4 SIMDs of every CU.  S minimises the busiest SIMD's share,
// ceil(4 R S / SIMDs) / S, plus a small charge per split for the partial sums, among the
// counts that put at least 1.5 waves on every SIMD when that is possible.  `forced` > 0
// overrides the choice (autotuning).
int stage5_splits(int64_t Ntpad, int64_t rows_wg, int n_cu, int max_split, int forced,
                  int64_t *lchunk_out) {
    const int64_t R = Ntpad / rows_wg;
    const int64_t simds = 4 * int64_t(n_cu);
    const int64_t cap = std::max<int64_t>(1, std::min<int64_t>(max_split, Ntpad / kSub));
    int64_t best = 1;
    if (forced > 0) {
        best = std::min<int64_t>(forced, cap);
    } else {
        double best_cost = 1e300;
        bool any_full = false;
        for (int64_t S = 1; S <= cap; ++S) if (4 * R * S * 2 >= 3 * simds) { any_full = true; break; }
        for (int64_t S = 1; S <= cap; ++S) {
            const int64_t waves = 4 * R * S;
            if (any_full && waves * 2 < 3 * simds) continue;
            const double cost = double((waves + simds - 1) / simds) / double(S) + 0.01 * double(S);
            if (cost < best_cost - 1e-12) { best_cost = cost; best = S; }
        }
    }
    // the split length is a multiple of kSub = 64 and Ntpad one of kPad: every split covers a
    // multiple of 64 points, which the staging of the stage-5 bodies relies on
    static_assert(kSub == 64 && kPad % 64 == 0, "64-point split granule");
    int64_t lchunk = ((Ntpad + best - 1) / best + kSub - 1) / kSub * kSub;
    const int64_t nsplit = (Ntpad + lchunk - 1) / lchunk;
    if (lchunk_out) *lchunk_out = lchunk;
    return int(nsplit);
}

int launch_stage5(const kl_problem *P, int precision, const void *Y5, void *Z5, void *Zf,
                  const double *wrow, double scale, hipStream_t s, hipEvent_t ev_start, hipEvent_t ev_stop,
                  bool defer_reduce, int max_split) {
    const int rbs = P->s5_rb[precision];
    const int rb = (rbs == 1 || rbs == 4 || (rbs == 8 && precision == KL_F32)) ? rbs : 2;
    int64_t lchunk;
    const int nsplit = stage5_splits(P->Ntpad, stage5_rows_per_wg(precision, rb), P->n_cu,
                                     max_split > 0 ? max_split : P->ws.max_split, P->s5_split[precision], &lchunk);
    if (ev_start) (void)hipEventRecord(ev_start, s);
    switch (P->hs.d) {
    case 1: launch_dim<1>(precision, P, Y5, Z5, Zf, nsplit, lchunk, rb, wrow, scale, s); break;
    case 2: launch_dim<2>(precision, P, Y5, Z5, Zf, nsplit, lchunk, rb, wrow, scale, s); break;
    default: launch_dim<3>(precision, P, Y5, Z5, Zf, nsplit, lchunk, rb, wrow, scale, s); break;
    }
    if (ev_stop) (void)hipEventRecord(ev_stop, s);
    if (nsplit > 1 && !defer_reduce) {
        const int64_t n4 = P->Ntpad * kBW / 4;
        const dim3 g(unsigned((n4 + kThreads - 1) / kThreads));
        if (precision == KL_F64)
            hipLaunchKernelGGL(split_reduce_kernel<double>, g, dim3(kThreads), 0, s,
                               static_cast<const double *>(Z5), static_cast<double *>(Zf), nsplit, n4,
                               P->Ntpad * kBW, P->Ntpad, wrow, scale);
        else
            hipLaunchKernelGGL(split_reduce_kernel<float>, g, dim3(kThreads), 0, s,
                               static_cast<const float *>(Z5), static_cast<float *>(Zf), nsplit, n4,
                               P->Ntpad * kBW, P->Ntpad, wrow, scale);
    }
    return nsplit;
}

// ---- symmetric FP64 stage 5: plan and launch ---------------------------------------------
SymPlan sym_plan(int64_t Ntpad, int n_cu, int chunk) {
    SymPlan pl;
    pl.NB = int(Ntpad / kSymCols);
    const int64_t tiles = int64_t(2) * pl.NB * (pl.NB + 1);      // sum over J of 4 (J + 1)
    // about three items per compute unit unless forced
    pl.chunk = chunk > 0 ? chunk : int(std::max<int64_t>(1, (tiles + 3 * n_cu - 1) / (3 * int64_t(n_cu))));
    pl.o_first.assign(size_t(pl.NB) + 1, 0);
    int oslot = 0;
    for (int J = 0; J < pl.NB; ++J) {
        pl.o_first[J] = oslot;
        const int nt = 4 * (J + 1);
        for (int t0 = 0; t0 < nt; t0 += pl.chunk) pl.items.push_back(SymItem{J, t0, std::min(nt, t0 + pl.chunk), oslot++});
    }
    pl.o_first[pl.NB] = oslot;
    pl.n_oslots = oslot;
    pl.n_items = int(pl.items.size());
    pl.f_slots = int64_t(2) * pl.NB * (pl.NB - 1);
    std::stable_sort(pl.items.begin(), pl.items.end(),
                     [](const SymItem &a, const SymItem &b) { return a.t1 - a.t0 > b.t1 - b.t0; });
    return pl;
}

size_t sym_f_bytes(const SymPlan &pl) { return size_t(std::max<int64_t>(1, pl.f_slots)) * kSymTile * kBW * sizeof(double); }
size_t sym_o_bytes(const SymPlan &pl) { return size_t(pl.n_oslots) * kSymCols * kBW * sizeof(double); }

void launch_stage5_sym(const kl_problem *P, int precision, const Workspace &ws, const void *Y5,
                       const double *wrow, double scale, hipStream_t s, hipEvent_t ev_start, hipEvent_t ev_stop) {
    const SymItem *items = static_cast<const SymItem *>(ws.symTab);
    const int *o_first = reinterpret_cast<const int *>(items + ws.sym_items);
    const dim3 grid(unsigned(ws.sym_grid));
    if (ev_start) (void)hipEventRecord(ev_start, s);
    if (precision == KL_F64) {
        const double *Y = static_cast<const double *>(Y5);
#define KL_SYM(KIND_, D_)                                                                                    \
    do {                                                                                                     \
        static const bool attr_set = [] {                                                                    \
            (void)hipFuncSetAttribute(reinterpret_cast<const void *>(&stage5_f64_sym_kernel<KIND_, D_>),      \
                                      hipFuncAttributeMaxDynamicSharedMemorySize, int(kLdsSym));             \
            return true;                                                                                     \
        }();                                                                                                 \
        (void)attr_set;                                                                                      \
        hipLaunchKernelGGL((stage5_f64_sym_kernel<KIND_, D_>), grid, dim3(kSymThreads), kLdsSym, s, P->dX64, Y, \
                           P->Ntpad, items, ws.sym_items, ws.symF, ws.symO);                                 \
    } while (0)
#define KL_SYM_D(KIND_)                        \
    switch (P->hs.d) {                         \
    case 1: KL_SYM(KIND_, 1); break;           \
    case 2: KL_SYM(KIND_, 2); break;           \
    default: KL_SYM(KIND_, 3); break;          \
    }
        switch (P->cov_kind) {
        case KL_COV_EXP: KL_SYM_D(KL_COV_EXP); break;
        case KL_COV_SQEXP: KL_SYM_D(KL_COV_SQEXP); break;
        case KL_COV_EXP_L1: KL_SYM_D(KL_COV_EXP_L1); break;
        case KL_COV_CONST: KL_SYM_D(KL_COV_CONST); break;
        default: KL_SYM_D(KL_COV_LIN); break;
        }
#undef KL_SYM_D
#undef KL_SYM
        hipLaunchKernelGGL(sym_reduce_kernel<double>, dim3(unsigned(P->Ntpad / kSymTile)), dim3(kThreads), 0, s,
                           ws.symF, ws.symO, o_first, ws.sym_NB, P->Ntpad, wrow, scale, static_cast<double *>(ws.Zf));
    } else {
        // BF16 operands: hi part at Y5, lo part right after it (Ntpad x kBW each); FP32
        // partial sums in the same buffers
        const __bf16 *yh = static_cast<const __bf16 *>(Y5);
        const __bf16 *yl = yh + P->Ntpad * kBW;
        float *Fp = reinterpret_cast<float *>(ws.symF), *Op = reinterpret_cast<float *>(ws.symO);
#define KL_SYMB(KIND_, D_, X3_)                                                                              \
    do {                                                                                                     \
        constexpr size_t lds = sizeof(SymBf16Lds<X3_>);                                                       \
        static const bool attr_set = [] {                                                                    \
            (void)hipFuncSetAttribute(reinterpret_cast<const void *>(&stage5_bf16_sym_kernel<KIND_, D_, X3_>), \
                                      hipFuncAttributeMaxDynamicSharedMemorySize, int(lds));                 \
            return true;                                                                                     \
        }();                                                                                                 \
        (void)attr_set;                                                                                      \
        hipLaunchKernelGGL((stage5_bf16_sym_kernel<KIND_, D_, X3_>), grid, dim3(kSymThreads), lds, s, P->dX32, \
                           yh, yl, P->Ntpad, items, ws.sym_items, Fp, Op);                                   \
    } while (0)
#define KL_SYMB_X(KIND_, D_)                                       \
    if (precision == KL_BF16X3) KL_SYMB(KIND_, D_, true);          \
    else KL_SYMB(KIND_, D_, false);
#define KL_SYMB_D(KIND_)                       \
    switch (P->hs.d) {                         \
    case 1: KL_SYMB_X(KIND_, 1); break;        \
    case 2: KL_SYMB_X(KIND_, 2); break;        \
    default: KL_SYMB_X(KIND_, 3); break;       \
    }
        switch (P->cov_kind) {
        case KL_COV_EXP: KL_SYMB_D(KL_COV_EXP); break;
        case KL_COV_SQEXP: KL_SYMB_D(KL_COV_SQEXP); break;
        case KL_COV_EXP_L1: KL_SYMB_D(KL_COV_EXP_L1); break;
        case KL_COV_CONST: KL_SYMB_D(KL_COV_CONST); break;
        default: KL_SYMB_D(KL_COV_LIN); break;
        }
#undef KL_SYMB_D
#undef KL_SYMB_X
#undef KL_SYMB
        hipLaunchKernelGGL(sym_reduce_kernel<float>, dim3(unsigned(P->Ntpad / kSymTile)), dim3(kThreads), 0, s, Fp,
                           Op, o_first, ws.sym_NB, P->Ntpad, wrow, scale, static_cast<float *>(ws.Zf));
    }
    if (ev_stop) (void)hipEventRecord(ev_stop, s);
}

int stage5_batch_grid(int precision, int d, int rb, int n_cu) {
    int per_cu = 1;
    hipError_t e;
    const void *fn;
    size_t lds = 0;
    if (precision == KL_F64) {
        fn = d == 1 ? reinterpret_cast<const void *>(&stage5_f64_batch_kernel<1>)
           : d == 2 ? reinterpret_cast<const void *>(&stage5_f64_batch_kernel<2>)
                    : reinterpret_cast<const void *>(&stage5_f64_batch_kernel<3>);
        (void)hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, int(kLds64));
        lds = kLds64;
    } else if (rb == 4) {
        fn = d == 1 ? reinterpret_cast<const void *>(&stage5_f32_batch_kernel<1, 4>)
           : d == 2 ? reinterpret_cast<const void *>(&stage5_f32_batch_kernel<2, 4>)
                    : reinterpret_cast<const void *>(&stage5_f32_batch_kernel<3, 4>);
    } else {
        fn = d == 1 ? reinterpret_cast<const void *>(&stage5_f32_batch_kernel<1, 2>)
           : d == 2 ? reinterpret_cast<const void *>(&stage5_f32_batch_kernel<2, 2>)
                    : reinterpret_cast<const void *>(&stage5_f32_batch_kernel<3, 2>);
    }
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, kThreads, lds);
    if (e != hipSuccess || per_cu < 1) per_cu = 1;
    return per_cu * n_cu;
}

void launch_stage5_batch(int precision, int d, int rb, const S5Prob *probs, const S5Item *items, int n_items,
                         int *counter, const int *active, int grid, hipStream_t s) {
    hipLaunchKernelGGL(reset_counter_kernel, dim3(1), dim3(64), 0, s, counter);
    const dim3 g(unsigned(std::max(grid, 1)));
    if (precision == KL_F64) {
        if (d == 1) hipLaunchKernelGGL(stage5_f64_batch_kernel<1>, g, dim3(kThreads), kLds64, s, probs, items, n_items, counter, active);
        else if (d == 2) hipLaunchKernelGGL(stage5_f64_batch_kernel<2>, g, dim3(kThreads), kLds64, s, probs, items, n_items, counter, active);
        else hipLaunchKernelGGL(stage5_f64_batch_kernel<3>, g, dim3(kThreads), kLds64, s, probs, items, n_items, counter, active);
    } else if (rb == 4) {
        if (d == 1) hipLaunchKernelGGL((stage5_f32_batch_kernel<1, 4>), g, dim3(kThreads), 0, s, probs, items, n_items, counter, active);
        else if (d == 2) hipLaunchKernelGGL((stage5_f32_batch_kernel<2, 4>), g, dim3(kThreads), 0, s, probs, items, n_items, counter, active);
        else hipLaunchKernelGGL((stage5_f32_batch_kernel<3, 4>), g, dim3(kThreads), 0, s, probs, items, n_items, counter, active);
    } else {
        if (d == 1) hipLaunchKernelGGL((stage5_f32_batch_kernel<1, 2>), g, dim3(kThreads), 0, s, probs, items, n_items, counter, active);
        else if (d == 2) hipLaunchKernelGGL((stage5_f32_batch_kernel<2, 2>), g, dim3(kThreads), 0, s, probs, items, n_items, counter, active);
        else hipLaunchKernelGGL((stage5_f32_batch_kernel<3, 2>), g, dim3(kThreads), 0, s, probs, items, n_items, counter, active);
    }
}

void launch_split_reduce_batch(int precision, const RedProb *probs, int nprob, int64_t total4, const int *active,
                               hipStream_t s) {
    if (nprob < 1 || total4 < 1) return;
    const dim3 g(unsigned((total4 + kThreads - 1) / kThreads));
    if (precision == KL_F64)
        hipLaunchKernelGGL(split_reduce_batch_kernel<double>, g, dim3(kThreads), 0, s, probs, nprob, total4, active);
    else
        hipLaunchKernelGGL(split_reduce_batch_kernel<float>, g, dim3(kThreads), 0, s, probs, nprob, total4, active);
}

}  // namespace kl
