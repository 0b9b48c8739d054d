// Kernels of the warm-start network: FP32 GEMM on the matrix cores (a float4 form for
// aligned operands, a scalar-load form otherwise, and one thread per output for products
// of a few inputs) with fused bias / tanh / tanh-derivative / Adam epilogues, the
// sign-invariant loss and its subspace term, column sums for the bias gradients, Adam on
// the whole parameter vector or on parameter ranges, and a row gather for minibatches.
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

// Adam update of one parameter from its gradient g (every Adam path of the network goes
// through it, so fused and separate steps give the same bits: with contraction off, each
// product and sum rounds on its own wherever the function is inlined).  The bias
// corrections are multiplications by their reciprocals, the square root and the final
// reciprocal the hardware's (about 1 ulp each): a few vector instructions per parameter
// instead of three correctly rounded divisions and a square root, which matters where the
// update runs in a matrix product's epilogue.
__device__ __forceinline__ void adam_update(float &p, float &m, float &v, float g, const AdamArgs &a) {
#pragma clang fp contract(off)
    const float mi = a.b1 * m + (1.0f - a.b1) * g;
    const float vi = a.b2 * v + (1.0f - a.b2) * g * g;
    m = mi;
    v = vi;
    const float den = __builtin_amdgcn_sqrtf(vi * a.ic2) + a.eps;
    p -= a.lr * (mi * a.ic1) * __builtin_amdgcn_rcpf(den);
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

// Stores of a wave's 32 x 32 accumulator block: acc[r] of a lane is row
// rl + (r & 3) + 8 (r >> 2) of the column its pointer addresses (base at row rl); rows past
// M are skipped unless the tile is interior.  The epilogue kind is a template argument, so
// that the stores carry no per-element branching.
template <int EPI, bool INTERIOR>
__device__ __forceinline__ void store_block(float *base, int64_t ld, const float *aux, int64_t ldaux, float bj,
                                            int rl, int M, const floatx16 &acc) {
    const int64_t l2 = 2 * ld, l3 = 3 * ld, l8 = 8 * ld;
    const int64_t a2 = 2 * ldaux, a3 = 3 * ldaux, a8 = 8 * ldaux;
#pragma unroll
    for (int rg = 0; rg < 4; ++rg) {
#pragma unroll
        for (int rr = 0; rr < 4; ++rr) {
            if (!INTERIOR && rl + rr + 8 * rg >= M) continue;
            const int64_t off = rr == 0 ? 0 : rr == 1 ? ld : rr == 2 ? l2 : l3;
            float v = acc[4 * rg + rr];
            if (EPI == EPI_BIAS) v += bj;
            if (EPI == EPI_BIAS_TANH) v = tanhf(v + bj);
            if (EPI == EPI_DTANH) {
                const float h = aux[rr == 0 ? 0 : rr == 1 ? ldaux : rr == 2 ? a2 : a3];
                v *= 1.0f - h * h;
            }
            base[off] = v;
        }
        base += l8;
        if (EPI == EPI_DTANH) aux += a8;
    }
}

template <bool INTERIOR>
__device__ __forceinline__ void store_tile(const GemmArgs &g, int rl, int col, const floatx16 &acc) {
    if (gridDim.z > 1) {
        store_block<EPI_NONE, INTERIOR>(g.part + (int64_t(blockIdx.z) * g.M + rl) * g.N + col, g.N, nullptr, 0,
                                        0.0f, rl, g.M, acc);
        return;
    }
    float *c = g.C + int64_t(rl) * g.ldc + col;
    switch (g.epi) {
    case EPI_BIAS: store_block<EPI_BIAS, INTERIOR>(c, g.ldc, nullptr, 0, g.bias[col], rl, g.M, acc); break;
    case EPI_BIAS_TANH:
        store_block<EPI_BIAS_TANH, INTERIOR>(c, g.ldc, nullptr, 0, g.bias[col], rl, g.M, acc);
        break;
    case EPI_DTANH:
        store_block<EPI_DTANH, INTERIOR>(c, g.ldc, g.aux + int64_t(rl) * g.ldaux + col, g.ldaux, 0.0f, rl, g.M,
                                         acc);
        break;
    default: store_block<EPI_NONE, INTERIOR>(c, g.ldc, nullptr, 0, 0.0f, rl, g.M, acc); break;
    }
}

// The same product for operands whose contiguous index runs in whole float4s (16-byte
// aligned bases, leading dimensions and contiguous extents multiples of 4; gemm_vec_ok).
// 64 x 64 tiles with 64-deep K chunks, staged in LDS with k contiguous (sA[i][k], sB[j][k];
// rows padded to 68 floats, so the 16 lanes served together by a 128-bit LDS read fall on
// distinct banks).  Within a chunk, MFMA step s takes k = s from the lower half-wave and
// k = 32 + s from the upper one, so a lane reads its 32 operands of the chunk as eight
// 128-bit LDS loads; every term is added as in gemm_f32_kernel, in another order.  Global
// loads are one float4 per thread and operand row, eight per thread and chunk, with the
// next chunk prefetched into registers while the current one is consumed.
// An operand whose contiguous index is not k (A when TA, B unless TB) reaches LDS as four
// scalar writes per float4; in its rows the float4 group k/4 is stored at
// (k/4) ^ ((row/16) & 3), which spreads a wave's scalar writes over all 64 banks (four-way
// conflicts otherwise) and leaves the 128-bit reads conflict-free.
// ADAM (EPI_ADAM, one K range): the accumulators are gradients of the parameters at C
// (moments at am, av, same layout); the lane's 16 parameters and their moments are loaded
// right after the first operand chunk, so that they arrive during the products, and the
// updated values are stored in place of the tile.
constexpr int kVK = 64, kVS = kVK + 4;

// Column sums (g.colsum, TA and not TB): the workgroups of the first row tile add the 64
// entries of each column of every staged B chunk, wave q taking the chunk's physical
// positions 16 q .. 16 q + 15 of the column's LDS row, and the four quarter sums in wave
// order, chunk after chunk.
template <bool TA, bool TB, bool ADAM = false>
__global__ __launch_bounds__(kThreads) void gemm_f32_vec_kernel(GemmArgs g) {
    __shared__ float4 sA[kTM * kVS / 4];
    __shared__ float4 sB[kTN * kVS / 4];
    __shared__ float cs[TA && !TB ? 4 : 1][64];
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    const int i0 = blockIdx.y * kTM, j0 = blockIdx.x * kTN;
    const int kb = blockIdx.z * g.kchunk;
    const int ke = min(g.K, kb + g.kchunk);
    const int wi = (w >> 1) * 32, wj = (w & 1) * 32;
    // float4 number r * 256 + t of a 64 x 64 operand tile: c4 = t & 15 counts float4s along
    // the contiguous index, o + 16 r (o = t >> 4) is the other index.
    const int c4 = t & 15, o = t >> 4;
    // Per-thread bases at k = 0 and row / column o; A(r) and B(r) add 16 r rows, the chunk
    // start adds kc along k.
    const float *baseA = TA ? g.A + int64_t(o) * g.lda + i0 + 4 * c4 : g.A + int64_t(i0 + o) * g.lda + 4 * c4;
    const float *baseB = TB ? g.B + int64_t(j0 + o) * g.ldb + 4 * c4 : g.B + int64_t(o) * g.ldb + j0 + 4 * c4;
    const int64_t rowA = 16 * g.lda, rowB = 16 * g.ldb;
    const bool colA = !TA || i0 + 4 * c4 < g.M;   // contiguous index in range (i for TA)
    const bool colB = TB || j0 + 4 * c4 < g.N;    // contiguous index in range (j unless TB)
    floatx16 acc;
    for (int r = 0; r < 16; ++r) acc[r] = 0.0f;
    float4 ra[4], rb[4];
    auto load = [&](int kc) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int other = o + 16 * r;
            const bool va = TA ? (colA && kc + other < ke) : (i0 + other < g.M && kc + 4 * c4 < ke);
            const bool vb = TB ? (j0 + other < g.N && kc + 4 * c4 < ke) : (colB && kc + other < ke);
            const float *pa = baseA + r * rowA + (TA ? int64_t(kc) * g.lda : int64_t(kc));
            const float *pb = baseB + r * rowB + (TB ? int64_t(kc) : int64_t(kc) * g.ldb);
            ra[r] = va ? *reinterpret_cast<const float4 *>(pa) : make_float4(0.0f, 0.0f, 0.0f, 0.0f);
            rb[r] = vb ? *reinterpret_cast<const float4 *>(pb) : make_float4(0.0f, 0.0f, 0.0f, 0.0f);
        }
    };
    // scalar writes of float4 rows 4 c4 .. 4 c4 + 3 at k = other (swizzle (4 c4 / 16) & 3)
    auto put_t = [&](float *f, const float4 &v, int other) {
        const int at = 4 * ((other >> 2) ^ (c4 >> 2)) + (other & 3);
        f[(4 * c4 + 0) * kVS + at] = v.x;
        f[(4 * c4 + 1) * kVS + at] = v.y;
        f[(4 * c4 + 2) * kVS + at] = v.z;
        f[(4 * c4 + 3) * kVS + at] = v.w;
    };
    auto store = [&]() {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int other = o + 16 * r;
            if (TA) put_t(reinterpret_cast<float *>(sA), ra[r], other);   // ra[r] = A(4 c4.., other)
            else sA[other * (kVS / 4) + c4] = ra[r];                     // ra[r] = A(other, 4 c4..)
            if (TB) sB[other * (kVS / 4) + c4] = rb[r];                  // rb[r] = B(4 c4.., other)
            else put_t(reinterpret_cast<float *>(sB), rb[r], other);     // rb[r] = B(other, 4 c4..)
        }
    };
    // LDS read pointers: group s4 = 4 q + p of the lane's half sits at p ^ sw in a swizzled row
    const int ra_row = wi + (lane & 31), rb_row = wj + (lane & 31);
    const int swa = TA ? (ra_row >> 4) & 3 : 0, swb = TB ? 0 : (rb_row >> 4) & 3;
    const float4 *la[4], *lb[4];
#pragma unroll
    for (int p = 0; p < 4; ++p) {
        la[p] = sA + ra_row * (kVS / 4) + 8 * (lane >> 5) + (p ^ swa);
        lb[p] = sB + rb_row * (kVS / 4) + 8 * (lane >> 5) + (p ^ swb);
    }
    if (kb < ke) load(kb);
    // ADAM: acc[r] of the lane belongs to row rl + (r & 3) + 8 (r >> 2) of column col
    const int col = j0 + wj + (lane & 31);
    const int rl = i0 + wi + 4 * (lane >> 5);
    float pp[ADAM ? 16 : 1], mm[ADAM ? 16 : 1], vv[ADAM ? 16 : 1];
    if constexpr (ADAM) {
        const int64_t o = int64_t(rl) * g.ldc + min(col, g.N - 1);
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const int dr = (r & 3) + 8 * (r >> 2);
            const int64_t off = o + int64_t(min(dr, g.M - 1 - rl)) * g.ldc;   // clamped: rows past M
            pp[r] = g.C[off];
            mm[r] = g.am[off];
            vv[r] = g.av[off];
        }
    }
    const bool do_cs = TA && !TB && g.colsum != nullptr && blockIdx.y == 0;   // uniform
    float csum = 0.0f;
    for (int kc = kb; kc < ke; kc += kVK) {
        __syncthreads();
        store();
        __syncthreads();
        if (kc + kVK < ke) load(kc + kVK);
        if constexpr (TA && !TB) {
            if (do_cs) {
                const float *row = reinterpret_cast<const float *>(sB) + (t & 63) * kVS + 16 * w;
                float part = 0.0f;
#pragma unroll
                for (int u = 0; u < 16; ++u) part += row[u];
                cs[w][t & 63] = part;
                __syncthreads();
                if (t < 64) csum += ((cs[0][t] + cs[1][t]) + cs[2][t]) + cs[3][t];
            }
        }
#pragma unroll
        for (int q = 0; q < 2; ++q) {
#pragma unroll
            for (int p = 0; p < 4; ++p) {
                const float4 a = la[p][4 * q], b = lb[p][4 * q];
                acc = __builtin_amdgcn_mfma_f32_32x32x2f32(a.x, b.x, acc, 0, 0, 0);
                acc = __builtin_amdgcn_mfma_f32_32x32x2f32(a.y, b.y, acc, 0, 0, 0);
                acc = __builtin_amdgcn_mfma_f32_32x32x2f32(a.z, b.z, acc, 0, 0, 0);
                acc = __builtin_amdgcn_mfma_f32_32x32x2f32(a.w, b.w, acc, 0, 0, 0);
            }
        }
    }
    if (do_cs && t < 64 && j0 + t < g.N) {
        const int j = j0 + t;
        if (g.epi == EPI_ADAM) {
            float pb = g.colsum[j], mb = g.bm[j], vb = g.bv[j];
            adam_update(pb, mb, vb, csum, g.adam);
            g.colsum[j] = pb;
            g.bm[j] = mb;
            g.bv[j] = vb;
        } else {
            g.colsum[j] = csum;
        }
    }
    if (col >= g.N) return;
    if constexpr (ADAM) {
        const int64_t o = int64_t(rl) * g.ldc + col;
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const int dr = (r & 3) + 8 * (r >> 2);
            if (rl + dr >= g.M) continue;
            adam_update(pp[r], mm[r], vv[r], acc[r], g.adam);
            const int64_t off = o + int64_t(dr) * g.ldc;
            g.C[off] = pp[r];
            g.am[off] = mm[r];
            g.av[off] = vv[r];
        }
        return;
    }
    if (i0 + kTM <= g.M) store_tile<true>(g, rl, col, acc);
    else store_tile<false>(g, rl, col, acc);
}

// Products with a fan-in of at most kDirectK and at most kDirectOut outputs (the first
// layer of a network on a few inputs): one thread per output, the K terms added in order
// in FP32, then the epilogue.  64 x 64 matrix tiles would leave these launches to a
// handful of workgroups (7.3 against 4.0 us for 64 x 3 by 3 x 256); longer fan-ins and
// larger outputs stay on the matrix cores.
template <bool TA, bool TB>
__global__ __launch_bounds__(kThreads) void gemm_direct_kernel(GemmArgs g) {
    const int64_t e = int64_t(blockIdx.x) * kThreads + threadIdx.x;
    if (e >= int64_t(g.M) * g.N) return;
    const int i = int(e / g.N), j = int(e - int64_t(i) * g.N);
    float acc = 0.0f;
    for (int k = 0; k < g.K; ++k) {
        const float a = TA ? g.A[int64_t(k) * g.lda + i] : g.A[int64_t(i) * g.lda + k];
        const float b = TB ? g.B[int64_t(j) * g.ldb + k] : g.B[int64_t(k) * g.ldb + j];
        acc = fmaf(a, b, acc);
    }
    g.C[int64_t(i) * g.ldc + j] = epilogue(g, i, j, acc);
}

// Sum of the K-range partials in a fixed order, then the epilogue: a workgroup takes 64
// output elements, wave w adds the w-th quarter of the partials of its lane's element in
// split order (loads issued eight at a time), and the quarter sums are added in wave order
// through LDS.
__global__ __launch_bounds__(256) void splitk_reduce_kernel(GemmArgs g, int splits) {
    __shared__ float qs[4][64];
    const int64_t total = int64_t(g.M) * g.N;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int64_t e = int64_t(blockIdx.x) * 64 + lane;
    const int64_t ec = min(e, total - 1);               // lanes past the end read the last element
    const int s0 = (splits * w) / 4, s1 = (splits * (w + 1)) / 4;
    float v = 0.0f;
    int sp = s0;
    for (; sp + 8 <= s1; sp += 8) {
        float t[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) t[u] = g.part[int64_t(sp + u) * total + ec];
#pragma unroll
        for (int u = 0; u < 8; ++u) v += t[u];
    }
    for (; sp < s1; ++sp) v += g.part[int64_t(sp) * total + ec];
    qs[w][lane] = v;
    __syncthreads();
    if (w == 0 && e < total) {
        const float sum = ((qs[0][lane] + qs[1][lane]) + qs[2][lane]) + qs[3][lane];
        const int row = int(e / g.N), col = int(e % g.N);
        g.C[int64_t(row) * g.ldc + col] = epilogue(g, row, col, sum);
    }
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

// Sign-invariant loss, one workgroup per (group, sample): with y_g and t_g the group's
// output and target, s = +1 if <y_g, t_g> >= 0 else -1 (dot accumulated in FP64);
// dy_g = (y_g - s t_g) * inv_b and loss_part = 0.5 ||y_g - s t_g||^2 (FP64).
// signed_ == 0 keeps s = +1 (plain squared error).
// Groups of up to kLossRegs * kThreads elements are read once into registers (all loads
// issued together, clamped into the group and masked where used); longer groups are read
// twice.  Both sums use block_sum.
constexpr int kLossRegs = 16;

__global__ __launch_bounds__(kThreads) void loss_kernel(const float *__restrict__ y, int64_t ldy,
                                                        const float *__restrict__ tgt, int64_t ldt,
                                                        const int *__restrict__ rows, int group,
                                                        int signed_, float inv_b, float *__restrict__ dy,
                                                        int64_t lddy, double *__restrict__ loss_part) {
    const int gi = blockIdx.x, s = blockIdx.y;
    const float *yr = y + int64_t(s) * ldy + int64_t(gi) * group;
    const int trow = rows ? rows[s] : s;
    const float *tr = tgt + int64_t(trow) * ldt + int64_t(gi) * group;
    float *dr = dy + int64_t(s) * lddy + int64_t(gi) * group;
    __shared__ double red[kThreads / 64];
    const int t0 = threadIdx.x;
    const bool cached = group <= kLossRegs * kThreads;
    float yv[kLossRegs], tv[kLossRegs];
    if (cached) {
#pragma unroll
        for (int u = 0; u < kLossRegs; ++u) {
            const int i = min(t0 + u * kThreads, group - 1);
            yv[u] = yr[i];
            tv[u] = tr[i];
        }
    }
    float sg = 1.0f;
    if (signed_) {
        double dot = 0.0;
        if (cached) {
#pragma unroll
            for (int u = 0; u < kLossRegs; ++u)
                if (t0 + u * kThreads < group) dot += double(yv[u]) * double(tv[u]);
        } else {
            for (int i = t0; i < group; i += kThreads) dot += double(yr[i]) * double(tr[i]);
        }
        sg = block_sum(dot, red) >= 0.0 ? 1.0f : -1.0f;
    }
    double l2 = 0.0;
    if (cached) {
#pragma unroll
        for (int u = 0; u < kLossRegs; ++u) {
            const int i = t0 + u * kThreads;
            if (i < group) {
                const float e = yv[u] - sg * tv[u];
                dr[i] = e * inv_b;
                l2 += double(e) * double(e);
            }
        }
    } else {
        for (int i = t0; i < group; i += kThreads) {
            const float e = yr[i] - sg * tr[i];
            dr[i] = e * inv_b;
            l2 += double(e) * double(e);
        }
    }
    l2 = block_sum(l2, red);
    if (t0 == 0) loss_part[int64_t(s) * gridDim.x + gi] = 0.5 * l2;
}

// Subspace term of the loss in three passes (after loss_kernel on the same stream).  With
// y_a the sample's output groups and t_b its target groups (a, b < ng):
//   gram:     per slice of the group index, the FP64 sums <y_a, t_b> and <t_b, t_b>;
//   coef:     per sample, the slices summed in order, c_ab = <y_a, t_b> / <t_b, t_b>;
//   residual: r_a = y_a - sum_b c_ab t_b (the part of y_a outside the span of orthogonal
//             targets), dy += w inv_b r_a and loss_part += 0.5 w ||r_a||^2.
// Every output and target element is read once per pass.
constexpr int kSubChunk = 128;    // group elements staged in LDS per step of the gram pass
constexpr int kSubSlices = 32;    // at most this many gram workgroups per sample
constexpr int kSubPairs = (kMaxSubGroups * (kMaxSubGroups + 1) + kThreads - 1) / kThreads;

int sub_slices(int group) { return std::min(kSubSlices, (group + kSubChunk - 1) / kSubChunk); }

// part[(s ns + sl) P + q], P = ng^2 + ng: q < ng^2 holds <y_a, t_b> (a = q / ng, b = q % ng),
// q = ng^2 + b holds <t_b, t_b>; workgroup sl sums the chunks sl, sl + ns, ... of the group.
__global__ __launch_bounds__(kThreads) void subspace_gram_kernel(const float *__restrict__ y, int64_t ldy,
                                                                 const float *__restrict__ tgt, int64_t ldt,
                                                                 const int *__restrict__ rows, int group, int ng,
                                                                 double *__restrict__ part) {
    const int sl = blockIdx.x, ns = gridDim.x, s = blockIdx.y;
    const float *yr = y + int64_t(s) * ldy;
    const float *tr = tgt + int64_t(rows ? rows[s] : s) * ldt;
    // rows 0..ng-1: the output groups, rows kMaxSubGroups + b: the target groups
    __shared__ float sb[2 * kMaxSubGroups][kSubChunk + 1];
    const int nn = ng * ng, P = nn + ng;
    int ru[kSubPairs], rv[kSubPairs];
#pragma unroll
    for (int k = 0; k < kSubPairs; ++k) {
        const int q = threadIdx.x + k * kThreads;
        ru[k] = q < nn ? q / ng : kMaxSubGroups + (q - nn);
        rv[k] = kMaxSubGroups + (q < nn ? q % ng : q - nn);
    }
    double acc[kSubPairs];
#pragma unroll
    for (int k = 0; k < kSubPairs; ++k) acc[k] = 0.0;
    for (int c0 = sl * kSubChunk; c0 < group; c0 += ns * kSubChunk) {
        const int len = min(kSubChunk, group - c0);
        // all loads of the chunk are issued before the LDS stores
        constexpr int kRowsPer = kThreads / kSubChunk;
        const int a0 = threadIdx.x / kSubChunk, i = threadIdx.x % kSubChunk;
        float vy[kMaxSubGroups / kRowsPer], vt[kMaxSubGroups / kRowsPer];
#pragma unroll
        for (int k = 0; k < kMaxSubGroups / kRowsPer; ++k) {
            const int a = a0 + k * kRowsPer;
            const bool in = a < ng && i < len;
            const int64_t g = int64_t(a) * group + c0 + i;
            vy[k] = in ? yr[g] : 0.0f;
            vt[k] = in ? tr[g] : 0.0f;
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < kMaxSubGroups / kRowsPer; ++k) {
            const int a = a0 + k * kRowsPer;
            if (a < ng) {
                sb[a][i] = vy[k];
                sb[kMaxSubGroups + a][i] = vt[k];
            }
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < kSubPairs; ++k)
            if (threadIdx.x + k * kThreads < P) {
                double d = 0.0;
#pragma unroll 8
                for (int i = 0; i < kSubChunk; ++i) d += double(sb[ru[k]][i]) * double(sb[rv[k]][i]);
                acc[k] += d;
            }
    }
#pragma unroll
    for (int k = 0; k < kSubPairs; ++k) {
        const int q = threadIdx.x + k * kThreads;
        if (q < P) part[(int64_t(s) * ns + sl) * P + q] = acc[k];
    }
}

// coef[s ng^2 + a ng + b] = c_ab from the ns slices of the gram pass (0 for a zero target).
__global__ __launch_bounds__(kThreads) void subspace_coef_kernel(const double *__restrict__ part, int ns, int ng,
                                                                 double *__restrict__ coef) {
    const int s = blockIdx.x, nn = ng * ng, P = nn + ng;
    for (int q = threadIdx.x; q < nn; q += kThreads) {
        const int b = q % ng;
        double c = 0.0, n = 0.0;
        // the loads of eight slices are issued together; the sums stay in slice order
#pragma unroll 8
        for (int sl = 0; sl < ns; ++sl) {
            const double *p = part + (int64_t(s) * ns + sl) * P;
            c += p[q];
            n += p[nn + b];
        }
        coef[int64_t(s) * nn + q] = n > 0.0 ? c / n : 0.0;
    }
}

// One workgroup per (slice of the group index, sample), gridDim.x = ng slices; each thread
// loads the ng outputs, targets and deltas of its element first and keeps the ng residuals in
// registers (MG >= ng).
template <int MG>
__global__ __launch_bounds__(kThreads) void subspace_residual_kernel(const float *__restrict__ y, int64_t ldy,
                                                                     const float *__restrict__ tgt, int64_t ldt,
                                                                     const int *__restrict__ rows, int group, int ng,
                                                                     const double *__restrict__ coef, float w,
                                                                     float inv_b, float *__restrict__ dy,
                                                                     int64_t lddy, double *__restrict__ loss_part) {
    const int sl = blockIdx.x, s = blockIdx.y;
    const float *yr = y + int64_t(s) * ldy;
    const float *tr = tgt + int64_t(rows ? rows[s] : s) * ldt;
    float *dr = dy + int64_t(s) * lddy;
    __shared__ double cf[MG][MG];
    __shared__ double red[kThreads / 64];
    for (int q = threadIdx.x; q < ng * ng; q += kThreads) cf[q / ng][q % ng] = coef[int64_t(s) * ng * ng + q];
    __syncthreads();
    const int len = (group + ng - 1) / ng;
    const int i0 = sl * len, i1 = min(group, i0 + len);
    const float sc = w * inv_b;
    double l2 = 0.0;
    for (int i = i0 + int(threadIdx.x); i < i1; i += kThreads) {
        float yv[MG], tv[MG], dv[MG];
#pragma unroll
        for (int a = 0; a < MG; ++a) {
            yv[a] = a < ng ? yr[int64_t(a) * group + i] : 0.0f;
            tv[a] = a < ng ? tr[int64_t(a) * group + i] : 0.0f;
            dv[a] = a < ng ? dr[int64_t(a) * group + i] : 0.0f;
        }
#pragma unroll
        for (int a = 0; a < MG; ++a) {
            if (a >= ng) break;
            double r = yv[a];
#pragma unroll
            for (int b = 0; b < MG; ++b)
                if (b < ng) r -= double(tv[b]) * cf[a][b];
            dr[int64_t(a) * group + i] = dv[a] + sc * float(r);
            l2 += r * r;
        }
    }
    const double tot = block_sum(l2, red);
    if (threadIdx.x == 0) loss_part[int64_t(s) * gridDim.x + sl] += 0.5 * double(w) * tot;
}

// db[j] = sum_i D[i][j] over M rows: a workgroup takes 64 columns, wave w adds the w-th
// quarter of the rows for its lane's column (loads issued eight at a time), and the four
// quarter sums are added in wave order through LDS (a fixed order: the same bits every call).
__global__ __launch_bounds__(256) void colsum_kernel(const float *__restrict__ D, int64_t ldd, int M, int N,
                                                     float *__restrict__ out) {
    __shared__ float part[4][64];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int j = int(blockIdx.x) * 64 + lane;
    const int jc = min(j, N - 1);                        // lanes past N read column N - 1, store nothing
    const int r0 = (M * w) / 4, r1 = (M * (w + 1)) / 4;
    float s = 0.0f;
    int i = r0;
    for (; i + 8 <= r1; i += 8) {
        float v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) v[u] = D[int64_t(i + u) * ldd + jc];
#pragma unroll
        for (int u = 0; u < 8; ++u) s += v[u];
    }
    for (; i < r1; ++i) s += D[int64_t(i) * ldd + jc];
    part[w][lane] = s;
    __syncthreads();
    if (w == 0 && j < N) out[j] = ((part[0][lane] + part[1][lane]) + part[2][lane]) + part[3][lane];
}

// Adam with bias correction: m = b1 m + (1 - b1) g, v = b2 v + (1 - b2) g^2,
// p -= lr (m / c1) / (sqrt(v / c2) + eps), c1 = 1 - b1^t, c2 = 1 - b2^t.
__global__ __launch_bounds__(kThreads) void adam_kernel(float *__restrict__ p, const float *__restrict__ g,
                                                        float *__restrict__ m, float *__restrict__ v,
                                                        int64_t n, AdamArgs a) {
    for (int64_t i = int64_t(blockIdx.x) * kThreads + threadIdx.x; i < n; i += int64_t(gridDim.x) * kThreads) {
        float pi = p[i], mi = m[i], vi = v[i];
        adam_update(pi, mi, vi, g[i], a);
        p[i] = pi;
        m[i] = mi;
        v[i] = vi;
    }
}

// The same step on the parameter ranges of r (the parameters whose update did not run in
// a product's epilogue): element e of the concatenated ranges is parameter
// off[k] + e - end[k - 1] for the first k with e < end[k].
__global__ __launch_bounds__(kThreads) void adam_ranges_kernel(float *__restrict__ p, const float *__restrict__ g,
                                                               float *__restrict__ m, float *__restrict__ v,
                                                               AdamRanges r, AdamArgs a) {
    const int64_t total = r.end[r.n - 1];
    for (int64_t e = int64_t(blockIdx.x) * kThreads + threadIdx.x; e < total; e += int64_t(gridDim.x) * kThreads) {
        int k = 0;
        while (e >= r.end[k]) ++k;
        const int64_t i = r.off[k] + (e - (k ? r.end[k - 1] : 0));
        float pi = p[i], mi = m[i], vi = v[i];
        adam_update(pi, mi, vi, g[i], a);
        p[i] = pi;
        m[i] = mi;
        v[i] = vi;
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

bool gemm_vec_ok(bool ta, bool tb, const GemmArgs &g) {
    auto aligned = [](const void *p) { return (reinterpret_cast<uintptr_t>(p) & 15) == 0; };
    if (!aligned(g.A) || !aligned(g.B) || (g.lda & 3) || (g.ldb & 3)) return false;
    return ((ta ? g.M : g.K) & 3) == 0 && ((tb ? g.K : g.N) & 3) == 0;
}

int gemm_splits(int M, int N, int K, int n_cu, int64_t part_cap, bool vec, int *kchunk) {
    const int kstep = vec ? kVK : kTK;
    const int64_t tiles = int64_t((M + kTM - 1) / kTM) * ((N + kTN - 1) / kTN);
    const int ksteps = std::max(1, (K + kstep - 1) / kstep);
    int splits = 1;
    const int64_t want = 2 * int64_t(n_cu);
    if (tiles < want) splits = int(std::min<int64_t>(ksteps, (want + tiles - 1) / tiles));
    while (splits > 1 && int64_t(splits) * M * N > part_cap) --splits;
    const int steps_per = (ksteps + splits - 1) / splits;
    *kchunk = steps_per * kstep;
    return (ksteps + steps_per - 1) / steps_per;
}

bool gemm_direct_ok(const GemmArgs &g) {
    return g.epi != EPI_ADAM && g.K <= kDirectK && int64_t(g.M) * g.N <= kDirectOut;
}

void launch_gemm_direct(bool ta, bool tb, const GemmArgs &g, hipStream_t s) {
    const int64_t n = int64_t(g.M) * g.N;
    if (n < 1) return;
    const dim3 grid(unsigned((n + kThreads - 1) / kThreads));
    if (ta && tb) hipLaunchKernelGGL((gemm_direct_kernel<true, true>), grid, dim3(kThreads), 0, s, g);
    else if (ta) hipLaunchKernelGGL((gemm_direct_kernel<true, false>), grid, dim3(kThreads), 0, s, g);
    else if (tb) hipLaunchKernelGGL((gemm_direct_kernel<false, true>), grid, dim3(kThreads), 0, s, g);
    else hipLaunchKernelGGL((gemm_direct_kernel<false, false>), grid, dim3(kThreads), 0, s, g);
}

void launch_gemm(bool ta, bool tb, bool vec, GemmArgs g, int splits, hipStream_t s) {
    const dim3 grid((g.N + kTN - 1) / kTN, (g.M + kTM - 1) / kTM, splits);
    if (vec && g.epi == EPI_ADAM) {   // the weight gradient h^T D (TA, not TB), one K range
        hipLaunchKernelGGL((gemm_f32_vec_kernel<true, false, true>), grid, dim3(kThreads), 0, s, g);
        return;
    }
    if (vec) {
        if (ta && tb) hipLaunchKernelGGL((gemm_f32_vec_kernel<true, true>), grid, dim3(kThreads), 0, s, g);
        else if (ta) hipLaunchKernelGGL((gemm_f32_vec_kernel<true, false>), grid, dim3(kThreads), 0, s, g);
        else if (tb) hipLaunchKernelGGL((gemm_f32_vec_kernel<false, true>), grid, dim3(kThreads), 0, s, g);
        else hipLaunchKernelGGL((gemm_f32_vec_kernel<false, false>), grid, dim3(kThreads), 0, s, g);
    } else if (ta && tb) hipLaunchKernelGGL((gemm_f32_kernel<true, true>), grid, dim3(kThreads), 0, s, g);
    else if (ta) hipLaunchKernelGGL((gemm_f32_kernel<true, false>), grid, dim3(kThreads), 0, s, g);
    else if (tb) hipLaunchKernelGGL((gemm_f32_kernel<false, true>), grid, dim3(kThreads), 0, s, g);
    else hipLaunchKernelGGL((gemm_f32_kernel<false, false>), grid, dim3(kThreads), 0, s, g);
    if (splits > 1)
        hipLaunchKernelGGL(splitk_reduce_kernel, dim3(unsigned((int64_t(g.M) * g.N + 63) / 64)), dim3(256), 0, s,
                           g, splits);
}

void launch_loss(const float *y, int64_t ldy, const float *t, int64_t ldt, const int *rows, int batch,
                 int n_out, int group, int signed_, float *dy, int64_t lddy, double *loss_part,
                 hipStream_t s) {
    const int ng = n_out / group;
    hipLaunchKernelGGL(loss_kernel, dim3(ng, batch), dim3(kThreads), 0, s, y, ldy, t, ldt, rows, group, signed_,
                       1.0f / float(batch), dy, lddy, loss_part);
}

int64_t subspace_scratch(int batch, int n_out, int group) {
    const int ng = n_out / group;
    return int64_t(batch) * (int64_t(sub_slices(group)) * (ng * ng + ng) + ng * ng);
}

void launch_subspace(const float *y, int64_t ldy, const float *t, int64_t ldt, const int *rows, int batch,
                     int n_out, int group, float weight, float *dy, int64_t lddy, double *loss_part,
                     double *scratch, hipStream_t s) {
    const int ng = n_out / group, ns = sub_slices(group);
    double *part = scratch, *coef = scratch + int64_t(batch) * ns * (ng * ng + ng);
    hipLaunchKernelGGL(subspace_gram_kernel, dim3(ns, batch), dim3(kThreads), 0, s, y, ldy, t, ldt, rows, group, ng,
                       part);
    hipLaunchKernelGGL(subspace_coef_kernel, dim3(batch), dim3(kThreads), 0, s, part, ns, ng, coef);
    const dim3 grid(ng, batch);
    const float inv_b = 1.0f / float(batch);
    if (ng <= 4)
        hipLaunchKernelGGL(subspace_residual_kernel<4>, grid, dim3(kThreads), 0, s, y, ldy, t, ldt, rows, group, ng,
                           coef, weight, inv_b, dy, lddy, loss_part);
    else if (ng <= 8)
        hipLaunchKernelGGL(subspace_residual_kernel<8>, grid, dim3(kThreads), 0, s, y, ldy, t, ldt, rows, group, ng,
                           coef, weight, inv_b, dy, lddy, loss_part);
    else if (ng <= 16)
        hipLaunchKernelGGL(subspace_residual_kernel<16>, grid, dim3(kThreads), 0, s, y, ldy, t, ldt, rows, group,
                           ng, coef, weight, inv_b, dy, lddy, loss_part);
    else
        hipLaunchKernelGGL(subspace_residual_kernel<32>, grid, dim3(kThreads), 0, s, y, ldy, t, ldt, rows, group,
                           ng, coef, weight, inv_b, dy, lddy, loss_part);
}

void launch_colsum(const float *D, int64_t ldd, int M, int N, float *out, hipStream_t s) {
    if (N < 1) return;
    hipLaunchKernelGGL(colsum_kernel, dim3((N + 63) / 64), dim3(256), 0, s, D, ldd, M, N, out);
}

void launch_adam(float *p, const float *g, float *m, float *v, int64_t n, const AdamArgs &a, hipStream_t s) {
    hipLaunchKernelGGL(adam_kernel, dim3(grid_for(n, 4096)), dim3(kThreads), 0, s, p, g, m, v, n, a);
}

void launch_adam_ranges(float *p, const float *g, float *m, float *v, const AdamRanges &r, const AdamArgs &a,
                        hipStream_t s) {
    if (r.n < 1 || r.end[r.n - 1] < 1) return;
    hipLaunchKernelGGL(adam_ranges_kernel, dim3(grid_for(r.end[r.n - 1], 4096)), dim3(kThreads), 0, s, p, g, m, v,
                       r, a);
}

void launch_gather(const float *src, int64_t lds, const int *rows, int nrows, int ncols, float *dst,
                   hipStream_t s) {
    hipLaunchKernelGGL(gather_kernel, dim3(grid_for(int64_t(nrows) * ncols, 1024)), dim3(kThreads), 0, s, src,
                       lds, rows, nrows, ncols, dst);
}

}  // namespace mlp
}  // namespace kl
