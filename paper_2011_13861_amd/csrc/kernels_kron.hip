// Kronecker-stage kernels (Algorithm 1 stages 1-4 and 6-9, composed per direction).
//
// Sec. 2.2: (D_d x ... x D_1) vec(X) is evaluated as d mode-k contractions.  One
// contraction is a batched small GEMM over "rows" r = (a, c, j):
//     OUT[r][o] = sum_i D[o][i] IN[r][i],
// with a < A (the directions before k), c < Clo (the directions after k), j the vector
// index.  IN/OUT addresses:  a + A (i + nin c) + ldj j  (and nout for OUT), i.e. the
// column-major tensor of each vector, with a free leading dimension ldj between vectors.
//
// Fusions (one launch per direction):
//   * last forward direction (stage 4): multiplies by J[p] and writes the stage-5 input
//     in its precision (column-major, ld = padded grid);
//   * first backward direction (stage 6): reads the stage-5 output (FP32 or FP64), which
//     stage 5 has already multiplied by sigma^2 J[p]; an optional per-point input weight
//     (in_w, in_scale) remains available.
// The point index of an entry is its address without the vector term, p = a + A (i + nin c).
//
// Each wave computes one 16 x 16 tile of OUT on the FP64 matrix cores (see below).
#include <algorithm>
#include <type_traits>

#include "kl_internal.h"

namespace kl {
namespace {

constexpr int kThreads = 256;

template <typename TOUT>
__device__ __forceinline__ void store_out(TOUT *out, void *out_lo, int64_t addr, double v) {
    if constexpr (std::is_same<TOUT, __bf16>::value) {
        const float f = float(v);
        const __bf16 hi = __bf16(f);
        out[addr] = hi;
        if (out_lo) static_cast<__bf16 *>(out_lo)[addr] = __bf16(f - float(hi));
    } else {
        out[addr] = TOUT(v);
    }
}

typedef double doublex4 __attribute__((ext_vector_type(4)));

// One wave per 16 x 16 output tile on v_mfma_f64_16x16x4_f64, operands loaded straight
// from memory into registers (all loads of a wave are issued before the first MFMA), no
// LDS and no barriers.  Lane layout: A[i][k] and B[k][j] sit in lane (i or j) + 16 k;
// accumulator r of lane L holds C[(L >> 4) + 4 r][L & 15].
//  * First direction (A == 1): C = IN D^T  (16 rows x 16 o): A = IN[row][i], B = D^T[i][o];
//    a lane of the result holds 16 consecutive o of one row -> coalesced stores.
//  * Later directions: C = D IN^T (16 o x 16 rows): A = D[o][i], B = IN[row][i]; a lane
//    holds 16 consecutive rows (consecutive a) of one o -> coalesced stores.
// The contraction index is processed in chunks of 64 (16 MFMA steps).
constexpr int kChunk = 16;                 // MFMA steps per operand batch (64 indices)

template <bool FIRST, typename TIN, typename TOUT>
__device__ __forceinline__ void mode_tile(const ModeArgs &g, int64_t tile) {
    const int lane = threadIdx.x & 63;
    const int li = lane & 15, lk = lane >> 4;
    const int nin = g.nin, nout = g.nout;
    // row counts fit in 32 bits (checked on the host), so the row -> (a, c, j) split uses
    // 32-bit division (64-bit division is a long software sequence on the GPU)
    const uint32_t A = uint32_t(g.A), Clo = uint32_t(g.Clo);
    const uint32_t nrows = A * Clo * uint32_t(g.nvec);
    const uint32_t rtiles = (nrows + 15) / 16;
    const uint32_t otiles = uint32_t(nout + 15) / 16;
    if (tile >= int64_t(rtiles) * otiles) return;  // whole wave leaves together
    const uint32_t rt = uint32_t(tile / otiles);
    const int ot = int(tile - int64_t(rt) * otiles);
    // this lane's row (operand index li) and its address bases
    const uint32_t r = rt * 16 + li;
    const bool rok = r < nrows;
    uint32_t ra = 0, rc = 0, rj = 0;
    if (rok) {
        const uint32_t t = FIRST ? r : r / A;
        ra = FIRST ? 0 : r - t * A;
        rj = t / Clo;
        rc = t - rj * Clo;
    }
    const int64_t pin = int64_t(ra) + g.A * int64_t(nin) * rc;
    const int64_t bin = pin + g.in_ldj * int64_t(rj);
    const int o_l = ot * 16 + li;                  // this lane's o (operand index li)
    const bool ook = o_l < nout;
    const TIN *in = static_cast<const TIN *>(g.in);
    doublex4 acc = {0.0, 0.0, 0.0, 0.0};
    for (int kc = 0; kc < nin; kc += 4 * kChunk) {
        double xa[kChunk], xb[kChunk];
#pragma unroll
        for (int s = 0; s < kChunk; ++s) {
            const int i = kc + 4 * s + lk;
            double vin = 0.0, vd = 0.0;
            if (i < nin) {
                if (rok) {
                    vin = double(in[bin + g.A * i]);
                    if (g.in_w) vin *= g.in_scale * g.in_w[pin + g.A * i];
                }
                if (ook) vd = g.D[int64_t(o_l) * nin + i];
            }
            if (FIRST) { xa[s] = vin; xb[s] = vd; }
            else { xa[s] = vd; xb[s] = vin; }
        }
#pragma unroll
        for (int s = 0; s < kChunk; ++s)
            if (kc + 4 * s < nin)
                acc = __builtin_amdgcn_mfma_f64_16x16x4f64(xa[s], xb[s], acc, 0, 0, 0);
    }
    // ---- store: C[(lane >> 4) + 4 q][lane & 15] --------------------------------------
    TOUT *out = static_cast<TOUT *>(g.out);
    if (FIRST) {
        // rows rt 16 + lk + 4 q (A == 1): split the first one, then step by 4
        uint32_t rr = rt * 16 + lk;
        uint32_t j = rr / Clo, c = rr - j * Clo;
        const int o = ot * 16 + li;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            if (rr < nrows && o < nout) {
                const int64_t p = int64_t(o) + int64_t(nout) * c;
                double v = acc[q];
                if (g.out_w) v *= g.out_w[p];
                store_out<TOUT>(out, g.out_lo, p + g.out_ldj * int64_t(j), v);
            }
            rr += 4;
            c += 4;
            while (c >= Clo) { c -= Clo; ++j; }
        }
    } else if (rok) {
        // row r (this lane's), outputs o = ot 16 + lk + 4 q
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int o = ot * 16 + lk + 4 * q;
            if (o < nout) {
                const int64_t p = int64_t(ra) + g.A * (int64_t(o) + int64_t(nout) * rc);
                double v = acc[q];
                if (g.out_w) v *= g.out_w[p];
                store_out<TOUT>(out, g.out_lo, p + g.out_ldj * int64_t(rj), v);
            }
        }
    }
}

template <bool FIRST, typename TIN, typename TOUT>
__global__ __launch_bounds__(kThreads) void mode_kernel(ModeArgs g) {
    mode_tile<FIRST, TIN, TOUT>(g, int64_t(blockIdx.x) * (kThreads / 64) + (threadIdx.x >> 6));
}

// One direction for every problem of a batch: workgroup b belongs to the problem p with
// wg_prefix[p] <= b < wg_prefix[p + 1] (binary search over nprob + 1 entries) and
// computes that problem's tiles 4 (b - wg_prefix[p]) + wave.
template <bool FIRST, typename TIN, typename TOUT>
__global__ __launch_bounds__(kThreads) void mode_batch_kernel(const ModeArgs *__restrict__ args,
                                                              const int64_t *__restrict__ wg_prefix, int nprob,
                                                              const int *__restrict__ active) {
    const int64_t b = blockIdx.x;
    int lo = 0, hi = nprob;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (wg_prefix[mid] <= b) lo = mid; else hi = mid;
    }
    if (active && active[lo] == 0) return;
    const ModeArgs g = args[lo];
    mode_tile<FIRST, TIN, TOUT>(g, (b - wg_prefix[lo]) * (kThreads / 64) + (threadIdx.x >> 6));
}

__global__ __launch_bounds__(kThreads) void copy_cols_kernel(
    const double *__restrict__ src, int64_t lds, double *__restrict__ dst, int64_t ldd,
    int64_t rows, int cols) {
    const int64_t total = rows * cols;
    for (int64_t idx = int64_t(blockIdx.x) * kThreads + threadIdx.x; idx < total;
         idx += int64_t(gridDim.x) * kThreads) {
        const int64_t r = idx % rows;
        const int64_t c = idx / rows;
        dst[r + ldd * c] = src[r + lds * c];
    }
}

template <typename T>
__global__ __launch_bounds__(kThreads) void pack_stage5_kernel(const double *__restrict__ y,
                                                               int64_t ldy, int64_t Nt, int nvec,
                                                               int64_t Ntpad, T *__restrict__ Y5,
                                                               void *Y5lo) {
    const int64_t total = Nt * nvec;
    for (int64_t idx = int64_t(blockIdx.x) * kThreads + threadIdx.x; idx < total;
         idx += int64_t(gridDim.x) * kThreads) {
        const int64_t p = idx % Nt, j = idx / Nt;
        store_out<T>(Y5, Y5lo, j * Ntpad + p, y[p + ldy * j]);
    }
}

template <typename T>
__global__ __launch_bounds__(kThreads) void unpack_stage5_kernel(
    const T *__restrict__ Z5, int nsplit, int64_t Ntpad, int64_t Nt, int nvec, double scale,
    double *__restrict__ z, int64_t ldz) {
    const int64_t total = Nt * nvec;
    for (int64_t idx = int64_t(blockIdx.x) * kThreads + threadIdx.x; idx < total;
         idx += int64_t(gridDim.x) * kThreads) {
        const int64_t p = idx % Nt, j = idx / Nt;
        double s = 0.0;
        for (int q = 0; q < nsplit; ++q) s += double(Z5[(q * int64_t(kBW) + j) * Ntpad + p]);
        z[p + ldz * j] = scale * s;
    }
}

unsigned grid_for(int64_t total) {
    int64_t g = (total + kThreads - 1) / kThreads;
    if (g > 65536) g = 65536;
    if (g < 1) g = 1;
    return unsigned(g);
}

}  // namespace

bool mode_fits(int nin, int nout) { return nin >= 1 && nout >= 1 && nin <= 4096 && nout <= 4096; }

ModeArgs mode_args(const ModeSpec &m) {
    ModeArgs a;
    a.D = m.D; a.DT = m.DT; a.in = m.in; a.out = m.out; a.A = m.A; a.nin = m.nin; a.nout = m.nout;
    a.Clo = m.Clo; a.nvec = m.nvec; a.in_ldj = m.in_ldj; a.out_ldj = m.out_ldj;
    a.nsplit = 1; a.in_split = 0;
    a.in_w = m.in_w; a.in_scale = m.in_scale; a.out_w = m.out_w; a.out_lo = m.out_lo;
    return a;
}

int64_t mode_workgroups(const ModeSpec &m) {
    const int64_t nrows = m.A * m.Clo * m.nvec;
    const int64_t tiles = (nrows + 15) / 16 * ((m.nout + 15) / 16);
    return (tiles + 3) / 4;
}

void launch_mode_batch(const ModeSpec &kind, const ModeArgs *args, const int64_t *wg_prefix, int nprob,
                       int64_t total_wgs, const int *active, hipStream_t s) {
    if (total_wgs < 1) return;
    const dim3 grid(static_cast<unsigned>(total_wgs));
    const bool first = kind.A == 1;
#define KL_MODEB(F, TI, TO) hipLaunchKernelGGL((mode_batch_kernel<F, TI, TO>), grid, dim3(kThreads), 0, s, \
                                               args, wg_prefix, nprob, active)
    if (kind.in_f32) {
        if (first) KL_MODEB(true, float, double); else KL_MODEB(false, float, double);
    } else if (kind.out_f32) {
        if (first) KL_MODEB(true, double, float); else KL_MODEB(false, double, float);
    } else if (kind.out_bf16) {
        if (first) KL_MODEB(true, double, __bf16); else KL_MODEB(false, double, __bf16);
    } else {
        if (first) KL_MODEB(true, double, double); else KL_MODEB(false, double, double);
    }
#undef KL_MODEB
}

void launch_mode(const ModeSpec &m, hipStream_t s) {
    const ModeArgs a = mode_args(m);
    const dim3 grid(unsigned(mode_workgroups(m)));
    const bool first = m.A == 1;
#define KL_MODE(F, TI, TO) hipLaunchKernelGGL((mode_kernel<F, TI, TO>), grid, dim3(kThreads), 0, s, a)
    if (m.in_f32) {
        if (first) KL_MODE(true, float, double); else KL_MODE(false, float, double);
    } else if (m.out_f32) {
        if (first) KL_MODE(true, double, float); else KL_MODE(false, double, float);
    } else if (m.out_bf16) {
        if (first) KL_MODE(true, double, __bf16); else KL_MODE(false, double, __bf16);
    } else {
        if (first) KL_MODE(true, double, double); else KL_MODE(false, double, double);
    }
#undef KL_MODE
}

void launch_pack_stage5(int precision, const double *y, int64_t ldy, int64_t Nt, int nvec,
                        int64_t Ntpad, void *Y5, hipStream_t s) {
    const unsigned g = grid_for(Nt * nvec);
    if (precision == KL_F64)
        hipLaunchKernelGGL(pack_stage5_kernel<double>, dim3(g), dim3(kThreads), 0, s, y, ldy, Nt, nvec,
                           Ntpad, static_cast<double *>(Y5), nullptr);
    else if (precision == KL_F32)
        hipLaunchKernelGGL(pack_stage5_kernel<float>, dim3(g), dim3(kThreads), 0, s, y, ldy, Nt, nvec,
                           Ntpad, static_cast<float *>(Y5), nullptr);
    else
        hipLaunchKernelGGL(pack_stage5_kernel<__bf16>, dim3(g), dim3(kThreads), 0, s, y, ldy, Nt, nvec,
                           Ntpad, static_cast<__bf16 *>(Y5),
                           precision == KL_BF16X3 ? static_cast<void *>(static_cast<__bf16 *>(Y5) + Ntpad * kBW)
                                                  : nullptr);
}

void launch_unpack_stage5(int precision, const void *Z5, int nsplit, int64_t Ntpad, int64_t Nt,
                          int nvec, double scale, double *z, int64_t ldz, hipStream_t s) {
    const unsigned g = grid_for(Nt * nvec);
    if (precision == KL_F64)
        hipLaunchKernelGGL(unpack_stage5_kernel<double>, dim3(g), dim3(kThreads), 0, s,
                           static_cast<const double *>(Z5), nsplit, Ntpad, Nt, nvec, scale, z, ldz);
    else
        hipLaunchKernelGGL(unpack_stage5_kernel<float>, dim3(g), dim3(kThreads), 0, s,
                           static_cast<const float *>(Z5), nsplit, Ntpad, Nt, nvec, scale, z, ldz);
}

void launch_copy_cols(const double *src, int64_t lds, double *dst, int64_t ldd, int64_t rows,
                      int cols, hipStream_t s) {
    hipLaunchKernelGGL(copy_cols_kernel, dim3(grid_for(rows * cols)), dim3(kThreads), 0, s, src,
                       lds, dst, ldd, rows, cols);
}

}  // namespace kl
