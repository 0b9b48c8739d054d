// Kronecker-stage kernels (Algorithm 1 stages 1-4 and 6-9, composed per direction).
//
// Sec. 2.2: (D_d x ... x D_1) vec(X) is evaluated as d mode-k contractions.  One
// contraction is a batched small GEMM over "rows" r = (a, c, j):
//     OUT[r][o] = sum_i D[o][i] IN[r][i],
// with a < A (the directions before k), c < Clo (the directions after k), j the vector
// index.  IN/OUT addresses:  a + A (i + nin c) + ldj j  (and nout for OUT), i.e. the
// column-major tensor of each vector, with a free leading dimension ldj between vectors.
//
// Fusions (one launch per direction, 2d + 1 launches per apply):
//   * last forward direction (stage 4): multiplies by J[p] and writes the stage-5 input
//     in its precision (column-major, ld = padded grid);
//   * first backward direction (stage 6): sums the stage-5 split partials, multiplies by
//     sigma^2 J[p], in FP64.
// The point index of an entry is its address without the vector term, p = a + A (i + nin c).
//
// A workgroup owns 32 consecutive rows and a range of o: it stages the 32 x nin input
// slice and the factor rows D[o0:o0+oc][:] in LDS (loads coalesced along the contiguous
// index) and each thread accumulates up to R outputs for one row.
#include <algorithm>
#include <type_traits>

#include "kl_internal.h"

namespace kl {
namespace {

constexpr int kThreads = 256;
constexpr int kRT = 32;                 // rows per workgroup
constexpr size_t kLdsBudget = 64 * 1024;

struct ModeArgs {
    const double *D;          // nout x nin row-major
    const void *in;           // TIN
    void *out;                // TOUT
    int64_t A;                // product of the sizes before the direction (1 = first)
    int nin, nout;
    int64_t Clo;              // product of the sizes after the direction
    int nvec;
    int64_t in_ldj, out_ldj;  // distance between vectors
    int nsplit;               // input partial sums to add (stage-5 splits)
    int64_t in_split;         // distance between splits
    const double *in_w;       // optional per-point input scale (times in_scale)
    double in_scale;
    const double *out_w;      // optional per-point output scale
    void *out_lo;             // BF16 output only: low part v - bf16(v), or NULL
    int oc;                   // o-range per workgroup
};

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

template <bool FIRST, int R, typename TIN, typename TOUT>
__global__ __launch_bounds__(kThreads) void mode_kernel(ModeArgs g) {
    extern __shared__ double smem[];
    const int nin = g.nin;
    double *sIN = smem;                                   // [nin][kRT + 1]
    double *sD = smem + size_t(nin) * (kRT + 1);          // [oc][nin]
    const int64_t nrows = g.A * g.Clo * g.nvec;
    const int64_t r0 = int64_t(blockIdx.x) * kRT;
    const int rows = int(min<int64_t>(kRT, nrows - r0));
    const int o0 = blockIdx.y * g.oc;
    const int oc = min(g.oc, g.nout - o0);
    const int tid = threadIdx.x;
    const TIN *in = static_cast<const TIN *>(g.in);
    // ---- stage the input rows (with the stage-6 split sum and scale) -----------------
    const int tile = kRT * nin;
    for (int e = tid; e < tile; e += kThreads) {
        int rr, i;
        if (FIRST) { rr = e / nin; i = e % nin; }          // contiguous along i
        else { rr = e % kRT; i = e / kRT; }                // contiguous along a
        double v = 0.0;
        if (rr < rows) {
            const int64_t r = r0 + rr;
            const int64_t a = r % g.A, t = r / g.A;
            const int64_t c = t % g.Clo, j = t / g.Clo;
            const int64_t p = a + g.A * (i + int64_t(nin) * c);
            const int64_t addr = p + g.in_ldj * j;
            for (int q = 0; q < g.nsplit; ++q) v += double(in[addr + q * g.in_split]);
            if (g.in_w) v *= g.in_scale * g.in_w[p];
        }
        sIN[i * (kRT + 1) + rr] = v;
    }
    for (int e = tid; e < oc * nin; e += kThreads) sD[e] = g.D[int64_t(o0) * nin + e];
    __syncthreads();
    // ---- compute: 32 lanes = 32 rows, 8 groups take o = grp + 8 q ----------------------
    const int row = tid & 31;
    const int grp = tid >> 5;
    double acc[R];
#pragma unroll
    for (int q = 0; q < R; ++q) acc[q] = 0.0;
    for (int i = 0; i < nin; ++i) {
        const double v = sIN[i * (kRT + 1) + row];
#pragma unroll
        for (int q = 0; q < R; ++q) {
            const int o = grp + 8 * q;
            if (o < oc) acc[q] = fma(sD[o * nin + i], v, acc[q]);
        }
    }
    // ---- write -------------------------------------------------------------------------
    TOUT *out = static_cast<TOUT *>(g.out);
    if (FIRST) {
        // through LDS so that consecutive threads write consecutive o
        __syncthreads();
        double *sOUT = smem;                               // [kRT][oc + 1]
#pragma unroll
        for (int q = 0; q < R; ++q) {
            const int o = grp + 8 * q;
            if (o < oc) sOUT[row * (oc + 1) + o] = acc[q];
        }
        __syncthreads();
        for (int e = tid; e < rows * oc; e += kThreads) {
            const int rr = e / oc, ol = e % oc;
            const int64_t r = r0 + rr;
            const int64_t c = r % g.Clo, j = r / g.Clo;
            const int64_t p = (o0 + ol) + int64_t(g.nout) * c;
            double v = sOUT[rr * (oc + 1) + ol];
            if (g.out_w) v *= g.out_w[p];
            store_out<TOUT>(out, g.out_lo, p + g.out_ldj * j, v);
        }
    } else if (row < rows) {
        const int64_t r = r0 + row;
        const int64_t a = r % g.A, t = r / g.A;
        const int64_t c = t % g.Clo, j = t / g.Clo;
#pragma unroll
        for (int q = 0; q < R; ++q) {
            const int o = grp + 8 * q;
            if (o < oc) {
                const int64_t p = a + g.A * ((o0 + o) + int64_t(g.nout) * c);
                double v = acc[q];
                if (g.out_w) v *= g.out_w[p];
                store_out<TOUT>(out, g.out_lo, p + g.out_ldj * j, v);
            }
        }
    }
}

template <bool FIRST, typename TIN, typename TOUT>
void launch_r(const ModeArgs &a, dim3 grid, size_t lds, hipStream_t s) {
    const int R = (a.oc + 7) / 8;
    if (R <= 4) hipLaunchKernelGGL((mode_kernel<FIRST, 4, TIN, TOUT>), grid, dim3(kThreads), lds, s, a);
    else if (R <= 8) hipLaunchKernelGGL((mode_kernel<FIRST, 8, TIN, TOUT>), grid, dim3(kThreads), lds, s, a);
    else if (R <= 12) hipLaunchKernelGGL((mode_kernel<FIRST, 12, TIN, TOUT>), grid, dim3(kThreads), lds, s, a);
    else hipLaunchKernelGGL((mode_kernel<FIRST, 16, TIN, TOUT>), grid, dim3(kThreads), lds, s, a);
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

bool mode_fits(int nin) {
    // at least 8 factor rows must fit next to the 32 x nin input slice
    return nin >= 1 && size_t(nin) * (kRT + 1) * 8 + size_t(8) * nin * 8 <= kLdsBudget;
}

void launch_mode(const ModeSpec &m, hipStream_t s) {
    ModeArgs a;
    a.D = m.D; a.in = m.in; a.out = m.out; a.A = m.A; a.nin = m.nin; a.nout = m.nout;
    a.Clo = m.Clo; a.nvec = m.nvec; a.in_ldj = m.in_ldj; a.out_ldj = m.out_ldj;
    a.nsplit = m.nsplit > 0 ? m.nsplit : 1; a.in_split = m.in_split;
    a.in_w = m.in_w; a.in_scale = m.in_scale; a.out_w = m.out_w; a.out_lo = m.out_lo;
    // o-range: as many factor rows as fit next to the input slice, at most 128
    const size_t in_bytes = size_t(m.nin) * (kRT + 1) * 8;
    int oc = int(std::min<size_t>(128, (kLdsBudget - in_bytes) / (size_t(m.nin) * 8)));
    oc = std::min(oc, m.nout);
    a.oc = oc;
    const size_t lds = std::max(in_bytes + size_t(oc) * m.nin * 8, size_t(kRT) * (oc + 1) * 8);
    const int64_t nrows = m.A * m.Clo * m.nvec;
    const dim3 grid(unsigned((nrows + kRT - 1) / kRT), unsigned((m.nout + oc - 1) / oc));
    const bool first = m.A == 1;
    if (m.in_f32) {
        if (first) launch_r<true, float, double>(a, grid, lds, s);
        else launch_r<false, float, double>(a, grid, lds, s);
    } else if (m.out_f32) {
        if (first) launch_r<true, double, float>(a, grid, lds, s);
        else launch_r<false, double, float>(a, grid, lds, s);
    } else if (m.out_bf16) {
        if (first) launch_r<true, double, __bf16>(a, grid, lds, s);
        else launch_r<false, double, __bf16>(a, grid, lds, s);
    } else {
        if (first) launch_r<true, double, double>(a, grid, lds, s);
        else launch_r<false, double, double>(a, grid, lds, s);
    }
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
