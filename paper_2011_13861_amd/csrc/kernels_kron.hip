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
// A workgroup owns 32 consecutive rows and every o: it stages the 32 x nin input slice
// and D^T in LDS (loads coalesced along the contiguous index), runs the contraction on
// FP64 matrix cores and writes through LDS so that stores are coalesced too.
#include <algorithm>
#include <type_traits>

#include "kl_internal.h"

namespace kl {
namespace {

constexpr int kThreads = 256;
constexpr int kRT = 32;                 // rows per workgroup
constexpr size_t kLdsBudget = 160 * 1024;   // gfx950: up to 160 KB per workgroup

struct ModeArgs {
    const double *D;          // nout x nin row-major
    const double *DT;         // nin x nout row-major (D transposed)
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

typedef double doublex4 __attribute__((ext_vector_type(4)));

// MFMA form: v_mfma_f64_16x16x4_f64 with A = IN[16 rows][4 i], B = D^T[4 i][16 o];
// A[i][k] / B[k][j] sit in lane (i or j) + 16 k; accumulator r of lane L holds
// C[(L >> 4) + 4 r][L & 15].  The 32-row input slice and D^T are staged in LDS with the
// contraction index padded to a multiple of 4 by zeros; the (2 row tiles) x (o tiles)
// products are spread over the 4 waves.
template <bool FIRST, typename TIN, typename TOUT>
__global__ __launch_bounds__(kThreads) void mode_kernel(ModeArgs g) {
    extern __shared__ double smem[];
    const int nin = g.nin, nout = g.nout;
    const int Kp = (nin + 3) & ~3;
    const int NOp = (nout + 15) & ~15;
    const int ldi = kRT + 1;                              // sIN[i][row]
    const int ldo = NOp + 1;                              // sDT[i][o], sOUT[row][o]
    // per-row address bases first, so that the output staging below (which reuses the
    // tile region) can never overwrite them
    int64_t *rin = reinterpret_cast<int64_t *>(smem);     // input base per row
    int64_t *rout = rin + kRT;                            // output base per row
    int64_t *pin = rout + kRT;                            // input point base per row
    int64_t *pout = pin + kRT;                            // output point base per row
    double *tiles = smem + 4 * kRT;
    double *sIN = tiles;                                  // Kp * ldi
    double *sDT = sIN + size_t(Kp) * ldi;                 // Kp * ldo
    const int64_t nrows = g.A * g.Clo * g.nvec;
    const int64_t r0 = int64_t(blockIdx.x) * kRT;
    const int rows = int(min<int64_t>(kRT, nrows - r0));
    const int tid = threadIdx.x;
    // ---- per-row address bases (the only divisions) ----------------------------------
    if (tid < kRT) {
        int64_t bi = 0, bo = 0, qi = 0, qo = 0;
        if (tid < rows) {
            const int64_t r = r0 + tid;
            const int64_t a = r % g.A, t = r / g.A;
            const int64_t c = t % g.Clo, j = t / g.Clo;
            qi = a + g.A * int64_t(nin) * c;
            qo = a + g.A * int64_t(nout) * c;
            bi = qi + g.in_ldj * j;
            bo = qo + g.out_ldj * j;
        }
        rin[tid] = bi; rout[tid] = bo; pin[tid] = qi; pout[tid] = qo;
    }
    __syncthreads();
    // ---- stage IN (with the split sum and the scale) and D^T ---------------------------
    const TIN *in = static_cast<const TIN *>(g.in);
    const int tile = kRT * Kp;
    // batches of 8 elements per thread: the loads of a batch are issued before any of
    // its LDS stores, so that their latencies overlap
    for (int e0 = 0; e0 < tile; e0 += 8 * kThreads) {
        double vb[8];
        int64_t off[8], pidx[8];
        bool ok[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int e = e0 + u * kThreads + tid;
            int rr, i;
            if (FIRST) { rr = e / Kp; i = e % Kp; }        // contiguous along i
            else { rr = e % kRT; i = e / kRT; }            // contiguous along a
            ok[u] = e < tile && rr < rows && i < nin;
            off[u] = ok[u] ? rin[rr] + g.A * i : 0;
            pidx[u] = ok[u] ? pin[rr] + g.A * i : 0;
            vb[u] = 0.0;
        }
        // split partial sums: 8 independent loads per split
        for (int q = 0; q < g.nsplit; ++q) {
            const TIN *src = in + q * g.in_split;
#pragma unroll
            for (int u = 0; u < 8; ++u)
                if (ok[u]) vb[u] += double(src[off[u]]);
        }
        if (g.in_w) {
#pragma unroll
            for (int u = 0; u < 8; ++u)
                if (ok[u]) vb[u] *= g.in_scale * g.in_w[pidx[u]];
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int e = e0 + u * kThreads + tid;
            if (e < tile) {
                int rr, i;
                if (FIRST) { rr = e / Kp; i = e % Kp; }
                else { rr = e % kRT; i = e / kRT; }
                sIN[i * ldi + rr] = vb[u];
            }
        }
    }
    for (int e0 = 0; e0 < Kp * NOp; e0 += 8 * kThreads) {
        double vb[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int e = e0 + u * kThreads + tid;
            const int i = e / NOp, o = e % NOp;           // D^T row-major: contiguous in o
            vb[u] = (e < Kp * NOp && i < nin && o < nout) ? g.DT[int64_t(i) * nout + o] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int e = e0 + u * kThreads + tid;
            if (e < Kp * NOp) sDT[(e / NOp) * ldo + e % NOp] = vb[u];
        }
    }
    __syncthreads();
    // ---- MFMA over the (2 row tiles) x (NOp / 16 o tiles), 4 waves --------------------
    const int lane = tid & 63, wave = tid >> 6;
    const int li = lane & 15, lk = lane >> 4;
    const int ntiles = 2 * (NOp / 16);                    // <= 16 for nout <= 128
    doublex4 acc[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) acc[t] = doublex4{0.0, 0.0, 0.0, 0.0};
    for (int k0 = 0; k0 < Kp; k0 += 4) {
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            const int tt = wave + 4 * t;
            if (tt < ntiles) {
                const int rt = tt & 1, ot = tt >> 1;
                const double a = sIN[(k0 + lk) * ldi + rt * 16 + li];
                const double b = sDT[(k0 + lk) * ldo + ot * 16 + li];
                acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[t], 0, 0, 0);
            }
        }
    }
    // ---- results through LDS (the IN region is reused: kRT x (NOp + 1)) ---------------
    __syncthreads();
    double *sOUT = tiles;                                 // kRT * ldo, within the tile region
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        const int tt = wave + 4 * t;
        if (tt < ntiles) {
            const int rt = tt & 1, ot = tt >> 1;
#pragma unroll
            for (int r = 0; r < 4; ++r) sOUT[(rt * 16 + lk + 4 * r) * ldo + ot * 16 + li] = acc[t][r];
        }
    }
    __syncthreads();
    TOUT *out = static_cast<TOUT *>(g.out);
    const int outs = kRT * nout;
    for (int e = tid; e < outs; e += kThreads) {
        int rr, o;
        if (FIRST) { rr = e / nout; o = e % nout; }        // contiguous along o
        else { rr = e % kRT; o = e / kRT; }                // contiguous along a
        if (rr < rows) {
            double v = sOUT[rr * ldo + o];
            if (g.out_w) v *= g.out_w[pout[rr] + g.A * o];
            store_out<TOUT>(out, g.out_lo, rout[rr] + g.A * o, v);
        }
    }
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

// LDS: 4 x kRT row bases, then max(staged tiles, output staging)
size_t mode_lds_bytes(int nin, int nout) {
    const size_t Kp = (size_t(nin) + 3) & ~size_t(3), NOp = (size_t(nout) + 15) & ~size_t(15);
    const size_t tiles = Kp * (kRT + 1) * 8 + Kp * (NOp + 1) * 8;
    const size_t outs = size_t(kRT) * (NOp + 1) * 8;
    return 4 * kRT * 8 + std::max(tiles, outs);
}

bool mode_fits(int nin, int nout) {
    return nin >= 1 && nout >= 1 && nout <= 128 && mode_lds_bytes(nin, nout) <= kLdsBudget;
}

template <bool FIRST, typename TIN, typename TOUT>
void launch_mode_t(const ModeArgs &a, dim3 grid, size_t lds, hipStream_t s) {
    static bool attr_set = false;       // opt in to more than 64 KB of LDS, once
    if (!attr_set) {
        (void)hipFuncSetAttribute(reinterpret_cast<const void *>(&mode_kernel<FIRST, TIN, TOUT>),
                                  hipFuncAttributeMaxDynamicSharedMemorySize, int(kLdsBudget));
        attr_set = true;
    }
    hipLaunchKernelGGL((mode_kernel<FIRST, TIN, TOUT>), grid, dim3(kThreads), lds, s, a);
}

void launch_mode(const ModeSpec &m, hipStream_t s) {
    ModeArgs a;
    a.D = m.D; a.DT = m.DT; a.in = m.in; a.out = m.out; a.A = m.A; a.nin = m.nin; a.nout = m.nout;
    a.Clo = m.Clo; a.nvec = m.nvec; a.in_ldj = m.in_ldj; a.out_ldj = m.out_ldj;
    a.nsplit = m.nsplit > 0 ? m.nsplit : 1; a.in_split = m.in_split;
    a.in_w = m.in_w; a.in_scale = m.in_scale; a.out_w = m.out_w; a.out_lo = m.out_lo;
    const size_t lds = mode_lds_bytes(m.nin, m.nout);
    const int64_t nrows = m.A * m.Clo * m.nvec;
    const dim3 grid(unsigned((nrows + kRT - 1) / kRT));
    const bool first = m.A == 1;
    if (m.in_f32) {
        if (first) launch_mode_t<true, float, double>(a, grid, lds, s);
        else launch_mode_t<false, float, double>(a, grid, lds, s);
    } else if (m.out_f32) {
        if (first) launch_mode_t<true, double, float>(a, grid, lds, s);
        else launch_mode_t<false, double, float>(a, grid, lds, s);
    } else if (m.out_bf16) {
        if (first) launch_mode_t<true, double, __bf16>(a, grid, lds, s);
        else launch_mode_t<false, double, __bf16>(a, grid, lds, s);
    } else {
        if (first) launch_mode_t<true, double, double>(a, grid, lds, s);
        else launch_mode_t<false, double, double>(a, grid, lds, s);
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
