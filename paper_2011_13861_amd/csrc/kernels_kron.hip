// Kronecker-stage kernels (Algorithm 1 stages 1-4 and 6-9, composed per direction).
//
// Sec. 2.2: (D_d x ... x D_1) vec(X) is evaluated as d mode-k contractions; each
// contraction here is one launch over column-major FP64 tensors.  The forward
// epilogue scales by J and converts to the stage-5 layout and precision (stage 4);
// the backward prologue sums the stage-5 split partials, scales by sigma^2 J and
// returns to FP64 (stage 6).
#include "kl_internal.h"

namespace kl {
namespace {

constexpr int kThreads = 256;

__global__ __launch_bounds__(kThreads) void mode_contract_kernel(
    const double *__restrict__ D, const double *__restrict__ in, double *__restrict__ out,
    int64_t A, int nin, int nout, int64_t Cn) {
    const int64_t total = A * nout * Cn;
    for (int64_t idx = int64_t(blockIdx.x) * kThreads + threadIdx.x; idx < total;
         idx += int64_t(gridDim.x) * kThreads) {
        const int64_t a = idx % A;
        const int64_t t = idx / A;
        const int o = int(t % nout);
        const int64_t c = t / nout;
        const double *src = in + a + A * nin * c;
        const double *row = D + int64_t(o) * nin;
        double s = 0.0;
        for (int i = 0; i < nin; ++i) s = fma(row[i], src[A * i], s);
        out[idx] = s;
    }
}

template <typename T>
__global__ __launch_bounds__(kThreads) void to_stage5_kernel(
    const double *__restrict__ Tin, int64_t Nt, int64_t ldt, int nvec,
    const double *__restrict__ J, int64_t Ntpad, T *__restrict__ Y5) {
    const int64_t total = Ntpad * kBW;
    for (int64_t idx = int64_t(blockIdx.x) * kThreads + threadIdx.x; idx < total;
         idx += int64_t(gridDim.x) * kThreads) {
        const int j = int(idx % kBW);
        const int64_t p = idx / kBW;
        double v = 0.0;
        if (p < Nt && j < nvec) v = J ? J[p] * Tin[p + ldt * j] : Tin[p + ldt * j];
        Y5[idx] = T(v);
    }
}

template <typename T>
__global__ __launch_bounds__(kThreads) void from_stage5_kernel(
    const T *__restrict__ Z5, int nsplit, int64_t Ntpad, int64_t Nt, int nvec,
    const double *__restrict__ w, double scale, double *__restrict__ Tout, int64_t ldt) {
    const int64_t total = Nt * nvec;
    for (int64_t idx = int64_t(blockIdx.x) * kThreads + threadIdx.x; idx < total;
         idx += int64_t(gridDim.x) * kThreads) {
        const int j = int(idx % nvec);
        const int64_t p = idx / nvec;
        double s = 0.0;
        for (int q = 0; q < nsplit; ++q) s += double(Z5[(q * Ntpad + p) * kBW + j]);
        const double f = w ? scale * w[p] : scale;
        Tout[p + ldt * j] = f * s;
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

unsigned grid_for(int64_t total) {
    int64_t g = (total + kThreads - 1) / kThreads;
    if (g > 65536) g = 65536;
    if (g < 1) g = 1;
    return unsigned(g);
}

}  // namespace

void launch_mode_contract(const double *D, const double *in, double *out, int64_t A, int nin,
                          int nout, int64_t Cn, hipStream_t s) {
    hipLaunchKernelGGL(mode_contract_kernel, dim3(grid_for(A * nout * Cn)), dim3(kThreads), 0, s,
                       D, in, out, A, nin, nout, Cn);
}

void launch_to_stage5(int precision, const double *T, int64_t Nt, int64_t ldt, int nvec,
                      const double *J, int64_t Ntpad, void *Y5, hipStream_t s) {
    const unsigned g = grid_for(Ntpad * kBW);
    if (precision == KL_F64)
        hipLaunchKernelGGL(to_stage5_kernel<double>, dim3(g), dim3(kThreads), 0, s, T, Nt, ldt, nvec,
                           J, Ntpad, static_cast<double *>(Y5));
    else
        hipLaunchKernelGGL(to_stage5_kernel<float>, dim3(g), dim3(kThreads), 0, s, T, Nt, ldt, nvec,
                           J, Ntpad, static_cast<float *>(Y5));
}

void launch_from_stage5(int precision, const void *Z5, int nsplit, int64_t Ntpad, int64_t Nt,
                        int nvec, const double *w, double scale, double *T, int64_t ldt,
                        hipStream_t s) {
    const unsigned g = grid_for(Nt * nvec);
    if (precision == KL_F64)
        hipLaunchKernelGGL(from_stage5_kernel<double>, dim3(g), dim3(kThreads), 0, s,
                           static_cast<const double *>(Z5), nsplit, Ntpad, Nt, nvec, w, scale, T, ldt);
    else
        hipLaunchKernelGGL(from_stage5_kernel<float>, dim3(g), dim3(kThreads), 0, s,
                           static_cast<const float *>(Z5), nsplit, Ntpad, Nt, nvec, w, scale, T, ldt);
}

void launch_copy_cols(const double *src, int64_t lds, double *dst, int64_t ldd, int64_t rows,
                      int cols, hipStream_t s) {
    hipLaunchKernelGGL(copy_cols_kernel, dim3(grid_for(rows * cols)), dim3(kThreads), 0, s, src,
                       lds, dst, ldd, rows, cols);
}

}  // namespace kl
