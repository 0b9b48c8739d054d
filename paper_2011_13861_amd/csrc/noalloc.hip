// kl_apply_noalloc: the apply of kl_apply (Algorithm 1) for callers that cannot allocate
// device memory (code under HIP graph capture, tight serving loops).  Every intermediate of
// the apply -- the Kronecker ping-pong buffers, the stage-5 input block, the stage-5 split
// partials and the stage-5 output -- lives in one file-scope device array of fixed size
// instead of the problem's own workspace.  The array's device address is taken once per
// device with hipGetSymbolAddress (with that device current); host code never passes the
// array's name itself to a kernel.  All calls on one device share that device's array.
#include <algorithm>
#include <mutex>
#include <sstream>

#include "kl_internal.h"

namespace kl {
namespace {

constexpr size_t kScratchBytes = size_t(64) << 20;      // 64 MiB per device
constexpr int kMaxDevices = 64;

__device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on the current device (looked up on the first call there).
kl_status scratch_address(void **out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess || dev < 0 || dev >= kMaxDevices) {
        set_error("kl_apply_noalloc: no usable current device");
        return KL_EHIP;
    }
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            set_error(std::string("kl_apply_noalloc: hipGetSymbolAddress: ") + hipGetErrorString(e));
            return KL_EHIP;
        }
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return KL_OK;
}

// Zeroes rows [r0, r1) of ncols columns (leading dimension ld elements of elem bytes).
__global__ __launch_bounds__(256) void zero_rows_kernel(unsigned char *__restrict__ base, int64_t ld, int64_t r0,
                                                        int64_t r1, int ncols, int elem) {
    const int64_t per_col = (r1 - r0) * elem;
    const int64_t total = per_col * ncols;
    for (int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x; i < total; i += int64_t(gridDim.x) * 256) {
        const int64_t c = i / per_col, b = i % per_col;
        base[(c * ld + r0) * elem + b] = 0;
    }
}

size_t round256(size_t b) { return (b + 255) / 256 * 256; }

}  // namespace
}  // namespace kl

using namespace kl;

extern "C" kl_status kl_apply_noalloc(kl_problem *P, int32_t precision, int32_t nvec, const double *x,
                                      int64_t ldx, double *y, int64_t ldy, void *stream) {
    if (!P || P->host_only) { set_error("kl_apply_noalloc: NULL or host-only handle"); return KL_EINVAL; }
    if (precision < KL_F64 || precision > KL_BF16X3) { set_error("kl_apply_noalloc: unsupported precision"); return KL_EINVAL; }
    if (nvec < 0) { set_error("kl_apply_noalloc: nvec < 0"); return KL_EINVAL; }
    if (nvec == 0) return KL_OK;
    if (!x || !y) { set_error("kl_apply_noalloc: NULL vector"); return KL_EINVAL; }
    if (ldx < P->hs.N || ldy < P->hs.N) { set_error("kl_apply_noalloc: leading dimension < N"); return KL_EINVAL; }
    const char *xb = reinterpret_cast<const char *>(x), *yb = reinterpret_cast<const char *>(y);
    const size_t xbytes = size_t(ldx) * (nvec - 1) * 8 + size_t(P->hs.N) * 8;
    const size_t ybytes = size_t(ldy) * (nvec - 1) * 8 + size_t(P->hs.N) * 8;
    if (xb < yb + ybytes && yb < xb + xbytes) { set_error("kl_apply_noalloc: x and y overlap"); return KL_EINVAL; }
    // layout of the scratch array for one 32-column chunk: T0, T1 (FP64), the stage-5 input
    // in the stage-5 precision (BF16: high then low parts), the stage-5 output and as many
    // split partials as fit (at least one)
    const int64_t Np = P->Ntpad;
    const size_t t_bytes = round256(size_t(problem_max_intermediate(P)) * kBW * sizeof(double));
    const int y5_elem = precision == KL_F64 ? 8 : precision == KL_F32 ? 4 : 2;
    const int y5_cols = precision == KL_BF16X3 ? 2 * kBW : kBW;   // BF16x3: high then low parts
    const size_t y5_bytes = round256(size_t(Np) * y5_cols * y5_elem);
    const int z_elem = precision == KL_F64 ? 8 : 4;
    const size_t z_bytes = round256(size_t(Np) * kBW * z_elem);
    const size_t fixed = 2 * t_bytes + y5_bytes + z_bytes;
    if (fixed + z_bytes > kScratchBytes) {
        std::ostringstream os;
        os << "kl_apply_noalloc: the problem needs " << ((fixed + z_bytes + (1 << 20) - 1) >> 20)
           << " MiB of scratch; the static scratch holds " << (kScratchBytes >> 20) << " MiB";
        set_error(os.str());
        return KL_EINVAL;
    }
    void *base = nullptr;
    kl_status st = scratch_address(&base);
    if (st != KL_OK) return st;
    unsigned char *b = static_cast<unsigned char *>(base);
    Workspace ws;
    ws.T0 = reinterpret_cast<double *>(b);
    ws.T1 = reinterpret_cast<double *>(b + t_bytes);
    void *y5 = b + 2 * t_bytes;
    ws.Y5d = ws.Y5f = ws.Y5b = y5;
    ws.Zf = b + 2 * t_bytes + y5_bytes;
    ws.Z5 = b + fixed;
    ws.max_split = int(std::min<size_t>(std::max(P->ws.max_split, 1), (kScratchBytes - fixed) / z_bytes));
    hipStream_t s = static_cast<hipStream_t>(stream);
    // the padding rows of the stage-5 input take part in the contraction and must be zero;
    // the previous call on this device may have left anything there
    if (Np > P->hs.Nt)
        hipLaunchKernelGGL(zero_rows_kernel, dim3(64), dim3(256), 0, s, static_cast<unsigned char *>(y5), Np,
                           P->hs.Nt, Np, y5_cols, y5_elem);
    for (int c0 = 0; c0 < nvec; c0 += kBW) {
        const int nb = std::min(kBW, nvec - c0);
        st = apply_chunk(P, precision, nb, x + int64_t(c0) * ldx, ldx, y + int64_t(c0) * ldy, ldy, s, &ws);
        if (st != KL_OK) return st;
    }
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
        set_error(std::string("kl_apply_noalloc: kernel launch: ") + hipGetErrorString(e));
        return KL_EHIP;
    }
    return KL_OK;
}
