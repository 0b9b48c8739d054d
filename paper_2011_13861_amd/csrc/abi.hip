// C ABI: problem setup, the matrix-free apply (Algorithm 1) and accessors.
#include <chrono>
#include <cmath>
#include <cstring>
#include <new>
#include <sstream>

#include "kl_internal.h"

namespace kl {

namespace {
thread_local std::string g_error;
}

void set_error(const std::string &msg) { g_error = msg; }

namespace {

kl_status hip_check(hipError_t e, const char *what) {
    if (e == hipSuccess) return KL_OK;
    std::ostringstream os;
    os << what << ": " << hipGetErrorString(e);
    set_error(os.str());
    return e == hipErrorOutOfMemory ? KL_ENOMEM : KL_EHIP;
}

template <typename T>
kl_status dev_alloc(T **p, size_t count, const char *what) {
    *p = nullptr;
    if (count == 0) count = 1;
    return hip_check(hipMalloc(reinterpret_cast<void **>(p), count * sizeof(T)), what);
}

void free_problem(kl_problem *P) {
    if (!P) return;
    for (kl_problem *Q : P->patches) free_problem(Q);
    free_solver_cache(P->solver);
    for (hipEvent_t e : P->prof_ev) hipEventDestroy(e);
    hipFree(P->dX64);
    hipFree(P->dX32);
    hipFree(P->dJ);
    for (int k = 0; k < 3; ++k) {
        hipFree(P->dC[k]);
        hipFree(P->dCT[k]);
        hipFree(P->dE[k]);
        hipFree(P->dET[k]);
        hipFree(P->dLT[k]);
        hipFree(P->dL1[k]);
    }
    hipFree(P->ws.T0);
    hipFree(P->ws.T1);
    hipFree(P->ws.Y5d);
    hipFree(P->ws.Y5f);
    hipFree(P->ws.Y5b);
    hipFree(P->ws.Z5);
    hipFree(P->ws.Zf);
    hipFree(P->ws.symF);
    hipFree(P->ws.symO);
    hipFree(P->ws.symTab);
    delete P;
}

// Coordinate scale for stage 5: every kernel evaluates a base-2 exponential, so the
// coordinates absorb log2(e) / ell (exp, exp-L1) or sqrt(log2 e) / ell (sqexp).
double coord_scale(int cov_kind, double ell) {
    const double log2e = 1.4426950408889634;
    switch (cov_kind) {
    case KL_COV_EXP:
    case KL_COV_EXP_L1: return log2e / ell;
    case KL_COV_SQEXP: return std::sqrt(log2e) / ell;
    default: return 1.0;
    }
}


bool valid_precision(int precision) { return precision >= KL_F64 && precision <= KL_BF16X3; }

// Scaled Greville points for the stage-5 kernels (Sec. 4.3): X log2(e) / ell (or with
// sqrt(log2 e) for the squared exponential) per direction, in FP64 and rounded to FP32.
// The padding points stay zero (their rows and columns carry zero weight).
kl_status upload_points(kl_problem *P, hipStream_t s) {
    const HostSetup &hs = P->hs;
    const int d = hs.d;
    const int64_t Np = P->Ntpad;
    std::vector<double> x64(size_t(d) * Np, 0.0);
    std::vector<float> x32(size_t(d) * Np, 0.f);
    for (int k = 0; k < d; ++k) {
        const double sc = coord_scale(P->cov_kind, P->ell[k]);
        for (int64_t p = 0; p < hs.Nt; ++p) {
            const double v = hs.X[size_t(p) * d + k] * sc;
            x64[size_t(k) * Np + p] = v;
            x32[size_t(k) * Np + p] = float(v);
        }
    }
    kl_status st = hip_check(hipMemcpyAsync(P->dX64, x64.data(), x64.size() * 8, hipMemcpyHostToDevice, s),
                             "copy X64");
    if (st != KL_OK) return st;
    st = hip_check(hipMemcpyAsync(P->dX32, x32.data(), x32.size() * 4, hipMemcpyHostToDevice, s), "copy X32");
    if (st != KL_OK) return st;
    // the host staging vectors go out of scope here
    return hip_check(hipStreamSynchronize(s), "hipStreamSynchronize");
}

void *stage5_input(const Workspace &ws, int precision) {
    switch (precision) {
    case KL_F64: return ws.Y5d;
    case KL_F32: return ws.Y5f;
    default: return ws.Y5b;
    }
}

}  // namespace

int64_t max_intermediate(const HostSetup &hs) {
    int64_t best = std::max(hs.N, hs.Nt);
    for (int k = 0; k <= hs.d; ++k) {
        int64_t f = 1, b = 1;
        for (int j = 0; j < hs.d; ++j) {
            f *= (j < k) ? hs.nt[j] : hs.n[j];
            b *= (j < k) ? hs.n[j] : hs.nt[j];
        }
        best = std::max(best, std::max(f, b));
    }
    return best;
}

// Stage-5 launch; while profiling is on, a pair of HIP events (without the system-scope
// fence, which would add a cache writeback to the interval) brackets the covariance kernel.
int timed_stage5(kl_problem *P, const Workspace &ws, int precision, const void *Y5, const double *wrow,
                 double scale, hipStream_t s, bool defer_reduce = false) {
    const bool rec = P->prof_on && P->prof_used + 2 <= P->prof_ev.size();
    if (P->s5_sym[precision] && ws.symF) {
        launch_stage5_sym(P, precision, ws, Y5, wrow, scale, s, rec ? P->prof_ev[P->prof_used] : nullptr,
                          rec ? P->prof_ev[P->prof_used + 1] : nullptr);
        if (rec) {
            P->prof_prec.push_back(precision);
            P->prof_used += 2;
        }
        return 1;
    }
    const int nsplit = launch_stage5(P, precision, Y5, ws.Z5, ws.Zf, wrow, scale, s,
                                     rec ? P->prof_ev[P->prof_used] : nullptr,
                                     rec ? P->prof_ev[P->prof_used + 1] : nullptr, defer_reduce, ws.max_split);
    if (rec) {
        P->prof_prec.push_back(precision);
        P->prof_used += 2;
    }
    return nsplit;
}

int64_t problem_max_intermediate(const kl_problem *P) {
    int64_t best = 0;
    for (int i = 0; i < patch_count(P); ++i) best = std::max(best, max_intermediate(patch_of(P, i)->hs));
    return best;
}

// Whether the first two directions of each side run as one fused launch (mode2_kernel):
// for every patch, or for none.
bool fused_directions(const kl_problem *P, int nb) {
    if (!P->fuse_dirs || P->hs.d < 2) return false;
    for (int i = 0; i < patch_count(P); ++i) {
        const HostSetup &hs = patch_of(P, i)->hs;
        int64_t clo_f = nb, clo_b = nb;
        for (int k = 2; k < hs.d; ++k) { clo_f *= hs.n[k]; clo_b *= hs.nt[k]; }
        if (!mode2_fits(hs.n[0], hs.n[1], hs.nt[0], hs.nt[1], clo_f) ||
            !mode2_fits(hs.nt[0], hs.nt[1], hs.n[0], hs.n[1], clo_b))
            return false;
    }
    return true;
}

// Stages 1-4 of one patch Q with the factors D[k] (nt_k x n_k, row-major) and their
// transposes DT[k]: x (Q's N x nb, ld ldx) -> its rows of Y5 (ld ldy5; BF16x3 writes the low
// parts to Y5lo), times J (its rows) unless J is NULL.
void forward_patch(const kl_problem *Q, const double *const *D, const double *const *DT, bool fuse, int y5_kind,
                   int nb, const double *x, int64_t ldx, void *Y5, void *Y5lo, int64_t ldy5, const double *J,
                   double *T0, double *T1, hipStream_t s) {
    const HostSetup &hs = Q->hs;
    const int d = hs.d;
    const void *cur = x;
    int64_t cur_ld = ldx;
    int64_t A = 1;
    int k0 = 0;
    if (fuse) {
        Mode2Args a{};
        a.D1 = D[0]; a.D2 = D[1]; a.D1T = DT[0]; a.D2T = DT[1];
        a.in = x; a.in_ldj = ldx;
        a.nin1 = hs.n[0]; a.nin2 = hs.n[1]; a.nout1 = hs.nt[0]; a.nout2 = hs.nt[1];
        a.Clo = 1;
        for (int j = 2; j < d; ++j) a.Clo *= hs.n[j];
        a.nvec = nb;
        a.nsplit = 1; a.in_split = 0; a.in_w = nullptr; a.in_scale = 1.0;
        if (d == 2) {
            a.out = Y5; a.out_lo = Y5lo; a.out_ldj = ldy5; a.out_w = J;
            launch_mode2(a, false, y5_kind, s);
        } else {
            a.out = T0; a.out_lo = nullptr; a.out_ldj = int64_t(hs.nt[0]) * hs.nt[1] * a.Clo; a.out_w = nullptr;
            launch_mode2(a, false, 0, s);
        }
        cur = T0;
        cur_ld = int64_t(hs.nt[0]) * hs.nt[1] * a.Clo;
        A = int64_t(hs.nt[0]) * hs.nt[1];
        k0 = 2;
    }
    for (int k = k0; k < d; ++k) {
        ModeSpec m;
        m.D = D[k];
        m.DT = DT[k];
        m.in = cur;
        m.in_ldj = cur_ld;
        m.A = A;
        m.nin = hs.n[k];
        m.nout = hs.nt[k];
        m.Clo = 1;
        for (int j = k + 1; j < d; ++j) m.Clo *= hs.n[j];
        m.nvec = nb;
        if (k == d - 1) {
            m.out = Y5;
            m.out_ldj = ldy5;
            m.out_w = J;
            m.out_f32 = y5_kind == 1;
            m.out_bf16 = y5_kind == 2;
            m.out_lo = Y5lo;
        } else {
            m.out = (cur == T0) ? T1 : T0;
            m.out_ldj = A * hs.nt[k] * m.Clo;
        }
        launch_mode(m, s);
        A *= hs.nt[k];
        cur = m.out;
        cur_ld = m.out_ldj;
    }
}

namespace {

// Stages 6-9 of one patch Q: its rows of the stage-5 output -> y (Q's N x nb, ld ldy).
// Fused: `in` holds nsplit partials `in_split` apart (or the finished rows when nsplit
// is 1), added in split order and scaled by sigma^2 J (in_w, in_scale) on the way in.
// Otherwise `in` holds the finished rows (sigma^2 J already applied).  in_f32: FP32 rows.
void backward_patch(const kl_problem *Q, bool fuse, bool in_f32, int nb, const void *in, int64_t ldin,
                    int nsplit, int64_t in_split, const double *in_w, double in_scale, double *y, int64_t ldy,
                    double *T0, double *T1, hipStream_t s) {
    const HostSetup &hs = Q->hs;
    const int d = hs.d;
    const void *cur = in;
    int64_t cur_ld = ldin;
    int64_t A = 1;
    int k0 = 0;
    if (fuse) {
        Mode2Args a{};
        a.D1 = Q->dCT[0]; a.D2 = Q->dCT[1]; a.D1T = Q->dC[0]; a.D2T = Q->dC[1];
        a.nin1 = hs.nt[0]; a.nin2 = hs.nt[1]; a.nout1 = hs.n[0]; a.nout2 = hs.n[1];
        a.Clo = 1;
        for (int j = 2; j < d; ++j) a.Clo *= hs.nt[j];
        a.nvec = nb;
        a.in = in; a.in_ldj = ldin;
        a.nsplit = nsplit; a.in_split = in_split; a.in_w = in_w; a.in_scale = in_scale;
        a.out_lo = nullptr; a.out_w = nullptr;
        if (d == 2) {
            a.out = y; a.out_ldj = ldy;
        } else {
            a.out = T0; a.out_ldj = int64_t(hs.n[0]) * hs.n[1] * a.Clo;
        }
        launch_mode2(a, in_f32, 0, s);
        cur = T0;
        cur_ld = int64_t(hs.n[0]) * hs.n[1] * a.Clo;
        A = int64_t(hs.n[0]) * hs.n[1];
        k0 = 2;
    }
    for (int k = k0; k < d; ++k) {
        ModeSpec m;
        m.D = Q->dCT[k];
        m.DT = Q->dC[k];
        m.in = cur;
        m.in_ldj = cur_ld;
        m.A = A;
        m.nin = hs.nt[k];
        m.nout = hs.n[k];
        m.Clo = 1;
        for (int j = k + 1; j < d; ++j) m.Clo *= hs.nt[j];
        m.nvec = nb;
        if (k == 0) m.in_f32 = in_f32;
        if (k == d - 1) {
            m.out = y;
            m.out_ldj = ldy;
        } else {
            m.out = (cur == T0) ? T1 : T0;
            m.out_ldj = A * hs.n[k] * m.Clo;
        }
        launch_mode(m, s);
        A *= hs.n[k];
        cur = m.out;
        cur_ld = m.out_ldj;
    }
}

}  // namespace

// One chunk (<= kBW columns) of Algorithm 1: x (N x nb, ld ldx) -> y (N x nb, ld ldy).
// Forward stages 1-4: C_k along each direction, J on the way out of the last one;
// stage 5 (its output rows scaled by sigma^2 J); backward stages 6-9: C_k^T per
// direction.  For d >= 2 the first two directions of each side are one launch (the
// backward one also adds the stage-5 split partials and applies sigma^2 J): 2d - 1
// launches for d >= 2, otherwise one per direction, stage 5 and its split sums.  With
// several patches the Kronecker stages run patch by patch on the patch's rows, around one
// stage 5 over the points of all patches (Sec. 3.6).
kl_status apply_chunk(kl_problem *P, int precision, int nb, const double *x, int64_t ldx,
                      double *y, int64_t ldy, hipStream_t s, const Workspace *wsp) {
    const Workspace &ws = wsp ? *wsp : P->ws;
    const bool lo = precision != KL_F64;
    void *Y5 = stage5_input(ws, precision);
    void *Y5lo = precision == KL_BF16X3 ? static_cast<void *>(static_cast<__bf16 *>(Y5) + P->Ntpad * kBW) : nullptr;
    const int y5_kind = precision == KL_F32 ? 1 : (precision == KL_BF16 || precision == KL_BF16X3) ? 2 : 0;
    const size_t y5_elem = y5_kind == 0 ? 8 : y5_kind == 1 ? 4 : 2;
    const size_t z_elem = lo ? 4 : 8;
    const bool fuse = fused_directions(P, nb);
    // ---- stages 1-4 ---------------------------------------------------------------------
    for (int i = 0; i < patch_count(P); ++i) {
        const int64_t toff = patch_toff(P, i);
        forward_patch(patch_of(P, i), patch_of(P, i)->dC, patch_of(P, i)->dCT, fuse, y5_kind, nb,
                      x + patch_noff(P, i), ldx,
                      static_cast<char *>(Y5) + toff * y5_elem,
                      Y5lo ? static_cast<void *>(static_cast<char *>(Y5lo) + toff * y5_elem) : nullptr,
                      P->Ntpad, P->dJ + toff, ws.T0, ws.T1, s);
    }
    // ---- stage 5, its output scaled by sigma^2 J (or left as split partials) ------------
    const int nsplit = timed_stage5(P, ws, precision, Y5, P->dJ, P->sigma2, s, fuse);
    // ---- stages 6-9 ---------------------------------------------------------------------
    for (int i = 0; i < patch_count(P); ++i) {
        const int64_t toff = patch_toff(P, i);
        const bool parts = fuse && nsplit > 1;
        const void *in = static_cast<const char *>(parts ? ws.Z5 : ws.Zf) + toff * z_elem;
        backward_patch(patch_of(P, i), fuse, lo, nb, in, P->Ntpad, parts ? nsplit : 1,
                       parts ? P->Ntpad * kBW : 0, parts ? P->dJ + toff : nullptr, parts ? P->sigma2 : 1.0,
                       y + patch_noff(P, i), ldy, ws.T0, ws.T1, s);
    }
    return hip_check(hipGetLastError(), "kernel launch");
}

// v = L^{-T} v' (Sec. 4.1) for one patch Q: its N_Q rows of x (ld ldx), tmp (ld ldt) as
// the ping-pong buffer.
static void coefficients_patch(const kl_problem *Q, double *x, int64_t ldx, int nvec, double *tmp, int64_t ldt,
                        hipStream_t s) {
    const HostSetup &hs = Q->hs;
    const int d = hs.d;
    const int64_t N = hs.N;
    for (int c0 = 0; c0 < nvec; c0 += kBW) {
        const int nb = std::min(kBW, nvec - c0);
        double *cur = x + int64_t(c0) * ldx;
        int64_t cur_ld = ldx;
        int64_t A = 1;
        for (int k = 0; k < d; ++k) {
            ModeSpec m;
            m.D = Q->dLT[k];
            m.DT = Q->dL1[k];
            m.in = cur;
            m.in_ldj = cur_ld;
            m.A = A;
            m.nin = m.nout = hs.n[k];
            m.Clo = 1;
            for (int j = k + 1; j < d; ++j) m.Clo *= hs.n[j];
            m.nvec = nb;
            // x -> tmp -> x -> ... (never in place); an odd d ends in tmp and is copied back
            const bool to_tmp = (k % 2) == 0;
            m.out = to_tmp ? tmp : x + int64_t(c0) * ldx;
            m.out_ldj = to_tmp ? ldt : ldx;
            launch_mode(m, s);
            A *= hs.n[k];
            cur = static_cast<double *>(m.out);
            cur_ld = m.out_ldj;
        }
        if (cur != x + int64_t(c0) * ldx) launch_copy_cols(cur, cur_ld, x + int64_t(c0) * ldx, ldx, N, nb, s);
    }
}


// v = L^{-T} v' one direction at a time (mode products with the upper triangular
// factors L_k^{-T}), patch by patch on the patch's rows; the result lands back in x.
void launch_to_coefficients(const kl_problem *P, double *x, int64_t ldx, int nvec, double *tmp, hipStream_t s) {
    for (int i = 0; i < patch_count(P); ++i) {
        const int64_t off = patch_noff(P, i);
        coefficients_patch(patch_of(P, i), x + off, ldx, nvec, tmp + off, P->hs.N, s);
    }
}

}  // namespace kl

using namespace kl;

extern "C" {

kl_status kl_setup_host(const kl_desc *desc, kl_problem **out) {
    if (!desc || !out) { set_error("kl_setup_host: NULL argument"); return KL_EINVAL; }
    kl_problem *P = new (std::nothrow) kl_problem();
    if (!P) { set_error("kl_setup_host: host allocation failed"); return KL_ENOMEM; }
    kl_status st = build_host_setup(*desc, P->hs);
    if (st != KL_OK) { delete P; return st; }
    P->host_only = true;
    *out = P;
    return KL_OK;
}

kl_status kl_setup(const kl_desc *desc, void *stream, kl_problem **out) {
    return kl::setup_problem(desc, true, static_cast<hipStream_t>(stream), out);
}

kl_status kl_setup_patches(int32_t npatch, const kl_desc *patches, void *stream, kl_problem **out) {
    return kl::setup_patches(npatch, patches, static_cast<hipStream_t>(stream), out);
}

kl_status kl_patch_info(const kl_problem *P, int32_t i, int64_t *N, int64_t *Ntilde, int64_t *dof_offset,
                        int64_t *point_offset) {
    if (!P) { set_error("kl_patch_info: NULL handle"); return KL_EINVAL; }
    if (i < 0 || i >= patch_count(P)) { set_error("kl_patch_info: patch index out of range"); return KL_EINVAL; }
    const kl_problem *Q = patch_of(P, i);
    if (N) *N = Q->hs.N;
    if (Ntilde) *Ntilde = Q->hs.Nt;
    if (dof_offset) *dof_offset = patch_noff(P, i);
    if (point_offset) *point_offset = patch_toff(P, i);
    return KL_OK;
}

int32_t kl_patch_count(const kl_problem *P) { return P ? patch_count(P) : 0; }

}  // extern "C"

namespace kl {

namespace {

// Covariance parameters, the padded point count, the scaled points and J on the device.
kl_status init_points(kl_problem *P, const kl_desc &desc, hipStream_t s) {
    const HostSetup &hs = P->hs;
    P->cov_kind = desc.cov_kind;
    P->sigma2 = desc.sigma2;
    for (int k = 0; k < 3; ++k) P->ell[k] = k < hs.d ? desc.corr_len[k] : 1.0;
    P->Ntpad = (hs.Nt + kPad - 1) / kPad * kPad;
    int dev = 0;
    kl_status st = hip_check(hipGetDevice(&dev), "hipGetDevice");
    if (st != KL_OK) return st;
    int ncu = 0;
    if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && ncu > 0)
        P->n_cu = ncu;
    const int64_t Np = P->Ntpad;
    std::vector<double> jpad(size_t(Np), 0.0);
    for (int64_t p = 0; p < hs.Nt; ++p) jpad[p] = hs.J[p];
    if ((st = dev_alloc(&P->dX64, size_t(hs.d) * Np, "hipMalloc X64")) != KL_OK ||
        (st = dev_alloc(&P->dX32, size_t(hs.d) * Np, "hipMalloc X32")) != KL_OK ||
        (st = dev_alloc(&P->dJ, jpad.size(), "hipMalloc J")) != KL_OK || (st = upload_points(P, s)) != KL_OK ||
        (st = hip_check(hipMemcpyAsync(P->dJ, jpad.data(), jpad.size() * 8, hipMemcpyHostToDevice, s), "copy J")) !=
            KL_OK)
        return st;
    return hip_check(hipStreamSynchronize(s), "hipStreamSynchronize");     // jpad dies here
}

// The factors of a single patch: C_k, C_k^T, E_k, E_k^T, L_k^{-T} and its transpose.
kl_status upload_factors(kl_problem *P, hipStream_t s) {
    const HostSetup &hs = P->hs;
    std::vector<double> CT[3], ET[3], L1[3];
    auto upload = [&](double **dst, const std::vector<double> &src, const char *what) -> kl_status {
        kl_status st2 = dev_alloc(dst, src.size(), what);
        if (st2 != KL_OK) return st2;
        return hip_check(hipMemcpyAsync(*dst, src.data(), src.size() * 8, hipMemcpyHostToDevice, s), what);
    };
    kl_status st = KL_OK;
    for (int k = 0; k < hs.d && st == KL_OK; ++k) {
        const int n = hs.n[k], nt = hs.nt[k];
        CT[k].resize(size_t(n) * nt);
        ET[k].resize(size_t(n) * nt);
        for (int i = 0; i < nt; ++i)
            for (int j = 0; j < n; ++j) {
                CT[k][size_t(j) * nt + i] = hs.C[k][size_t(i) * n + j];
                // evaluation factor of the truncated expansion (kl_kle_field)
                ET[k][size_t(j) * nt + i] = hs.E[k][size_t(i) * n + j];
            }
        L1[k].resize(size_t(n) * n);
        for (int i = 0; i < n; ++i)
            for (int j = 0; j < n; ++j) L1[k][size_t(j) * n + i] = hs.LT[k][size_t(i) * n + j];
        if ((st = upload(&P->dC[k], hs.C[k], "C")) != KL_OK || (st = upload(&P->dCT[k], CT[k], "CT")) != KL_OK ||
            (st = upload(&P->dE[k], hs.E[k], "E")) != KL_OK || (st = upload(&P->dET[k], ET[k], "ET")) != KL_OK ||
            (st = upload(&P->dLT[k], hs.LT[k], "LT")) != KL_OK || (st = upload(&P->dL1[k], L1[k], "L1")) != KL_OK)
            break;
    }
    kl_status st2 = hip_check(hipStreamSynchronize(s), "hipStreamSynchronize");   // staging dies here
    return st != KL_OK ? st : st2;
}

// The apply workspace: Kronecker ping-pong buffers for `tmax` rows per column, the stage-5
// inputs in every precision (padding rows zeroed once, never written), split partials
// and the finished stage-5 output.
kl_status alloc_workspace(kl_problem *P, int64_t tmax, hipStream_t s) {
    const int64_t Np = P->Ntpad;
    // split partials: at most 64 splits, at most ~512 MB
    P->ws.max_split = int(std::max<int64_t>(1, std::min<int64_t>(
        std::min<int64_t>(64, Np / 64), (int64_t(512) << 20) / (Np * kBW * int64_t(sizeof(double))))));
    P->ws.t_elems = size_t(tmax) * kBW;
    P->ws.y5_bytes = size_t(Np) * kBW * sizeof(double);
    P->ws.z5_bytes = size_t(P->ws.max_split) * Np * kBW * sizeof(double);
    kl_status st;
    if ((st = dev_alloc(&P->ws.T0, P->ws.t_elems, "hipMalloc T0")) != KL_OK ||
        (st = dev_alloc(&P->ws.T1, P->ws.t_elems, "hipMalloc T1")) != KL_OK ||
        (st = dev_alloc(reinterpret_cast<char **>(&P->ws.Y5d), P->ws.y5_bytes, "hipMalloc Y5")) != KL_OK ||
        (st = dev_alloc(reinterpret_cast<char **>(&P->ws.Y5f), P->ws.y5_bytes / 2, "hipMalloc Y5")) != KL_OK ||
        (st = dev_alloc(reinterpret_cast<char **>(&P->ws.Y5b), P->ws.y5_bytes / 2, "hipMalloc Y5")) != KL_OK ||
        (st = hip_check(hipMemsetAsync(P->ws.Y5d, 0, P->ws.y5_bytes, s), "memset Y5")) != KL_OK ||
        (st = hip_check(hipMemsetAsync(P->ws.Y5f, 0, P->ws.y5_bytes / 2, s), "memset Y5")) != KL_OK ||
        (st = hip_check(hipMemsetAsync(P->ws.Y5b, 0, P->ws.y5_bytes / 2, s), "memset Y5")) != KL_OK ||
        (st = dev_alloc(reinterpret_cast<char **>(&P->ws.Z5), P->ws.z5_bytes, "hipMalloc Z5")) != KL_OK ||
        (st = dev_alloc(reinterpret_cast<char **>(&P->ws.Zf), size_t(Np) * kBW * sizeof(double), "hipMalloc Zf")) !=
            KL_OK)
        return st;
    return hip_check(hipStreamSynchronize(s), "hipStreamSynchronize");
}

// Size limits of the kernels for one patch: per-direction Kronecker sizes, and the rows of
// a 32-vector chunk indexed with 32-bit integers.
kl_status check_patch_sizes(const HostSetup &hs) {
    for (int k = 0; k < hs.d; ++k)
        if (!mode_fits(hs.n[k], hs.nt[k]) || !mode_fits(hs.nt[k], hs.n[k])) {
            set_error("kl_setup: more than 4096 basis functions in one direction are not supported");
            return KL_EINVAL;
        }
    if (max_intermediate(hs) * kBW >= (int64_t(1) << 31)) {
        set_error("kl_setup: grid too large (intermediate size x 32 must stay below 2^31)");
        return KL_EINVAL;
    }
    return KL_OK;
}

}  // namespace

kl_status setup_problem(const kl_desc *desc, bool workspace, hipStream_t s, kl_problem **out) {
    const auto t0 = std::chrono::steady_clock::now();
    if (!desc || !out) { set_error("kl_setup: NULL argument"); return KL_EINVAL; }
    kl_problem *P = new (std::nothrow) kl_problem();
    if (!P) { set_error("kl_setup: host allocation failed"); return KL_ENOMEM; }
    kl_status st = build_host_setup(*desc, P->hs);
    if (st == KL_OK) st = check_patch_sizes(P->hs);
    if (st != KL_OK) { delete P; return st; }
    if ((st = init_points(P, *desc, s)) != KL_OK || (st = upload_factors(P, s)) != KL_OK ||
        (workspace && (st = alloc_workspace(P, max_intermediate(P->hs), s)) != KL_OK)) {
        free_problem(P);
        return st;
    }
    P->t_setup = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    *out = P;
    return KL_OK;
}

// Several patches (Sec. 3.6): one factor-only problem per patch, and the union's points,
// J, stage-5 buffers and workspace in the returned problem.
kl_status setup_patches(int npatch, const kl_desc *descs, hipStream_t s, kl_problem **out) {
    const auto t0 = std::chrono::steady_clock::now();
    if (!descs || !out || npatch < 1) { set_error("kl_setup_patches: NULL argument or npatch < 1"); return KL_EINVAL; }
    const kl_desc &d0 = descs[0];
    for (int i = 1; i < npatch; ++i) {
        const kl_desc &di = descs[i];
        bool same = di.dim == d0.dim && di.cov_kind == d0.cov_kind && di.sigma2 == d0.sigma2;
        for (int k = 0; k < d0.dim && k < 3 && same; ++k) same = di.corr_len[k] == d0.corr_len[k];
        if (!same) {
            set_error("kl_setup_patches: the patches must share dim and the covariance (kind, sigma2, corr_len)");
            return KL_EINVAL;
        }
    }
    kl_problem *P = new (std::nothrow) kl_problem();
    if (!P) { set_error("kl_setup_patches: host allocation failed"); return KL_ENOMEM; }
    kl_status st = KL_OK;
    HostSetup &hs = P->hs;
    P->noff.push_back(0);
    P->toff.push_back(0);
    for (int i = 0; i < npatch && st == KL_OK; ++i) {
        kl_problem *Q = nullptr;
        st = setup_problem(&descs[i], false, s, &Q);
        if (st != KL_OK) {
            set_error("kl_setup_patches: patch " + std::to_string(i) + ": " + kl_last_error());
            break;
        }
        P->patches.push_back(Q);
        P->noff.push_back(P->noff.back() + Q->hs.N);
        P->toff.push_back(P->toff.back() + Q->hs.Nt);
        hs.X.insert(hs.X.end(), Q->hs.X.begin(), Q->hs.X.end());
        hs.J.insert(hs.J.end(), Q->hs.J.begin(), Q->hs.J.end());
    }
    if (st == KL_OK) {
        // totals; the per-direction sizes reported by kl_info are those of patch 0
        const HostSetup &h0 = P->patches[0]->hs;
        hs.d = h0.d;
        for (int k = 0; k < 3; ++k) {
            hs.p[k] = h0.p[k]; hs.pt[k] = h0.pt[k]; hs.ne[k] = h0.ne[k]; hs.net[k] = h0.net[k];
            hs.n[k] = h0.n[k]; hs.nt[k] = h0.nt[k];
        }
        hs.N = P->noff.back();
        hs.Nt = P->toff.back();
        if ((hs.Nt + kPad) * kBW >= (int64_t(1) << 31) || hs.N * kBW >= (int64_t(1) << 31)) {
            set_error("kl_setup_patches: too many points (points x 32 must stay below 2^31)");
            st = KL_EINVAL;
        }
    }
    if (st == KL_OK) st = init_points(P, d0, s);
    if (st == KL_OK) st = alloc_workspace(P, problem_max_intermediate(P), s);
    if (st != KL_OK) { free_problem(P); return st; }
    P->t_setup = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    *out = P;
    return KL_OK;
}

void destroy_problem(kl_problem *P) { free_problem(P); }

}  // namespace kl

extern "C" {

kl_status kl_info(const kl_problem *P, int64_t *N, int64_t *Ntilde, int32_t *n, int32_t *nt) {
    if (!P) { set_error("kl_info: NULL handle"); return KL_EINVAL; }
    if (N) *N = P->hs.N;
    if (Ntilde) *Ntilde = P->hs.Nt;
    for (int k = 0; k < 3; ++k) {
        if (n) n[k] = k < P->hs.d ? P->hs.n[k] : 1;
        if (nt) nt[k] = k < P->hs.d ? P->hs.nt[k] : 1;
    }
    return KL_OK;
}

kl_status kl_set_cov(kl_problem *P, int32_t cov_kind, double sigma2, const double *corr_len) {
    if (!P || P->host_only) { set_error("kl_set_cov: NULL or host-only handle"); return KL_EINVAL; }
    if (!corr_len) { set_error("kl_set_cov: NULL corr_len"); return KL_EINVAL; }
    if (cov_kind < KL_COV_EXP || cov_kind > KL_COV_LIN) { set_error("kl_set_cov: unknown covariance kind"); return KL_EINVAL; }
    if (!(sigma2 > 0.0) || !std::isfinite(sigma2)) { set_error("kl_set_cov: sigma2 must be positive"); return KL_EINVAL; }
    for (int k = 0; k < P->hs.d; ++k)
        if (!(corr_len[k] > 0.0) || !std::isfinite(corr_len[k])) {
            set_error("kl_set_cov: correlation lengths must be positive");
            return KL_EINVAL;
        }
    // the device may still read the old points: wait for outstanding work first
    kl_status st = hip_check(hipDeviceSynchronize(), "hipDeviceSynchronize");
    if (st != KL_OK) return st;
    P->cov_kind = cov_kind;
    P->sigma2 = sigma2;
    for (int k = 0; k < 3; ++k) P->ell[k] = k < P->hs.d ? corr_len[k] : 1.0;
    return upload_points(P, nullptr);
}

kl_status kl_apply(kl_problem *P, int32_t precision, int32_t nvec, const double *x, int64_t ldx,
                   double *y, int64_t ldy, void *stream) {
    if (!P || P->host_only) { set_error("kl_apply: NULL or host-only handle"); return KL_EINVAL; }
    if (!valid_precision(precision)) { set_error("kl_apply: unsupported precision"); return KL_EINVAL; }
    if (nvec < 0) { set_error("kl_apply: nvec < 0"); return KL_EINVAL; }
    if (nvec == 0) return KL_OK;
    if (!x || !y) { set_error("kl_apply: NULL vector"); return KL_EINVAL; }
    if (ldx < P->hs.N || ldy < P->hs.N) { set_error("kl_apply: leading dimension < N"); return KL_EINVAL; }
    const char *xb = reinterpret_cast<const char *>(x), *yb = reinterpret_cast<const char *>(y);
    const size_t xbytes = size_t(ldx) * (nvec - 1) * 8 + size_t(P->hs.N) * 8;
    const size_t ybytes = size_t(ldy) * (nvec - 1) * 8 + size_t(P->hs.N) * 8;
    if (xb < yb + ybytes && yb < xb + xbytes) { set_error("kl_apply: x and y overlap"); return KL_EINVAL; }
    hipStream_t s = static_cast<hipStream_t>(stream);
    for (int c0 = 0; c0 < nvec; c0 += kBW) {
        const int nb = std::min(kBW, nvec - c0);
        kl_status st = apply_chunk(P, precision, nb, x + int64_t(c0) * ldx, ldx, y + int64_t(c0) * ldy,
                                   ldy, s);
        if (st != KL_OK) return st;
    }
    return KL_OK;
}

kl_status kl_stage5(kl_problem *P, int32_t precision, int32_t nvec, const double *y, int64_t ldy,
                    double *z, int64_t ldz, void *stream) {
    if (!P || P->host_only) { set_error("kl_stage5: NULL or host-only handle"); return KL_EINVAL; }
    if (!valid_precision(precision)) { set_error("kl_stage5: unsupported precision"); return KL_EINVAL; }
    if (nvec < 0) { set_error("kl_stage5: nvec < 0"); return KL_EINVAL; }
    if (nvec == 0) return KL_OK;
    if (!y || !z) { set_error("kl_stage5: NULL vector"); return KL_EINVAL; }
    if (ldy < P->hs.Nt || ldz < P->hs.Nt) { set_error("kl_stage5: leading dimension < Ntilde"); return KL_EINVAL; }
    hipStream_t s = static_cast<hipStream_t>(stream);
    for (int c0 = 0; c0 < nvec; c0 += kBW) {
        const int nb = std::min(kBW, nvec - c0);
        void *Y5 = stage5_input(P->ws, precision);
        launch_pack_stage5(precision, y + int64_t(c0) * ldy, ldy, P->hs.Nt, nb, P->Ntpad, Y5, s);
        const int nsplit = timed_stage5(P, P->ws, precision, Y5, nullptr, 1.0, s);
        (void)nsplit;
        launch_unpack_stage5(precision, P->ws.Zf, 1, P->Ntpad, P->hs.Nt, nb, P->sigma2,
                             z + int64_t(c0) * ldz, ldz, s);
        kl_status st = hip_check(hipGetLastError(), "kernel launch");
        if (st != KL_OK) return st;
    }
    return KL_OK;
}

kl_status kl_apply_config(kl_problem *P, int32_t fuse_directions, int32_t *fused_out) {
    if (!P || P->host_only) { set_error("kl_apply_config: NULL or host-only handle"); return KL_EINVAL; }
    if (fuse_directions != 0 && fuse_directions != 1) {
        set_error("kl_apply_config: fuse_directions must be 0 or 1");
        return KL_EINVAL;
    }
    P->fuse_dirs = fuse_directions != 0;
    if (fused_out) *fused_out = fused_directions(P, kBW) ? 1 : 0;
    return KL_OK;
}

kl_status kl_stage5_config(kl_problem *P, int32_t precision, int32_t rb, int32_t nsplit,
                           int32_t *rb_out, int32_t *nsplit_out) {
    if (!P || P->host_only) { set_error("kl_stage5_config: NULL or host-only handle"); return KL_EINVAL; }
    if (!valid_precision(precision)) { set_error("kl_stage5_config: bad precision"); return KL_EINVAL; }
    if (rb != 0 && rb != 1 && rb != 2 && rb != 4 && rb != 8) {
        set_error("kl_stage5_config: rb must be 0, 1, 2, 4 or 8");
        return KL_EINVAL;
    }
    if (nsplit < -1 || nsplit > 64) { set_error("kl_stage5_config: nsplit must be in -1..64"); return KL_EINVAL; }
    if (rb > 0) P->s5_rb[precision] = rb;
    if (nsplit >= 0) P->s5_split[precision] = nsplit;
    const int rbs = P->s5_rb[precision];
    const int rbe = (rbs == 1 || rbs == 4 || (rbs == 8 && precision == KL_F32)) ? rbs : 2;
    int64_t lchunk;
    const int ns = stage5_splits(P->Ntpad, stage5_rows_per_wg(precision, rbe), P->n_cu, P->ws.max_split,
                                 P->s5_split[precision], &lchunk);
    if (rb_out) *rb_out = precision == KL_F64 ? 4 : rbe;
    if (nsplit_out) *nsplit_out = ns;
    return KL_OK;
}

kl_status kl_stage5_symmetric(kl_problem *P, int32_t precision, int32_t on, int32_t chunk, int32_t *items_out) {
    if (!P || P->host_only) { set_error("kl_stage5_symmetric: NULL or host-only handle"); return KL_EINVAL; }
    if (precision != KL_F64 && precision != KL_BF16 && precision != KL_BF16X3) {
        set_error("kl_stage5_symmetric: the symmetric form exists for KL_F64, KL_BF16 and KL_BF16X3");
        return KL_EINVAL;
    }
    if (on != 0 && on != 1) { set_error("kl_stage5_symmetric: on must be 0 or 1"); return KL_EINVAL; }
    if (chunk < 0 || chunk > (1 << 20)) { set_error("kl_stage5_symmetric: chunk must be >= 0"); return KL_EINVAL; }
    if (!on) {
        P->s5_sym[precision] = false;
        if (items_out) *items_out = 0;
        return KL_OK;
    }
    Workspace &ws = P->ws;
    const SymPlan pl = sym_plan(P->Ntpad, P->n_cu, chunk);
    if (!ws.symF || pl.chunk != ws.sym_chunk) {
        hipStream_t s = nullptr;
        kl_status st = hip_check(hipDeviceSynchronize(), "hipDeviceSynchronize");   // no launch still reads them
        if (st != KL_OK) return st;
        hipFree(ws.symF);
        hipFree(ws.symO);
        hipFree(ws.symTab);
        ws.symF = ws.symO = nullptr;
        ws.symTab = nullptr;
        ws.sym_chunk = 0;
        const size_t tab = pl.items.size() * sizeof(SymItem) + pl.o_first.size() * sizeof(int);
        std::vector<char> host(tab);
        std::memcpy(host.data(), pl.items.data(), pl.items.size() * sizeof(SymItem));
        std::memcpy(host.data() + pl.items.size() * sizeof(SymItem), pl.o_first.data(), pl.o_first.size() * sizeof(int));
        if ((st = dev_alloc(reinterpret_cast<char **>(&ws.symF), sym_f_bytes(pl), "hipMalloc symmetric partials")) !=
                KL_OK ||
            (st = dev_alloc(reinterpret_cast<char **>(&ws.symO), sym_o_bytes(pl), "hipMalloc symmetric partials")) !=
                KL_OK ||
            (st = dev_alloc(reinterpret_cast<char **>(&ws.symTab), tab, "hipMalloc symmetric plan")) != KL_OK ||
            (st = hip_check(hipMemcpyAsync(ws.symTab, host.data(), tab, hipMemcpyHostToDevice, s), "copy plan")) !=
                KL_OK ||
            (st = hip_check(hipStreamSynchronize(s), "hipStreamSynchronize")) != KL_OK) {
            hipFree(ws.symF);
            hipFree(ws.symO);
            hipFree(ws.symTab);
            ws.symF = ws.symO = nullptr;
            ws.symTab = nullptr;
            for (bool &b : P->s5_sym) b = false;
            return st;
        }
        ws.sym_items = pl.n_items;
        ws.sym_NB = pl.NB;
        ws.sym_chunk = pl.chunk;
        ws.sym_grid = std::min(pl.n_items, P->n_cu);
    }
    P->s5_sym[precision] = true;
    if (items_out) *items_out = ws.sym_items;
    return KL_OK;
}

kl_status kl_get_points(const kl_problem *P, double *X, double *J) {
    if (!P) { set_error("kl_get_points: NULL handle"); return KL_EINVAL; }
    if (X) std::memcpy(X, P->hs.X.data(), P->hs.X.size() * sizeof(double));
    if (J) std::memcpy(J, P->hs.J.data(), P->hs.J.size() * sizeof(double));
    return KL_OK;
}

kl_status kl_get_factor(const kl_problem *P, int32_t k, double *C) {
    if (!P) { set_error("kl_get_factor: NULL handle"); return KL_EINVAL; }
    if (k < 0 || k >= P->hs.d) { set_error("kl_get_factor: direction out of range"); return KL_EINVAL; }
    if (!P->patches.empty()) { set_error("kl_get_factor: a problem of several patches has one factor per patch"); return KL_EINVAL; }
    if (C) std::memcpy(C, P->hs.C[k].data(), P->hs.C[k].size() * sizeof(double));
    return KL_OK;
}

kl_status kl_profile_enable(kl_problem *P, int32_t enable) {
    if (!P || P->host_only) { set_error("kl_profile_enable: NULL or host-only handle"); return KL_EINVAL; }
    const size_t pool = 2 * 8192;
    if (enable && P->prof_ev.size() < pool) {
        P->prof_ev.reserve(pool);
        while (P->prof_ev.size() < pool) {
            hipEvent_t e;
            kl_status st = hip_check(hipEventCreateWithFlags(&e, hipEventDisableSystemFence), "hipEventCreate");
            if (st != KL_OK) return st;
            P->prof_ev.push_back(e);
        }
    }
    P->prof_on = enable != 0;
    P->prof_used = 0;
    P->prof_prec.clear();
    P->prof_prec.reserve(pool / 2);
    for (int p = 0; p < 4; ++p) { P->prof_count[p] = 0; P->prof_ms[p] = 0.0; }
    return KL_OK;
}

kl_status kl_profile_read(kl_problem *P, int64_t *count, double *ms) {
    if (!P || P->host_only) { set_error("kl_profile_read: NULL or host-only handle"); return KL_EINVAL; }
    for (size_t i = 0; i < P->prof_prec.size(); ++i) {
        kl_status st = hip_check(hipEventSynchronize(P->prof_ev[2 * i + 1]), "hipEventSynchronize");
        if (st != KL_OK) return st;
        float t = 0.f;
        if ((st = hip_check(hipEventElapsedTime(&t, P->prof_ev[2 * i], P->prof_ev[2 * i + 1]),
                            "hipEventElapsedTime")) != KL_OK)
            return st;
        P->prof_count[P->prof_prec[i]] += 1;
        P->prof_ms[P->prof_prec[i]] += t;
    }
    P->prof_prec.clear();
    P->prof_used = 0;
    for (int p = 0; p < 4; ++p) {
        if (count) count[p] = P->prof_count[p];
        if (ms) ms[p] = P->prof_ms[p];
    }
    return KL_OK;
}

kl_status kl_destroy(kl_problem *P) {
    free_problem(P);
    return KL_OK;
}

const char *kl_last_error(void) { return g_error.c_str(); }

}  // extern "C"
