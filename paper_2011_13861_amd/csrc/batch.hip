// Many problems of uneven size in one apply (Algorithm 1 for each of them).
//
// A batch keeps one kl_problem per member for the setup data (composed factors C_k,
// points, J) and packs everything the apply touches into arenas indexed by per-problem
// offsets: the Kronecker intermediates, the stage-5 inputs and outputs per precision
// and the split partials.  One apply of the whole batch is 2d + 3 launches whatever the
// number of problems:
//   d forward directions (one launch each, workgroups mapped to problems by a prefix
//   table), a reset of the work-queue counter, the persistent stage-5 kernel that takes
//   (problem, row tile, l-split) items longest first, the split sums, and d backward
//   directions.
// The launches are captured once per precision into a HIP graph.  Every kernel reads
// its per-problem arguments and the active flags from device tables, so a replay with
// other vectors, other column counts (<= 32 per problem) or another set of active
// problems only rewrites those tables (one host-to-device copy) before the replay.
#include <algorithm>
#include <cstring>
#include <new>
#include <numeric>
#include <sstream>
#include <vector>

#include "kl_internal.h"

namespace kl {
namespace {

kl_status bhip(hipError_t e, const char *what) {
    if (e == hipSuccess) return KL_OK;
    std::ostringstream os;
    os << "kl_batch: " << what << ": " << hipGetErrorString(e);
    set_error(os.str());
    return e == hipErrorOutOfMemory ? KL_ENOMEM : KL_EHIP;
}

int prec_index(int precision) { return precision == KL_F64 ? 0 : 1; }

struct BatchPlan {
    bool ready = false;
    int rb = 2;
    int64_t lchunk = 0;
    // per-direction variant selectors and workgroup prefix tables (device, n + 1 entries)
    ModeSpec fwd_kind[3], bwd_kind[3];
    int64_t *fwd_pre[3] = {nullptr, nullptr, nullptr}, *bwd_pre[3] = {nullptr, nullptr, nullptr};
    int64_t fwd_total[3] = {0, 0, 0}, bwd_total[3] = {0, 0, 0};
    // base arguments (host) with the per-call fields left empty
    std::vector<ModeArgs> fwd_base[3], bwd_base[3];
    // stage 5
    S5Prob *s5 = nullptr;
    S5Item *items = nullptr;
    int n_items = 0, grid = 0;
    RedProb *red = nullptr;
    int nred = 0;
    int64_t total4 = 0;
    void *Z5 = nullptr;
    std::vector<int> nsplit;
    hipGraphExec_t exec = nullptr;
};

}  // namespace
}  // namespace kl

struct kl_batch {
    int n = 0, d = 0, n_cu = 256;
    std::vector<kl_problem *> probs;
    std::vector<int64_t> rowoff;          // sum of N over the preceding problems
    int64_t Ntot = 0;
    std::vector<int64_t> toff, poff;      // Kronecker arena / padded-grid arena offsets
    double *T0 = nullptr, *T1 = nullptr;
    void *Y5[2] = {nullptr, nullptr};     // stage-5 inputs: [0] FP64, [1] FP32
    void *Zf[2] = {nullptr, nullptr};     // stage-5 outputs
    int *counter = nullptr;
    // per-call tables: 2d x n ModeArgs, then n active flags (device + pinned staging)
    char *dyn = nullptr, *dyn_host = nullptr;
    size_t dyn_bytes = 0;
    hipEvent_t dyn_done = nullptr;
    hipStream_t stream = nullptr;         // capture stream, also used by kl_eigs_batch
    int cfg_rb[2] = {2, 2};
    int64_t cfg_lchunk[2] = {0, 0};
    kl::BatchPlan plan[2];
};

namespace kl {
namespace {

ModeArgs *dyn_fwd(kl_batch *B, int k) { return reinterpret_cast<ModeArgs *>(B->dyn) + size_t(k) * B->n; }
ModeArgs *dyn_bwd(kl_batch *B, int k) { return reinterpret_cast<ModeArgs *>(B->dyn) + size_t(B->d + k) * B->n; }
int *dyn_active(kl_batch *B) {
    return reinterpret_cast<int *>(B->dyn + sizeof(ModeArgs) * size_t(2 * B->d) * B->n);
}

void free_plan(BatchPlan &p) {
    if (p.exec) (void)hipGraphExecDestroy(p.exec);
    for (int k = 0; k < 3; ++k) {
        (void)hipFree(p.fwd_pre[k]);
        (void)hipFree(p.bwd_pre[k]);
        p.fwd_pre[k] = p.bwd_pre[k] = nullptr;
    }
    (void)hipFree(p.s5);
    (void)hipFree(p.items);
    (void)hipFree(p.red);
    (void)hipFree(p.Z5);
    p = BatchPlan();
}

void free_batch(kl_batch *B) {
    if (!B) return;
    if (B->stream) (void)hipStreamSynchronize(B->stream);
    for (auto &p : B->plan) free_plan(p);
    for (kl_problem *P : B->probs) destroy_problem(P);
    (void)hipFree(B->T0);
    (void)hipFree(B->T1);
    for (int q = 0; q < 2; ++q) {
        (void)hipFree(B->Y5[q]);
        (void)hipFree(B->Zf[q]);
    }
    (void)hipFree(B->counter);
    (void)hipFree(B->dyn);
    if (B->dyn_host) (void)hipHostFree(B->dyn_host);
    if (B->dyn_done) (void)hipEventDestroy(B->dyn_done);
    if (B->stream) (void)hipStreamDestroy(B->stream);
    delete B;
}

// Largest l-range per split such that the queue holds at least four items per resident
// workgroup (so that the longest-first order can even out the tail), at least 512.
int64_t auto_lchunk(const kl_batch *B, int64_t rows_wg, int grid) {
    int64_t best = 512;
    for (int64_t lc = 512; lc <= (int64_t(1) << 20); lc *= 2) {
        int64_t items = 0;
        for (const kl_problem *P : B->probs) items += (P->Ntpad / rows_wg) * ((P->Ntpad + lc - 1) / lc);
        if (items >= 4 * int64_t(grid)) best = lc;
        else break;
    }
    return best;
}

kl_status build_plan(kl_batch *B, int precision) {
    BatchPlan &pl = B->plan[prec_index(precision)];
    free_plan(pl);
    kl_status st;
    const int n = B->n, d = B->d;
    const int pi = prec_index(precision);
    const bool lo = precision != KL_F64;
    const size_t esz = lo ? sizeof(float) : sizeof(double);
    pl.rb = precision == KL_F64 ? 2 : B->cfg_rb[pi];
    const int64_t rows_wg = stage5_rows_per_wg(precision, pl.rb);
    pl.grid = stage5_batch_grid(precision, d, pl.rb, B->n_cu);
    pl.lchunk = B->cfg_lchunk[pi] > 0 ? B->cfg_lchunk[pi] : auto_lchunk(B, rows_wg, pl.grid);
    pl.lchunk = std::max<int64_t>(64, (pl.lchunk + 63) / 64 * 64);   // 64-point granule of the stage-5 staging
    // ---- Kronecker directions -----------------------------------------------------------
    for (int k = 0; k < d; ++k) {
        pl.fwd_base[k].resize(n);
        pl.bwd_base[k].resize(n);
    }
    std::vector<int64_t> fpre[3], bpre[3];
    for (int k = 0; k < d; ++k) {
        fpre[k].assign(n + 1, 0);
        bpre[k].assign(n + 1, 0);
    }
    for (int i = 0; i < n; ++i) {
        const kl_problem *P = B->probs[i];
        const HostSetup &hs = P->hs;
        double *T0 = B->T0 + B->toff[i], *T1 = B->T1 + B->toff[i];
        char *y5 = static_cast<char *>(B->Y5[pi]) + size_t(B->poff[i]) * esz;
        char *zf = static_cast<char *>(B->Zf[pi]) + size_t(B->poff[i]) * esz;
        // forward: x -> T -> ... -> Y5 (J applied on the way out)
        const void *cur = nullptr;
        int64_t cur_ld = 0, A = 1;
        for (int k = 0; k < d; ++k) {
            ModeSpec m;
            m.D = P->dC[k];
            m.DT = P->dCT[k];
            m.in = cur;
            m.in_ldj = cur_ld;
            m.A = A;
            m.nin = hs.n[k];
            m.nout = hs.nt[k];
            m.Clo = 1;
            for (int j = k + 1; j < d; ++j) m.Clo *= hs.n[j];
            m.nvec = kBW;
            if (k == d - 1) {
                m.out = y5;
                m.out_ldj = P->Ntpad;
                m.out_w = P->dJ;
                m.out_f32 = lo;
            } else {
                m.out = (k % 2 == 0) ? T0 : T1;
                m.out_ldj = A * hs.nt[k] * m.Clo;
            }
            if (i == 0) pl.fwd_kind[k] = m;
            pl.fwd_base[k][i] = mode_args(m);
            fpre[k][i + 1] = fpre[k][i] + mode_workgroups(m);
            A *= hs.nt[k];
            cur = m.out;
            cur_ld = m.out_ldj;
        }
        // backward: Zf (already scaled by sigma^2 J) -> T -> ... -> y
        cur = zf;
        cur_ld = P->Ntpad;
        A = 1;
        for (int k = 0; k < d; ++k) {
            ModeSpec m;
            m.D = P->dCT[k];
            m.DT = P->dC[k];
            m.in = cur;
            m.in_ldj = cur_ld;
            m.A = A;
            m.nin = hs.nt[k];
            m.nout = hs.n[k];
            m.Clo = 1;
            for (int j = k + 1; j < d; ++j) m.Clo *= hs.nt[j];
            m.nvec = kBW;
            if (k == 0) m.in_f32 = lo;
            if (k == d - 1) {
                m.out = nullptr;            // the caller's y, set per call
                m.out_ldj = 0;
            } else {
                m.out = (k % 2 == 0) ? T0 : T1;
                m.out_ldj = A * hs.n[k] * m.Clo;
            }
            if (i == 0) pl.bwd_kind[k] = m;
            pl.bwd_base[k][i] = mode_args(m);
            bpre[k][i + 1] = bpre[k][i] + mode_workgroups(m);
            A *= hs.n[k];
            cur = m.out;
            cur_ld = m.out_ldj;
        }
    }
    for (int k = 0; k < d; ++k) {
        pl.fwd_total[k] = fpre[k][n];
        pl.bwd_total[k] = bpre[k][n];
        if ((st = bhip(hipMalloc(&pl.fwd_pre[k], (n + 1) * sizeof(int64_t)), "alloc prefix")) != KL_OK) return st;
        if ((st = bhip(hipMalloc(&pl.bwd_pre[k], (n + 1) * sizeof(int64_t)), "alloc prefix")) != KL_OK) return st;
        if ((st = bhip(hipMemcpy(pl.fwd_pre[k], fpre[k].data(), (n + 1) * sizeof(int64_t), hipMemcpyHostToDevice),
                       "copy prefix")) != KL_OK)
            return st;
        if ((st = bhip(hipMemcpy(pl.bwd_pre[k], bpre[k].data(), (n + 1) * sizeof(int64_t), hipMemcpyHostToDevice),
                       "copy prefix")) != KL_OK)
            return st;
    }
    // ---- stage 5: problem table, work queue (longest first), split sums ----------------
    std::vector<S5Prob> s5(n);
    std::vector<S5Item> items;
    std::vector<RedProb> red;
    pl.nsplit.assign(n, 1);
    std::vector<int64_t> zoff(n, 0);
    int64_t zelems = 0;
    for (int i = 0; i < n; ++i) {
        const kl_problem *P = B->probs[i];
        const int64_t Np = P->Ntpad;
        const int64_t lc = std::min<int64_t>(pl.lchunk, Np);
        const int ns = int((Np + lc - 1) / lc);
        pl.nsplit[i] = ns;
        if (ns > 1) {
            zoff[i] = zelems;
            zelems += int64_t(ns) * Np * kBW;
        }
        S5Prob &q = s5[i];
        q.X32 = P->dX32;
        q.X64 = P->dX64;
        q.Y5 = static_cast<char *>(B->Y5[pi]) + size_t(B->poff[i]) * esz;
        q.Zf = static_cast<char *>(B->Zf[pi]) + size_t(B->poff[i]) * esz;
        q.Z5 = nullptr;
        q.Ntpad = Np;
        q.lchunk = lc;
        q.nsplit = ns;
        q.kind = P->cov_kind;
        q.wrow = P->dJ;
        q.scale = P->sigma2;
        for (int64_t r = 0; r < Np / rows_wg; ++r)
            for (int sp = 0; sp < ns; ++sp) items.push_back(S5Item{i, int(r), sp, 0});
    }
    if (zelems > 0 && (st = bhip(hipMalloc(&pl.Z5, size_t(zelems) * esz), "alloc split partials")) != KL_OK)
        return st;
    int64_t base4 = 0;
    for (int i = 0; i < n; ++i) {
        if (pl.nsplit[i] == 1) continue;
        s5[i].Z5 = static_cast<char *>(pl.Z5) + size_t(zoff[i]) * esz;
        RedProb r;
        r.Zpart = s5[i].Z5;
        r.Zf = s5[i].Zf;
        r.n4 = s5[i].Ntpad * kBW / 4;
        r.stride = s5[i].Ntpad * kBW;
        r.base4 = base4;
        r.nsplit = pl.nsplit[i];
        r.prob = i;
        r.Ntpad = s5[i].Ntpad;
        r.wrow = s5[i].wrow;
        r.scale = s5[i].scale;
        base4 += r.n4;
        red.push_back(r);
    }
    pl.nred = int(red.size());
    pl.total4 = base4;
    auto cost = [&](const S5Item &it) {
        const S5Prob &q = s5[it.prob];
        const int64_t l0 = int64_t(it.split) * q.lchunk;
        return std::min(q.lchunk, q.Ntpad - l0);
    };
    std::stable_sort(items.begin(), items.end(), [&](const S5Item &a, const S5Item &b) { return cost(a) > cost(b); });
    pl.n_items = int(items.size());
    if ((st = bhip(hipMalloc(&pl.s5, n * sizeof(S5Prob)), "alloc stage-5 table")) != KL_OK) return st;
    if ((st = bhip(hipMalloc(&pl.items, std::max<size_t>(1, items.size()) * sizeof(S5Item)), "alloc queue")) != KL_OK)
        return st;
    if ((st = bhip(hipMalloc(&pl.red, std::max<size_t>(1, red.size()) * sizeof(RedProb)), "alloc split table")) != KL_OK)
        return st;
    if ((st = bhip(hipMemcpy(pl.s5, s5.data(), n * sizeof(S5Prob), hipMemcpyHostToDevice), "copy table")) != KL_OK)
        return st;
    if (!items.empty() &&
        (st = bhip(hipMemcpy(pl.items, items.data(), items.size() * sizeof(S5Item), hipMemcpyHostToDevice),
                   "copy queue")) != KL_OK)
        return st;
    if (!red.empty() &&
        (st = bhip(hipMemcpy(pl.red, red.data(), red.size() * sizeof(RedProb), hipMemcpyHostToDevice), "copy table")) !=
            KL_OK)
        return st;
    // ---- capture the apply ----------------------------------------------------------------
    const int *active = dyn_active(B);
    hipGraph_t graph = nullptr;
    if ((st = bhip(hipStreamBeginCapture(B->stream, hipStreamCaptureModeThreadLocal), "begin capture")) != KL_OK)
        return st;
    for (int k = 0; k < d; ++k)
        launch_mode_batch(pl.fwd_kind[k], dyn_fwd(B, k), pl.fwd_pre[k], n, pl.fwd_total[k], active, B->stream);
    launch_stage5_batch(precision, d, pl.rb, pl.s5, pl.items, pl.n_items, B->counter, active, pl.grid, B->stream);
    launch_split_reduce_batch(precision, pl.red, pl.nred, pl.total4, active, B->stream);
    for (int k = 0; k < d; ++k)
        launch_mode_batch(pl.bwd_kind[k], dyn_bwd(B, k), pl.bwd_pre[k], n, pl.bwd_total[k], active, B->stream);
    const hipError_t le = hipGetLastError();
    const hipError_t ce = hipStreamEndCapture(B->stream, &graph);
    if ((st = bhip(le, "kernel launch")) != KL_OK || (st = bhip(ce, "end capture")) != KL_OK) {
        if (graph) (void)hipGraphDestroy(graph);
        return st;
    }
    st = bhip(hipGraphInstantiate(&pl.exec, graph, nullptr, nullptr, 0), "instantiate graph");
    (void)hipGraphDestroy(graph);
    if (st != KL_OK) return st;
    pl.ready = true;
    return KL_OK;
}

}  // namespace

int batch_size(const kl_batch *B) { return B->n; }
kl_problem *batch_problem(kl_batch *B, int i) { return B->probs[i]; }
hipStream_t batch_stream(kl_batch *B) { return B->stream; }

// Applies A~'_i to nvec[i] <= kBW columns of problem i (x[i], y[i] with leading
// dimensions ldx[i], ldy[i]); problems with nvec[i] == 0 are skipped and their y is
// left untouched.  Asynchronous on s.
kl_status batch_apply(kl_batch *B, int precision, const int *nvec, const double *const *x, const int64_t *ldx,
                      double *const *y, const int64_t *ldy, hipStream_t s) {
    kl_status st;
    if (precision != KL_F64 && precision != KL_F32) {
        set_error("kl_apply_batch: the batched path supports KL_F64 and KL_F32");
        return KL_EINVAL;
    }
    BatchPlan &pl = B->plan[prec_index(precision)];
    if (!pl.ready && (st = build_plan(B, precision)) != KL_OK) return st;
    // the staging buffer may still be read by the previous copy
    if ((st = bhip(hipEventSynchronize(B->dyn_done), "wait for staging")) != KL_OK) return st;
    ModeArgs *hf = reinterpret_cast<ModeArgs *>(B->dyn_host);
    const int n = B->n, d = B->d;
    int *act = reinterpret_cast<int *>(B->dyn_host + sizeof(ModeArgs) * size_t(2 * d) * n);
    for (int i = 0; i < n; ++i) {
        const int nv = nvec[i];
        act[i] = nv > 0 ? 1 : 0;
        for (int k = 0; k < d; ++k) {
            ModeArgs f = pl.fwd_base[k][i], b = pl.bwd_base[k][i];
            f.nvec = std::max(nv, 1);
            b.nvec = std::max(nv, 1);
            if (k == 0) {
                f.in = nv > 0 ? x[i] : nullptr;
                f.in_ldj = nv > 0 ? ldx[i] : 0;
            }
            if (k == d - 1) {
                b.out = nv > 0 ? y[i] : nullptr;
                b.out_ldj = nv > 0 ? ldy[i] : 0;
            }
            hf[size_t(k) * n + i] = f;
            hf[size_t(d + k) * n + i] = b;
        }
    }
    if ((st = bhip(hipMemcpyAsync(B->dyn, B->dyn_host, B->dyn_bytes, hipMemcpyHostToDevice, s), "copy tables")) != KL_OK)
        return st;
    if ((st = bhip(hipEventRecord(B->dyn_done, s), "record")) != KL_OK) return st;
    return bhip(hipGraphLaunch(pl.exec, s), "graph launch");
}

}  // namespace kl

using namespace kl;

extern "C" {

kl_status kl_setup_batch(int32_t n, const kl_desc *descs, kl_batch **out) {
    if (n < 1 || !descs || !out) { set_error("kl_setup_batch: need n >= 1, descs and out"); return KL_EINVAL; }
    kl_batch *B = new (std::nothrow) kl_batch();
    if (!B) { set_error("kl_setup_batch: host allocation failed"); return KL_ENOMEM; }
    kl_status st;
#define KB_TRY(expr) do { if ((st = (expr)) != KL_OK) { free_batch(B); return st; } } while (0)
    B->n = n;
    B->d = descs[0].dim;
    for (int i = 0; i < n; ++i) {
        if (descs[i].dim != B->d) {
            free_batch(B);
            set_error("kl_setup_batch: all problems of a batch need the same dimension");
            return KL_EINVAL;
        }
        kl_problem *P = nullptr;
        st = setup_problem(&descs[i], false, nullptr, &P);
        if (st != KL_OK) {
            const std::string msg = std::string(kl_last_error());
            free_batch(B);
            std::ostringstream os;
            os << "kl_setup_batch: problem " << i << ": " << msg;
            set_error(os.str());
            return st;
        }
        B->probs.push_back(P);
    }
    B->n_cu = B->probs[0]->n_cu;
    int64_t r = 0, t = 0, p = 0;
    for (kl_problem *P : B->probs) {
        B->rowoff.push_back(r);
        B->toff.push_back(t);
        B->poff.push_back(p);
        r += P->hs.N;
        t += max_intermediate(P->hs) * kBW;
        p += P->Ntpad * kBW;
    }
    B->Ntot = r;
    KB_TRY(bhip(hipMalloc(&B->T0, size_t(t) * sizeof(double)), "alloc Kronecker arena"));
    KB_TRY(bhip(hipMalloc(&B->T1, size_t(t) * sizeof(double)), "alloc Kronecker arena"));
    for (int q = 0; q < 2; ++q) {
        const size_t bytes = size_t(p) * (q == 0 ? sizeof(double) : sizeof(float));
        KB_TRY(bhip(hipMalloc(&B->Y5[q], bytes), "alloc stage-5 arena"));
        KB_TRY(bhip(hipMalloc(&B->Zf[q], bytes), "alloc stage-5 arena"));
        // padding rows of the stage-5 inputs are never written and must stay zero
        KB_TRY(bhip(hipMemset(B->Y5[q], 0, bytes), "clear stage-5 arena"));
        KB_TRY(bhip(hipMemset(B->Zf[q], 0, bytes), "clear stage-5 arena"));
    }
    KB_TRY(bhip(hipMalloc(&B->counter, sizeof(int)), "alloc counter"));
    B->dyn_bytes = sizeof(ModeArgs) * size_t(2 * B->d) * n + sizeof(int) * size_t(n);
    KB_TRY(bhip(hipMalloc(&B->dyn, B->dyn_bytes), "alloc tables"));
    KB_TRY(bhip(hipHostMalloc(reinterpret_cast<void **>(&B->dyn_host), B->dyn_bytes, hipHostMallocDefault),
                "alloc staging"));
    std::memset(B->dyn_host, 0, B->dyn_bytes);
    KB_TRY(bhip(hipMemcpy(B->dyn, B->dyn_host, B->dyn_bytes, hipMemcpyHostToDevice), "clear tables"));
    KB_TRY(bhip(hipEventCreateWithFlags(&B->dyn_done, hipEventDisableTiming), "event"));
    KB_TRY(bhip(hipStreamCreate(&B->stream), "stream"));
#undef KB_TRY
    *out = B;
    return KL_OK;
}

kl_status kl_batch_info(const kl_batch *B, int32_t i, int64_t *N, int64_t *Ntilde, int64_t *row_offset) {
    if (!B) { set_error("kl_batch_info: NULL handle"); return KL_EINVAL; }
    if (i < 0 || i >= B->n) { set_error("kl_batch_info: index out of range"); return KL_EINVAL; }
    if (N) *N = B->probs[i]->hs.N;
    if (Ntilde) *Ntilde = B->probs[i]->hs.Nt;
    if (row_offset) *row_offset = B->rowoff[i];
    return KL_OK;
}

kl_status kl_apply_batch(kl_batch *B, int32_t precision, int32_t nvec, const double *x, double *y,
                         const int32_t *active, void *stream) {
    if (!B) { set_error("kl_apply_batch: NULL handle"); return KL_EINVAL; }
    if (nvec < 0 || nvec > kBW) { set_error("kl_apply_batch: nvec must be in 0..32"); return KL_EINVAL; }
    if (nvec == 0) return KL_OK;
    if (!x || !y) { set_error("kl_apply_batch: NULL vector"); return KL_EINVAL; }
    const char *xb = reinterpret_cast<const char *>(x), *yb = reinterpret_cast<const char *>(y);
    const size_t bytes = size_t(B->Ntot) * nvec * sizeof(double);
    if (xb < yb + bytes && yb < xb + bytes) { set_error("kl_apply_batch: x and y overlap"); return KL_EINVAL; }
    std::vector<int> nv(B->n);
    std::vector<const double *> xs(B->n);
    std::vector<double *> ys(B->n);
    std::vector<int64_t> ld(B->n);
    for (int i = 0; i < B->n; ++i) {
        nv[i] = (!active || active[i]) ? nvec : 0;
        xs[i] = x + nvec * B->rowoff[i];
        ys[i] = y + nvec * B->rowoff[i];
        ld[i] = B->probs[i]->hs.N;
    }
    return batch_apply(B, precision, nv.data(), xs.data(), ld.data(), ys.data(), ld.data(),
                       static_cast<hipStream_t>(stream));
}

kl_status kl_batch_config(kl_batch *B, int32_t precision, int32_t rb, int64_t lchunk, int32_t *grid_out,
                          int32_t *items_out) {
    if (!B) { set_error("kl_batch_config: NULL handle"); return KL_EINVAL; }
    if (precision != KL_F64 && precision != KL_F32) { set_error("kl_batch_config: KL_F64 or KL_F32"); return KL_EINVAL; }
    if (rb != 0 && rb != 2 && rb != 4) { set_error("kl_batch_config: rb must be 0, 2 or 4"); return KL_EINVAL; }
    if (lchunk < 0) { set_error("kl_batch_config: lchunk must be >= 0"); return KL_EINVAL; }
    const int pi = prec_index(precision);
    const bool change = (rb > 0 && rb != B->cfg_rb[pi]) || lchunk != B->cfg_lchunk[pi];
    if (rb > 0) B->cfg_rb[pi] = rb;
    B->cfg_lchunk[pi] = lchunk;
    kl_status st;
    if (change || !B->plan[pi].ready) {
        if ((st = bhip(hipStreamSynchronize(B->stream), "sync")) != KL_OK) return st;
        if ((st = bhip(hipDeviceSynchronize(), "sync")) != KL_OK) return st;
        if ((st = build_plan(B, precision)) != KL_OK) return st;
    }
    if (grid_out) *grid_out = B->plan[pi].grid;
    if (items_out) *items_out = B->plan[pi].n_items;
    return KL_OK;
}

kl_status kl_batch_destroy(kl_batch *B) {
    free_batch(B);
    return KL_OK;
}

}  // extern "C"
