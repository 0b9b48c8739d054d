// C ABI of the warm-start network (kl_mlp_*): a tanh multilayer perceptron trained on
// the GPU with the kernels of kernels_mlp.hip (forward, backpropagation, Adam).
//
// Parameter layout (device, FP32, flat): for each layer l, W_l (fan_in x fan_out,
// row-major) followed by b_l (fan_out).  Gradients and the Adam moments use the same
// layout.  Hidden layers apply tanh; the output layer is linear.
#include <cmath>
#include <new>
#include <sstream>
#include <vector>

#include "kl_internal.h"
#include "mlp_internal.h"

struct kl_mlp {
    int L = 0;
    std::vector<int> sizes;
    std::vector<int64_t> offW, offb;
    int64_t n_params = 0;
    float *p = nullptr, *g = nullptr, *m = nullptr, *v = nullptr;
    int64_t adam_t = 0;
    int n_cu = 256;
    // activations and deltas for up to cap_batch rows
    int cap_batch = 0;
    std::vector<float *> H;          // H[l], l = 1..L-1: B x sizes[l]
    float *Y = nullptr;              // B x sizes[L]
    float *D0 = nullptr, *D1 = nullptr;   // B x max(sizes)
    float *xb = nullptr;             // B x sizes[0]
    float *part = nullptr;           // split-K partials
    int64_t part_cap = 0;
    double *loss_part = nullptr;     // per (row, group) losses
    int64_t loss_cap = 0;
    int *rows = nullptr;             // shuffled row indices (training)
    int64_t rows_cap = 0;
    float sub_w = 0.0f;              // weight of the subspace term of the grouped loss
    double *sub_buf = nullptr;       // partial sums and coefficients of the subspace term
    int64_t sub_cap = 0;
};

namespace kl {
namespace {

using namespace mlp;

kl_status hipc(hipError_t e, const char *what) {
    if (e == hipSuccess) return KL_OK;
    std::ostringstream os;
    os << "kl_mlp: " << what << ": " << hipGetErrorString(e);
    set_error(os.str());
    return e == hipErrorOutOfMemory ? KL_ENOMEM : KL_EHIP;
}

template <typename T>
kl_status alloc(T **ptr, int64_t count, const char *what) {
    (void)hipFree(*ptr);
    *ptr = nullptr;
    return hipc(hipMalloc(reinterpret_cast<void **>(ptr), size_t(std::max<int64_t>(count, 1)) * sizeof(T)), what);
}

int max_width(const kl_mlp *M) {
    int w = 0;
    for (int s : M->sizes) w = std::max(w, s);
    return w;
}

kl_status ensure_batch(kl_mlp *M, int B) {
    if (B <= M->cap_batch) return KL_OK;
    kl_status st;
    const int W = max_width(M);
    for (int l = 1; l < M->L; ++l)
        if ((st = alloc(&M->H[l], int64_t(B) * M->sizes[l], "alloc activations")) != KL_OK) return st;
    if ((st = alloc(&M->Y, int64_t(B) * M->sizes[M->L], "alloc output")) != KL_OK) return st;
    if ((st = alloc(&M->D0, int64_t(B) * W, "alloc deltas")) != KL_OK) return st;
    if ((st = alloc(&M->D1, int64_t(B) * W, "alloc deltas")) != KL_OK) return st;
    if ((st = alloc(&M->xb, int64_t(B) * M->sizes[0], "alloc input batch")) != KL_OK) return st;
    // split-K partials: the long-K product (delta times W^T of the widest layer) needs
    // up to 2 n_cu tiles' worth of splits
    M->part_cap = std::max<int64_t>(int64_t(1) << 22, int64_t(B) * W * 8);
    if ((st = alloc(&M->part, M->part_cap, "alloc partials")) != KL_OK) return st;
    M->cap_batch = B;
    return KL_OK;
}

kl_status ensure_loss(kl_mlp *M, int64_t n) {
    if (n <= M->loss_cap) return KL_OK;
    kl_status st = alloc(&M->loss_part, n, "alloc loss");
    if (st == KL_OK) M->loss_cap = n;
    return st;
}

kl_status ensure_subspace(kl_mlp *M, int B, int group) {
    const int64_t n = subspace_scratch(B, M->sizes[M->L], group);
    if (n <= M->sub_cap) return KL_OK;
    kl_status st = alloc(&M->sub_buf, n, "alloc subspace scratch");
    if (st == KL_OK) M->sub_cap = n;
    return st;
}

void gemm(kl_mlp *M, bool ta, bool tb, const float *A, int64_t lda, const float *B, int64_t ldb, float *C,
          int64_t ldc, int m, int n, int k, int epi, const float *bias, const float *aux, int64_t ldaux,
          hipStream_t s) {
    GemmArgs g;
    g.A = A; g.lda = lda; g.B = B; g.ldb = ldb; g.C = C; g.ldc = ldc;
    g.M = m; g.N = n; g.K = k;
    g.epi = epi; g.bias = bias; g.aux = aux; g.ldaux = ldaux;
    g.part = M->part;
    if (gemm_direct_ok(g)) {
        launch_gemm_direct(ta, tb, g, s);
        return;
    }
    const bool vec = gemm_vec_ok(ta, tb, g);
    const int splits = gemm_splits(m, n, k, M->n_cu, M->part_cap, vec, &g.kchunk);
    launch_gemm(ta, tb, vec, g, splits, s);
}

// Whether the weight gradient h^T D (h: B x fi, D: B x fo) runs in the float4 form in one
// K range, so that the Adam step of its parameters can run in the product's epilogue (a
// product that gemm() sends to the one-thread-per-output kernel is not fused, so that the
// gradient is the same sum either way).
bool adam_fusable(const kl_mlp *M, const float *h, const float *D, int fi, int fo, int B) {
    GemmArgs g;
    g.A = h; g.lda = fi; g.B = D; g.ldb = fo;
    g.M = fi; g.N = fo; g.K = B;
    if (gemm_direct_ok(g) || !gemm_vec_ok(true, false, g)) return false;
    int kchunk = 0;
    return gemm_splits(fi, fo, B, M->n_cu, M->part_cap, true, &kchunk) == 1;
}

// Layer l's weight gradient h^T D and bias gradient (column sums of D) in one product
// (adam_fusable holds): with `a`, the Adam step of W_l and b_l in its epilogue (no gradient
// stored), otherwise both gradients into M->g.
void gemm_dw(kl_mlp *M, int l, const float *h, const float *D, int fi, int fo, int B, const AdamArgs *a,
             hipStream_t s) {
    GemmArgs g;
    g.A = h; g.lda = fi; g.B = D; g.ldb = fo; g.ldc = fo;
    g.M = fi; g.N = fo; g.K = B;
    if (a) {
        g.C = M->p + M->offW[l];
        g.epi = EPI_ADAM; g.am = M->m + M->offW[l]; g.av = M->v + M->offW[l]; g.adam = *a;
        g.colsum = M->p + M->offb[l]; g.bm = M->m + M->offb[l]; g.bv = M->v + M->offb[l];
    } else {
        g.C = M->g + M->offW[l];
        g.colsum = M->g + M->offb[l];
    }
    g.part = M->part;
    gemm_splits(fi, fo, B, M->n_cu, M->part_cap, true, &g.kchunk);
    launch_gemm(true, false, true, g, 1, s);
}

// Forward pass of B rows of x (B x sizes[0]); the output goes to `out` (B x sizes[L]).
void forward(kl_mlp *M, int B, const float *x, float *out, hipStream_t s) {
    const float *h = x;
    for (int l = 0; l < M->L; ++l) {
        const int fi = M->sizes[l], fo = M->sizes[l + 1];
        const bool last = l == M->L - 1;
        float *dst = last ? out : M->H[l + 1];
        gemm(M, false, false, h, fi, M->p + M->offW[l], fo, dst, fo, B, fo, fi,
             last ? EPI_BIAS : EPI_BIAS_TANH, M->p + M->offb[l], nullptr, 0, s);
        h = dst;
    }
}

// Backpropagation from the output delta in M->D0 (B x sizes[L]); gradients into M->g.
// Where adam_fusable accepts a layer's weight-gradient product, that product also forms the
// bias gradient, and with `fuse` set (training) it takes the Adam step of the layer's
// weights and biases in its epilogue (no gradient stored); the ranges of all other
// parameters are added to *rest for one Adam launch afterwards.
// The delta through W_l is formed before W_l's product, which may update W_l.
void backward(kl_mlp *M, int B, const float *x, hipStream_t s, const AdamArgs *fuse = nullptr,
              AdamRanges *rest = nullptr) {
    float *D = M->D0, *Dn = M->D1;
    for (int l = M->L - 1; l >= 0; --l) {
        const int fi = M->sizes[l], fo = M->sizes[l + 1];
        const float *h = l == 0 ? x : M->H[l];
        // delta of layer l: (D W_l^T) * (1 - h_l^2)
        if (l > 0)
            gemm(M, false, true, D, fo, M->p + M->offW[l], fo, Dn, fi, B, fi, fo, EPI_DTANH, nullptr, h, fi, s);
        // dW_l = h_l^T D,  db_l = column sums of D: one product where it runs in one K range
        // of the float4 form (with or without the Adam step), else a product and column sums
        if (adam_fusable(M, h, D, fi, fo, B)) {
            gemm_dw(M, l, h, D, fi, fo, B, fuse, s);
        } else {
            gemm(M, true, false, h, fi, D, fo, M->g + M->offW[l], fo, fi, fo, B, EPI_NONE, nullptr, nullptr, 0, s);
            launch_colsum(D, fo, B, fo, M->g + M->offb[l], s);
            if (fuse) {
                rest->add(M->offW[l], int64_t(fi) * fo);
                rest->add(M->offb[l], fo);
            }
        }
        if (l > 0) std::swap(D, Dn);
    }
}

uint64_t splitmix64(uint64_t &state) {
    uint64_t z = (state += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

double uniform01(uint64_t &state) { return double(splitmix64(state) >> 11) * (1.0 / 9007199254740992.0); }

void free_mlp(kl_mlp *M) {
    if (!M) return;
    hipFree(M->p); hipFree(M->g); hipFree(M->m); hipFree(M->v);
    for (float *h : M->H) hipFree(h);
    hipFree(M->Y); hipFree(M->D0); hipFree(M->D1); hipFree(M->xb); hipFree(M->part);
    hipFree(M->loss_part); hipFree(M->rows); hipFree(M->sub_buf);
    delete M;
}

kl_status check_batch_args(const kl_mlp *M, int batch, const void *x, const char *fn) {
    if (!M) { set_error(std::string(fn) + ": NULL handle"); return KL_EINVAL; }
    if (batch < 0) { set_error(std::string(fn) + ": batch < 0"); return KL_EINVAL; }
    if (batch > 0 && !x) { set_error(std::string(fn) + ": NULL input"); return KL_EINVAL; }
    return KL_OK;
}

// Whether the grouped loss carries the subspace term; KL_EINVAL when it would need more
// target groups per row than the kernel holds.
kl_status check_subspace(const kl_mlp *M, int group, const char *fn, bool &on) {
    on = group > 0 && M->sub_w > 0.0f;
    if (on && M->sizes[M->L] / group > kMaxSubGroups) {
        set_error(std::string(fn) + ": the subspace term takes at most 32 groups per row");
        return KL_EINVAL;
    }
    return KL_OK;
}

kl_status check_group(const kl_mlp *M, int group, const char *fn) {
    const int n_out = M->sizes[M->L];
    if (group < 0 || (group > 0 && n_out % group != 0)) {
        set_error(std::string(fn) + ": group must be 0 or divide the output width");
        return KL_EINVAL;
    }
    return KL_OK;
}

// Arguments of the next Adam step (advances the step count t).
AdamArgs next_adam(kl_mlp *M, float lr, float beta1, float beta2, float eps) {
    M->adam_t += 1;
    AdamArgs a;
    a.lr = lr; a.b1 = beta1; a.b2 = beta2; a.eps = eps;
    a.ic1 = float(1.0 / (1.0 - std::pow(double(beta1), double(M->adam_t))));
    a.ic2 = float(1.0 / (1.0 - std::pow(double(beta2), double(M->adam_t))));
    return a;
}

}  // namespace
}  // namespace kl

using namespace kl;
using namespace kl::mlp;

extern "C" {

kl_status kl_mlp_create(int32_t n_layers, const int32_t *sizes, uint64_t seed, kl_mlp **out) {
    if (!sizes || !out || n_layers < 1 || n_layers > 16) {
        set_error("kl_mlp_create: need 1..16 layers, sizes and out");
        return KL_EINVAL;
    }
    for (int l = 0; l <= n_layers; ++l)
        if (sizes[l] < 1 || sizes[l] > (1 << 24)) { set_error("kl_mlp_create: layer width out of range"); return KL_EINVAL; }
    kl_mlp *M = new (std::nothrow) kl_mlp();
    if (!M) { set_error("kl_mlp_create: host allocation failed"); return KL_ENOMEM; }
    M->L = n_layers;
    M->sizes.assign(sizes, sizes + n_layers + 1);
    M->H.assign(n_layers, nullptr);
    int64_t off = 0;
    for (int l = 0; l < n_layers; ++l) {
        M->offW.push_back(off);
        off += int64_t(sizes[l]) * sizes[l + 1];
        M->offb.push_back(off);
        off += sizes[l + 1];
    }
    M->n_params = off;
    int dev = 0, ncu = 0;
    if (hipGetDevice(&dev) == hipSuccess &&
        hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && ncu > 0)
        M->n_cu = ncu;
    kl_status st;
    if ((st = alloc(&M->p, off, "alloc params")) != KL_OK || (st = alloc(&M->g, off, "alloc grads")) != KL_OK ||
        (st = alloc(&M->m, off, "alloc adam m")) != KL_OK || (st = alloc(&M->v, off, "alloc adam v")) != KL_OK) {
        free_mlp(M);
        return st;
    }
    // W_l ~ U(-1/sqrt(fan_in), 1/sqrt(fan_in)) from splitmix64(seed), b_l = 0
    std::vector<float> h(size_t(off), 0.0f);
    uint64_t state = seed;
    for (int l = 0; l < n_layers; ++l) {
        const double bound = 1.0 / std::sqrt(double(sizes[l]));
        const int64_t cnt = int64_t(sizes[l]) * sizes[l + 1];
        for (int64_t i = 0; i < cnt; ++i) h[M->offW[l] + i] = float(bound * (2.0 * uniform01(state) - 1.0));
    }
    if ((st = kl_mlp_set_params(M, h.data())) != KL_OK) { free_mlp(M); return st; }
    *out = M;
    return KL_OK;
}

kl_status kl_mlp_num_params(const kl_mlp *M, int64_t *n) {
    if (!M || !n) { set_error("kl_mlp_num_params: NULL argument"); return KL_EINVAL; }
    *n = M->n_params;
    return KL_OK;
}

kl_status kl_mlp_set_params(kl_mlp *M, const float *params) {
    if (!M || !params) { set_error("kl_mlp_set_params: NULL argument"); return KL_EINVAL; }
    const size_t bytes = size_t(M->n_params) * sizeof(float);
    kl_status st;
    if ((st = hipc(hipMemcpy(M->p, params, bytes, hipMemcpyHostToDevice), "copy params")) != KL_OK) return st;
    if ((st = hipc(hipMemset(M->m, 0, bytes), "clear adam m")) != KL_OK) return st;
    if ((st = hipc(hipMemset(M->v, 0, bytes), "clear adam v")) != KL_OK) return st;
    if ((st = hipc(hipMemset(M->g, 0, bytes), "clear grads")) != KL_OK) return st;
    M->adam_t = 0;
    return KL_OK;
}

kl_status kl_mlp_get_params(const kl_mlp *M, float *params) {
    if (!M || !params) { set_error("kl_mlp_get_params: NULL argument"); return KL_EINVAL; }
    return hipc(hipMemcpy(params, M->p, size_t(M->n_params) * sizeof(float), hipMemcpyDeviceToHost), "copy params");
}

kl_status kl_mlp_forward(kl_mlp *M, int32_t batch, const float *x, float *y, void *stream) {
    kl_status st = check_batch_args(M, batch, x, "kl_mlp_forward");
    if (st != KL_OK) return st;
    if (batch == 0) return KL_OK;
    if (!y) { set_error("kl_mlp_forward: NULL output"); return KL_EINVAL; }
    if ((st = ensure_batch(M, batch)) != KL_OK) return st;
    hipStream_t s = static_cast<hipStream_t>(stream);
    forward(M, batch, x, y, s);
    return hipc(hipGetLastError(), "kernel launch");
}

kl_status kl_mlp_gradients(kl_mlp *M, int32_t batch, const float *x, const float *t, int32_t group,
                           double *loss, float *grads, void *stream) {
    kl_status st = check_batch_args(M, batch, x, "kl_mlp_gradients");
    if (st != KL_OK) return st;
    if (batch < 1 || !t) { set_error("kl_mlp_gradients: need batch >= 1 and targets"); return KL_EINVAL; }
    if ((st = check_group(M, group, "kl_mlp_gradients")) != KL_OK) return st;
    bool sub = false;
    if ((st = check_subspace(M, group, "kl_mlp_gradients", sub)) != KL_OK) return st;
    const int n_out = M->sizes[M->L];
    const int gsz = group > 0 ? group : n_out;
    const int ng = n_out / gsz;
    if ((st = ensure_batch(M, batch)) != KL_OK) return st;
    if ((st = ensure_loss(M, int64_t(batch) * ng)) != KL_OK) return st;
    if (sub && (st = ensure_subspace(M, batch, gsz)) != KL_OK) return st;
    hipStream_t s = static_cast<hipStream_t>(stream);
    forward(M, batch, x, M->Y, s);
    launch_loss(M->Y, n_out, t, n_out, nullptr, batch, n_out, gsz, group > 0, M->D0, n_out, M->loss_part, s);
    if (sub)
        launch_subspace(M->Y, n_out, t, n_out, nullptr, batch, n_out, gsz, M->sub_w, M->D0, n_out, M->loss_part,
                        M->sub_buf, s);
    backward(M, batch, x, s);
    if ((st = hipc(hipGetLastError(), "kernel launch")) != KL_OK) return st;
    if (grads &&
        (st = hipc(hipMemcpyAsync(grads, M->g, size_t(M->n_params) * sizeof(float), hipMemcpyDeviceToDevice, s),
                   "copy grads")) != KL_OK)
        return st;
    if (loss) {
        std::vector<double> lp(size_t(batch) * ng);
        if ((st = hipc(hipMemcpyAsync(lp.data(), M->loss_part, lp.size() * sizeof(double), hipMemcpyDeviceToHost, s),
                       "copy loss")) != KL_OK)
            return st;
        if ((st = hipc(hipStreamSynchronize(s), "sync")) != KL_OK) return st;
        double sum = 0.0;
        for (double v : lp) sum += v;
        *loss = sum / batch;
    }
    return KL_OK;
}

kl_status kl_mlp_adam(kl_mlp *M, float lr, float beta1, float beta2, float eps, void *stream) {
    if (!M) { set_error("kl_mlp_adam: NULL handle"); return KL_EINVAL; }
    if (!(lr >= 0.0f) || !(beta1 >= 0.0f && beta1 < 1.0f) || !(beta2 >= 0.0f && beta2 < 1.0f) || !(eps > 0.0f)) {
        set_error("kl_mlp_adam: bad hyper-parameters");
        return KL_EINVAL;
    }
    const AdamArgs a = next_adam(M, lr, beta1, beta2, eps);
    launch_adam(M->p, M->g, M->m, M->v, M->n_params, a, static_cast<hipStream_t>(stream));
    return hipc(hipGetLastError(), "kernel launch");
}

kl_status kl_mlp_train(kl_mlp *M, int64_t n, const float *x, const float *t, int32_t group, int32_t epochs,
                       int32_t batch, float lr0, float lr1, uint64_t seed, double *epoch_loss, void *stream) {
    if (!M || !x || !t) { set_error("kl_mlp_train: NULL argument"); return KL_EINVAL; }
    if (n < 1 || n > (int64_t(1) << 30) || epochs < 1 || batch < 1) {
        set_error("kl_mlp_train: need n >= 1, epochs >= 1, batch >= 1");
        return KL_EINVAL;
    }
    if (!(lr0 > 0.0f) || !(lr1 > 0.0f)) { set_error("kl_mlp_train: learning rates must be positive"); return KL_EINVAL; }
    kl_status st = check_group(M, group, "kl_mlp_train");
    if (st != KL_OK) return st;
    bool sub = false;
    if ((st = check_subspace(M, group, "kl_mlp_train", sub)) != KL_OK) return st;
    const int n_in = M->sizes[0], n_out = M->sizes[M->L];
    const int gsz = group > 0 ? group : n_out;
    const int ng = n_out / gsz;
    const int B = int(std::min<int64_t>(batch, n));
    if ((st = ensure_batch(M, B)) != KL_OK) return st;
    if ((st = ensure_loss(M, n * ng)) != KL_OK) return st;
    if (sub && (st = ensure_subspace(M, B, gsz)) != KL_OK) return st;
    if (n > M->rows_cap) {
        if ((st = alloc(&M->rows, n, "alloc rows")) != KL_OK) return st;
        M->rows_cap = n;
    }
    hipStream_t s = static_cast<hipStream_t>(stream);
    std::vector<int> perm(static_cast<size_t>(n));
    std::vector<double> lp(static_cast<size_t>(n) * ng);
    uint64_t state = seed;
    for (int e = 0; e < epochs; ++e) {
        // Fisher-Yates shuffle with splitmix64(seed)
        for (int64_t i = 0; i < n; ++i) perm[i] = int(i);
        for (int64_t i = n - 1; i > 0; --i) {
            const int64_t j = int64_t(splitmix64(state) % uint64_t(i + 1));
            std::swap(perm[i], perm[j]);
        }
        if ((st = hipc(hipMemcpyAsync(M->rows, perm.data(), size_t(n) * sizeof(int), hipMemcpyHostToDevice, s),
                       "copy rows")) != KL_OK)
            return st;
        const double frac = epochs > 1 ? double(e) / double(epochs - 1) : 0.0;
        const float lr = float(double(lr0) * std::pow(double(lr1) / double(lr0), frac));
        for (int64_t b0 = 0; b0 < n; b0 += B) {
            const int nb = int(std::min<int64_t>(B, n - b0));
            const int *rows = M->rows + b0;
            launch_gather(x, n_in, rows, nb, n_in, M->xb, s);
            forward(M, nb, M->xb, M->Y, s);
            launch_loss(M->Y, n_out, t, n_out, rows, nb, n_out, gsz, group > 0, M->D0, n_out,
                        M->loss_part + b0 * ng, s);
            if (sub)
                launch_subspace(M->Y, n_out, t, n_out, rows, nb, n_out, gsz, M->sub_w, M->D0, n_out,
                                M->loss_part + b0 * ng, M->sub_buf, s);
            // the Adam step: in the epilogues of the weight products that allow it, then
            // one launch over the remaining parameters (the same bits as backward + kl_mlp_adam)
            const AdamArgs a = next_adam(M, lr, 0.9f, 0.999f, 1e-8f);
            AdamRanges rest;
            backward(M, nb, M->xb, s, &a, &rest);
            launch_adam_ranges(M->p, M->g, M->m, M->v, rest, a, s);
            if ((st = hipc(hipGetLastError(), "kernel launch")) != KL_OK) return st;
        }
        if ((st = hipc(hipMemcpyAsync(lp.data(), M->loss_part, lp.size() * sizeof(double), hipMemcpyDeviceToHost, s),
                       "copy loss")) != KL_OK)
            return st;
        if ((st = hipc(hipStreamSynchronize(s), "sync")) != KL_OK) return st;
        double sum = 0.0;
        for (double v : lp) sum += v;
        if (epoch_loss) epoch_loss[e] = sum / double(n);
        if (!std::isfinite(sum)) { set_error("kl_mlp_train: non-finite loss"); return KL_ENUMERIC; }
    }
    return KL_OK;
}

kl_status kl_mlp_set_subspace(kl_mlp *M, float weight) {
    if (!M) { set_error("kl_mlp_set_subspace: NULL handle"); return KL_EINVAL; }
    if (!(weight >= 0.0f) || !std::isfinite(weight)) {
        set_error("kl_mlp_set_subspace: the weight must be finite and >= 0");
        return KL_EINVAL;
    }
    M->sub_w = weight;
    return KL_OK;
}

kl_status kl_mlp_destroy(kl_mlp *M) {
    free_mlp(M);
    return KL_OK;
}

}  // extern "C"
