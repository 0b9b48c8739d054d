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

// The batched kernels read their pointers from a device table, so the compiler cannot tell
// that they point to global memory and would use flat loads, which also count against the
// counter that scalar loads wait on (a scalar argument load then waits for every load in
// flight).  Loads through these views are global loads.
template <typename T>
__device__ __forceinline__ const __attribute__((address_space(1))) T *global_view(const T *p) {
    return (const __attribute__((address_space(1))) T *)p;
}

// One wave per 16 x 16 output tile on v_mfma_f64_16x16x4_f64, operands loaded straight
// from memory into registers (all loads of a chunk are issued before the first of its
// MFMAs), no LDS and no barriers.  Lane layout: A[i][k] and B[k][j] sit in lane (i or j) + 16 k;
// accumulator r of lane L holds C[(L >> 4) + 4 r][L & 15].
//  * First direction (A == 1): C = IN D^T  (16 rows x 16 o): A = IN[row][i], B = D^T[i][o];
//    a lane of the result holds 16 consecutive o of one row -> coalesced stores.
//  * Later directions: C = D IN^T (16 o x 16 rows): A = D[o][i], B = IN[row][i]; a lane
//    holds 16 consecutive rows (consecutive a) of one o -> coalesced stores.
// The contraction index is processed in chunks of 32 (8 MFMA steps: operand registers
// small enough for four waves per SIMD, which these latency-bound tiles need).
constexpr int kChunk = 8;                  // MFMA steps per operand batch (32 indices)

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
    const int o_lc = min(o_l, nout - 1);
    const TIN *in = static_cast<const TIN *>(g.in);
    const bool has_w = g.in_w != nullptr, has_ow = g.out_w != nullptr;
    // output positions of this lane's four accumulators, and their weights (loaded here,
    // with the operands, not at the stores)
    int64_t pq[4], jq[4];
    bool okq[4];
    if (FIRST) {
        // rows rt 16 + lk + 4 q (A == 1): split the first one, then step by 4
        uint32_t rr = rt * 16 + lk;
        uint32_t j = rr / Clo, c = rr - j * Clo;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            okq[q] = rr < nrows && o_l < nout;
            pq[q] = int64_t(o_lc) + int64_t(nout) * (okq[q] ? c : 0);
            jq[q] = okq[q] ? j : 0;
            rr += 4;
            c += 4;
            while (c >= Clo) { c -= Clo; ++j; }
        }
    } else {
        // row r (this lane's), outputs o = ot 16 + lk + 4 q
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int o = ot * 16 + lk + 4 * q;
            okq[q] = rok && o < nout;
            pq[q] = int64_t(ra) + g.A * (int64_t(min(o, nout - 1)) + int64_t(nout) * rc);
            jq[q] = rj;
        }
    }
    double ow[4];                                           // read only when has_ow
    if (has_ow) {
        const auto wo = global_view(g.out_w);
#pragma unroll
        for (int q = 0; q < 4; ++q) ow[q] = wo[pq[q]];
    }
    doublex4 acc = {0.0, 0.0, 0.0, 0.0};
    // Every load reads a clamped, valid address (rows past the end use row 0, indices past
    // nin the last one) and is issued before any value is used; the values are masked
    // afterwards and pinned in registers ahead of the MFMA steps.  (Loads behind branches
    // that use them made each load wait for its value before the next was issued.)  The
    // factor is read transposed, D^T[i][o]: the 16 lanes of one i read 16 consecutive o.
    for (int kc = 0; kc < nin; kc += 4 * kChunk) {
        const int nst = min(kChunk, (nin - kc + 3) / 4);     // MFMA steps of this chunk
        TIN tin[kChunk];
        double td[kChunk], tw[kChunk];                      // tw read only when has_w
        const auto gin = global_view(in);
        const auto gdt = global_view(g.DT);
        // steps past nst load nothing (uniform guards; the blocks only load)
#pragma unroll
        for (int s = 0; s < kChunk; ++s) {
            if (s < nst) {
                const int ic = min(kc + 4 * s + lk, nin - 1);
                tin[s] = gin[bin + g.A * ic];
                td[s] = gdt[int64_t(ic) * nout + o_lc];
            }
        }
        if (has_w) {
            const auto gw = global_view(g.in_w);
#pragma unroll
            for (int s = 0; s < kChunk; ++s)
                if (s < nst) tw[s] = gw[pin + g.A * min(kc + 4 * s + lk, nin - 1)];
        }
        double xa[kChunk], xb[kChunk];
#pragma unroll
        for (int s = 0; s < kChunk; ++s) {
            const bool iok = kc + 4 * s + lk < nin;
            double vin = (rok && iok) ? double(tin[s]) : 0.0;
            vin *= has_w ? g.in_scale * tw[s] : 1.0;
            const double vd = (ook && iok) ? td[s] : 0.0;
            if (FIRST) { xa[s] = vin; xb[s] = vd; }
            else { xa[s] = vd; xb[s] = vin; }
            asm volatile("" : "+v"(xa[s]), "+v"(xb[s]));   // materialise before the steps
        }
#pragma unroll
        for (int s = 0; s < kChunk; ++s)
            if (s < nst) acc = __builtin_amdgcn_mfma_f64_16x16x4f64(xa[s], xb[s], acc, 0, 0, 0);
    }
    // ---- store: C[(lane >> 4) + 4 q][lane & 15] --------------------------------------
    // (first direction: a lane holds 16 consecutive o of one row; later directions: 16
    // consecutive rows of one o; both coalesced)
    TOUT *out = static_cast<TOUT *>(g.out);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        if (okq[q]) {
            const double v = has_ow ? acc[q] * ow[q] : acc[q];
            store_out<TOUT>(out, g.out_lo, pq[q] + g.out_ldj * jq[q], v);
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

// Directions 1 and 2 of one 2-D slab per workgroup (both Kronecker factors of a 2-D
// problem, or the first two of a 3-D one), Sec. 2.2 applied twice without a trip through
// memory:
//     U[o1][i2]     = sum_i1 D1[o1][i1] IN_s[i1][i2]       (phase 1, kept in LDS)
//     OUT_s[o1][o2] = sum_i2 D2[o2][i2] U[o1][i2]          (phase 2)
// for the slab s = c + Clo j (c < Clo: the index of the directions after the second,
// j: the vector), IN_s[i1][i2] at in + i1 + nin1 (i2 + nin2 c) + in_ldj j and OUT_s at
// out + o1 + nout1 (o2 + nout2 c) + out_ldj j.  Workgroup (s, b) owns the 16 values
// o1 = 16 b.. and all of o2, so that no output value is computed twice; the workgroups
// of one slab are nslab apart in launch order, which keeps them on one XCD (one L2)
// when nslab is a multiple of 8.
//  * The D1 rows of the block (the A operand of every phase-1 tile, the same for all
//    waves) are staged once in LDS, read from the transposed factor where the 16 values
//    of one contraction index are consecutive; each wave loads the D2 rows of its first
//    phase-2 tile into registers.  Both are issued before the slab, so that they arrive
//    while it is staged.
//  * Phase 0 stages the whole input slab in LDS with coalesced loads, 8 entries and up
//    to 8 partial inputs per thread in flight: the `nsplit` partials (stride in_split)
//    are added in split order and the sum scaled by in_scale in_w[p] when in_w is set
//    (the stage-5 split sums and sigma^2 J taken on the way in; the weights are loaded
//    with the first partials, not after the sum).
//  * Phase 1: 16 x 16 tiles of U on v_mfma_f64_16x16x4_f64, B = the slab from LDS.
//  * Phase 2: tiles of OUT^T (16 o2 x 16 o1), B = U from LDS; a lane's accumulators are
//    16 consecutive o1 of one o2 (coalesced stores), times out_w[p] when set (the weights
//    of the first tile loaded at the start), converted to TOUT (BF16 with an optional low
//    part).
//  * Tiles go to waves round robin.  With 8 waves (two per SIMD) the T mod 4 tiles left
//    after the largest multiple of 4 are cut into four quarters of the contraction on
//    waves of four different SIMDs, so that every SIMD carries the same number of MFMA
//    steps; the quarters' partial tiles meet in LDS and are added in quarter order.
// NS: MFMA steps per contraction, ceil(max(nin1, nin2) / 4) <= kMode2Steps.  Every load
// reads a clamped, valid address (a weight that is not given reads entry 0 of D1T) and
// its value is masked where it is used, not where it is loaded: the kernel has no
// branches around loads, which would make each load wait for its value before the next
// one is issued.
constexpr int kMode2Steps = 20;                            // largest NS (no spills)

template <typename TIN, typename TOUT, int NS>
__global__ __launch_bounds__(512) void mode2_kernel(Mode2Args g) {
    extern __shared__ double lds2[];
    const int n1 = g.nin1, n2 = g.nin2, m1 = g.nout1, m2 = g.nout2;
    const int ldx = n1 | 1;                               // odd strides: conflict-free columns
    const int t2 = (n2 + 15) / 16;
    const int ldu = 16 * t2 + 1;
    double *sX = lds2;                                    // [i2][ldx]
    double *sU = sX + n2 * ldx;                           // [16 o1][ldu]
    constexpr int NQ = (NS + 3) / 4;                      // MFMA steps of a quarter
    double *sA = sU + 16 * ldu;                           // [i1 < 16 NQ][16 o1]: D1 rows of the block
    double *sP = sA + 256 * NQ;                           // [4 R][256]: partial tiles of quarters
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, nw = blockDim.x >> 6;
    const int li = lane & 15, lk = lane >> 4;
    const int nt = blockDim.x;
    const uint32_t slab = blockIdx.x;
    const int ob = blockIdx.y;                            // block of 16 o1
    const uint32_t j = slab / uint32_t(g.Clo), c = slab - j * uint32_t(g.Clo);
    const int t2o = (m2 + 15) / 16;
    // tiles of the two phases done whole (F) and in quarters (R = T mod 4, 8 waves only);
    // quarter unit k < 4 R is quarter k mod 4 of tile F + k / 4, on wave (F + k) mod 8
    const bool quarters = nw == 8;
    const int R1 = quarters ? t2 % 4 : 0, F1 = t2 - R1;
    const int R2 = quarters ? t2o % 4 : 0, F2 = t2o - R2;
    const int kq1 = ((w - F1) % 8 + 8) % 8, kq2 = ((w - F2) % 8 + 8) % 8;   // first quarter units
    const int o1 = ob * 16 + li;                          // this lane's phase-2 o1 (and B column)
    const int o1c = min(o1, m1 - 1);
    const int64_t pslab = int64_t(m1) * m2 * c;
    // ---- loads in flight while the slab is staged ----------------------------------------
    // D1 rows of the block: entry q = 16 i + o of sA (i < 16 NQ; rows past nin1 are zero)
    constexpr int kA = 4;
    constexpr int na = 256 * NQ;
    double av[kA];
#pragma unroll
    for (int u = 0; u < kA; ++u) {
        const int q = threadIdx.x + u * nt, i = q >> 4, o = ob * 16 + (q & 15);
        av[u] = g.D1T[int64_t(min(i, n1 - 1)) * m1 + min(o, m1 - 1)];
    }
    // D2 rows and output weights of this wave's first phase-2 tile (masked in phase 2).
    // Loads that a wave does not need sit behind wave-uniform branches whose blocks do
    // not use the values, so that nothing waits for them there.
    const bool has_ow = g.out_w != nullptr;
    const double *owp = has_ow ? g.out_w + pslab : g.D1T;
    double a2[NS], ow[4], a2q[NQ], owr[2];
#pragma unroll
    for (int u = 0; u < NS; ++u) a2[u] = 0.0;
#pragma unroll
    for (int u = 0; u < NQ; ++u) a2q[u] = 0.0;
#pragma unroll
    for (int r = 0; r < 4; ++r) ow[r] = 1.0;
    owr[0] = owr[1] = 1.0;
    if (w < F2) {                                         // first whole tile
        const int o2c = min(w * 16 + li, m2 - 1);
#pragma unroll
        for (int u = 0; u < NS; ++u) a2[u] = g.D2T[int64_t(min(4 * u + lk, n2 - 1)) * m2 + o2c];
        if (has_ow) {
#pragma unroll
            for (int r = 0; r < 4; ++r)
                ow[r] = owp[int64_t(o1c) + int64_t(m1) * min(w * 16 + lk + 4 * r, m2 - 1)];
        }
    }
    if (kq2 < 4 * R2) {                                   // first quarter unit
        const int o2c = min((F2 + kq2 / 4) * 16 + li, m2 - 1), u0 = (kq2 % 4) * NQ;
#pragma unroll
        for (int u = 0; u < NQ; ++u) a2q[u] = g.D2T[int64_t(min(4 * (u0 + u) + lk, n2 - 1)) * m2 + o2c];
    }
    if (has_ow && R2 > 0) {                               // weights of the quartered outputs this thread adds
#pragma unroll
        for (int m = 0; m < 2; ++m) {
            const int idx = int(threadIdx.x) + m * nt, e = idx & 255;
            const int o1r = min(ob * 16 + (e & 15), m1 - 1), o2r = min((F2 + (idx >> 8)) * 16 + (e >> 4), m2 - 1);
            owr[m] = owp[int64_t(o1r) + int64_t(m1) * o2r];
        }
    }
    // ---- phase 0: the input slab, split partials summed, into LDS ---------------------
    // Lanes past the end of the slab read and write its last entry (the same value as
    // the lane that owns it), so that no load or store sits behind a branch; one pass
    // covers the slab in the common case and is then straight-line code.  The forms with
    // and without input weights are separate branches (HW below), each with its own
    // loads and uses.
    {
        const int64_t pbase = int64_t(n1) * n2 * c;        // point index of the slab's first entry
        const TIN *in = static_cast<const TIN *>(g.in) + pbase + g.in_ldj * int64_t(j);
        const double *inw = g.in_w + pbase;                // dereferenced only when in_w is set
        const double wscale = g.in_scale;
        const int ne = n1 * n2;
        const float rn1 = 1.0f / float(n1);
        auto put = [&](int e, double x) __attribute__((always_inline)) {                  // e < ne
            int i2 = int(float(e) * rn1);                  // e / n1 (e < 2^20: off by at most one)
            if (i2 * n1 > e) --i2;
            if ((i2 + 1) * n1 <= e) ++i2;
            sX[i2 * ldx + (e - i2 * n1)] = x;
        };
        if (g.nsplit == 1) {
            constexpr int kE = 12;
            auto pass = [&](int e0, auto hw) __attribute__((always_inline)) {
                constexpr bool HW = decltype(hw)::value;
                double wv[kE];
                TIN t[kE];
                if constexpr (HW) {
#pragma unroll
                    for (int u = 0; u < kE; ++u) wv[u] = inw[min(e0 + u * nt, ne - 1)];
                }
#pragma unroll
                for (int u = 0; u < kE; ++u) t[u] = in[min(e0 + u * nt, ne - 1)];
#pragma unroll
                for (int u = 0; u < kE; ++u) {
                    double x = double(t[u]);
                    if constexpr (HW) x *= wscale * wv[u];
                    put(min(e0 + u * nt, ne - 1), x);
                }
            };
            auto run = [&](auto hw) __attribute__((always_inline)) {
                if (ne <= kE * nt) pass(int(threadIdx.x), hw);
                else for (int e0 = threadIdx.x; e0 < ne; e0 += kE * nt) pass(e0, hw);
            };
            if (g.in_w) run(std::true_type{}); else run(std::false_type{});
        } else {
            constexpr int kE = 9, kQ = sizeof(TIN) == 4 ? 8 : 4;
            const uint32_t split = uint32_t(g.in_split);   // < 2^31 (checked on the host)
            // NQ > 0: exactly NQ partials in one group (no clamped duplicate loads);
            // NQ = 0: groups of kQ, the last one clamped and masked
            auto pass = [&](int e0, auto nq, auto hw) __attribute__((always_inline)) {
                constexpr bool HW = decltype(hw)::value;
                constexpr int NQ = decltype(nq)::value;
                double wv[kE], v[kE];
                if constexpr (HW) {
#pragma unroll
                    for (int u = 0; u < kE; ++u) wv[u] = inw[min(e0 + u * nt, ne - 1)];
                }
#pragma unroll
                for (int u = 0; u < kE; ++u) v[u] = 0.0;
                if constexpr (NQ > 0) {
                    TIN t[NQ][kE];
#pragma unroll
                    for (int q = 0; q < NQ; ++q)
#pragma unroll
                        for (int u = 0; u < kE; ++u) t[q][u] = in[uint32_t(q) * split + uint32_t(min(e0 + u * nt, ne - 1))];
#pragma unroll
                    for (int q = 0; q < NQ; ++q)
#pragma unroll
                        for (int u = 0; u < kE; ++u) v[u] += double(t[q][u]);
                } else {
                    for (int q0 = 0; q0 < g.nsplit; q0 += kQ) {
                        TIN t[kQ][kE];
#pragma unroll
                        for (int q = 0; q < kQ; ++q)
#pragma unroll
                            for (int u = 0; u < kE; ++u)
                                t[q][u] = in[uint32_t(min(q0 + q, g.nsplit - 1)) * split + uint32_t(min(e0 + u * nt, ne - 1))];
#pragma unroll
                        for (int q = 0; q < kQ; ++q)
#pragma unroll
                            for (int u = 0; u < kE; ++u) v[u] += (q0 + q < g.nsplit) ? double(t[q][u]) : 0.0;
                    }
                }
#pragma unroll
                for (int u = 0; u < kE; ++u) {
                    double x = v[u];
                    if constexpr (HW) x *= wscale * wv[u];
                    put(min(e0 + u * nt, ne - 1), x);
                }
            };
            auto one = [&](auto nq, auto hw) __attribute__((always_inline)) { pass(int(threadIdx.x), nq, hw); };
            auto run = [&](auto hw) __attribute__((always_inline)) {
                using std::integral_constant;
                if (ne <= kE * nt && g.nsplit <= kQ) {
                    switch (g.nsplit) {                        // 2..kQ (nsplit 1 takes the branch above)
                    case 2: one(integral_constant<int, 2>{}, hw); break;
                    case 3: one(integral_constant<int, 3>{}, hw); break;
                    case 4: one(integral_constant<int, 4>{}, hw); break;
                    default:
                        if constexpr (kQ > 4) {
                            switch (g.nsplit) {
                            case 5: one(integral_constant<int, 5>{}, hw); break;
                            case 6: one(integral_constant<int, 6>{}, hw); break;
                            case 7: one(integral_constant<int, 7>{}, hw); break;
                            default: one(integral_constant<int, kQ>{}, hw); break;
                            }
                        }
                        break;
                    }
                } else {
                    for (int e0 = threadIdx.x; e0 < ne; e0 += kE * nt) pass(e0, integral_constant<int, 0>{}, hw);
                }
            };
            if (g.in_w) run(std::true_type{}); else run(std::false_type{});
        }
    }
#pragma unroll
    for (int u = 0; u < kA; ++u) {
        const int q = threadIdx.x + u * nt;
        if (q < na) sA[q] = ((q >> 4) < n1 && ob * 16 + (q & 15) < m1) ? av[u] : 0.0;
    }
    for (int q = threadIdx.x + kA * nt; q < na; q += nt) {   // blocks of fewer than 8 waves
        const int i = q >> 4, o = ob * 16 + (q & 15);
        const double v = g.D1T[int64_t(min(i, n1 - 1)) * m1 + min(o, m1 - 1)];
        sA[q] = (i < n1 && o < m1) ? v : 0.0;
    }
    __syncthreads();
    // ---- phase 1: U = D1[block] IN_s ----------------------------------------------------
    // B operands are read unmasked from clamped addresses: past nin1 the A operand is
    // zero, and columns i2 >= nin2 of U (finite, from clamped reads) meet zero A
    // operands in phase 2.
    for (int t = w; t < F1; t += nw) {
        const double *col = sX + min(t * 16 + li, n2 - 1) * ldx;   // B operand column i2 of this lane
        // all operands of the chain are read first, so that LDS latency is paid once
        double opa[NS], opb[NS];
#pragma unroll
        for (int u = 0; u < NS; ++u) {
            opa[u] = sA[(4 * u + lk) * 16 + li];
            opb[u] = col[min(4 * u + lk, n1 - 1)];
        }
        __builtin_amdgcn_sched_barrier(0);
        doublex4 acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int u = 0; u < NS; ++u) acc = __builtin_amdgcn_mfma_f64_16x16x4f64(opa[u], opb[u], acc, 0, 0, 0);
        // acc[r] = U[o1 local lk + 4 r][i2 = t 16 + li]
#pragma unroll
        for (int r = 0; r < 4; ++r) sU[(lk + 4 * r) * ldu + t * 16 + li] = acc[r];
    }
    for (int k = kq1; k < 4 * R1; k += 8) {
        const int t = F1 + k / 4, u0 = (k % 4) * NQ;
        const double *col = sX + min(t * 16 + li, n2 - 1) * ldx;
        doublex4 acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int u = 0; u < NQ; ++u) {
            const int i = 4 * (u0 + u) + lk;                 // < 16 NQ: rows of sA past nin1 are zero
            acc = __builtin_amdgcn_mfma_f64_16x16x4f64(sA[i * 16 + li], col[min(i, n1 - 1)], acc, 0, 0, 0);
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) sP[k * 256 + lane * 4 + r] = acc[r];
    }
    __syncthreads();
    if (R1 > 0) {
        for (int idx = threadIdx.x; idx < R1 * 256; idx += nt) {
            const int rt = idx >> 8, e = idx & 255, ol = e >> 4, il = e & 15;
            const double *p = sP + rt * 1024 + (il + 16 * (ol & 3)) * 4 + (ol >> 2);
            sU[ol * ldu + (F1 + rt) * 16 + il] = ((p[0] + p[256]) + p[512]) + p[768];
        }
        __syncthreads();
    }
    // ---- phase 2: OUT_s^T[o2][o1] = D2[o2][:] U[o1][:]^T --------------------------------
    TOUT *out = static_cast<TOUT *>(g.out);
    const int64_t obase = pslab + g.out_ldj * int64_t(j);
    const double *urow = sU + li * ldu;
    // U columns past 16 t2 were not written: B reads clamp to the last written one (the A
    // operand is zero past nin2)
    for (int t = w; t < F2; t += nw) {
        if (t != w) {                                      // later tiles: their D2 rows and weights
            const int o2c = min(t * 16 + li, m2 - 1);
#pragma unroll
            for (int u = 0; u < NS; ++u) a2[u] = g.D2T[int64_t(min(4 * u + lk, n2 - 1)) * m2 + o2c];
            if (has_ow) {
#pragma unroll
                for (int r = 0; r < 4; ++r)
                    ow[r] = owp[int64_t(o1c) + int64_t(m1) * min(t * 16 + lk + 4 * r, m2 - 1)];
            }
        }
        const bool row_ok = t * 16 + li < m2;
        double opb[NS];                                    // B operands read first (see phase 1)
#pragma unroll
        for (int u = 0; u < NS; ++u) opb[u] = urow[min(4 * u + lk, 16 * t2 - 1)];
        __builtin_amdgcn_sched_barrier(0);
        doublex4 acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int u = 0; u < NS; ++u)
            acc = __builtin_amdgcn_mfma_f64_16x16x4f64((row_ok && 4 * u + lk < n2) ? a2[u] : 0.0, opb[u], acc, 0, 0, 0);
        // acc[r] = OUT^T[o2 = t 16 + lk + 4 r][o1]
        if (o1 < m1) {
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int o2 = t * 16 + lk + 4 * r;
                if (o2 < m2) {
                    const int64_t pl = int64_t(o1) + int64_t(m1) * o2;
                    store_out<TOUT>(out, g.out_lo, obase + pl, has_ow ? acc[r] * ow[r] : acc[r]);
                }
            }
        }
    }
    for (int k = kq2; k < 4 * R2; k += 8) {
        const int t = F2 + k / 4, u0 = (k % 4) * NQ;
        if (k != kq2) {                                    // later quarter units: their D2 rows
            const int o2c = min(t * 16 + li, m2 - 1);
#pragma unroll
            for (int u = 0; u < NQ; ++u) a2q[u] = g.D2T[int64_t(min(4 * (u0 + u) + lk, n2 - 1)) * m2 + o2c];
        }
        const bool row_ok = t * 16 + li < m2;
        doublex4 acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int u = 0; u < NQ; ++u) {
            const int i = 4 * (u0 + u) + lk;
            acc = __builtin_amdgcn_mfma_f64_16x16x4f64((row_ok && i < n2) ? a2q[u] : 0.0,
                                                      urow[min(i, 16 * t2 - 1)], acc, 0, 0, 0);
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) sP[k * 256 + lane * 4 + r] = acc[r];
    }
    if (R2 > 0) {
        __syncthreads();
#pragma unroll
        for (int m = 0; m < 2; ++m) {
            const int idx = int(threadIdx.x) + m * nt;
            if (idx < R2 * 256) {
                // entry e: o2 = 16 (F2 + rt) + (e >> 4), o1 = 16 ob + (e & 15)
                const int rt = idx >> 8, e = idx & 255, ol = e >> 4, il = e & 15;
                const double *p = sP + rt * 1024 + (il + 16 * (ol & 3)) * 4 + (ol >> 2);
                const double v = ((p[0] + p[256]) + p[512]) + p[768];
                const int o1e = ob * 16 + il, o2e = (F2 + rt) * 16 + ol;
                if (o1e < m1 && o2e < m2)
                    store_out<TOUT>(out, g.out_lo, obase + int64_t(o1e) + int64_t(m1) * o2e, has_ow ? v * owr[m] : v);
            }
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

// MFMA steps of mode2_kernel: ceil(max(nin1, nin2) / 4)
static int mode2_steps(int nin1, int nin2) { return (std::max(nin1, nin2) + 3) / 4; }

// Waves of a mode2_kernel block: 8 for slabs of more than 1024 values (one pass of the
// staging loads); small slabs take one wave per 16-wide tile of the larger phase.
static int mode2_waves(int nin1, int nin2, int nout2) {
    const int tiles = std::max((nin2 + 15) / 16, (nout2 + 15) / 16);
    return nin1 * nin2 > 1024 ? 8 : std::min(8, std::max(2, tiles));
}

// LDS bytes of mode2_kernel: the slab (nin2 rows of nin1 | 1), U (16 rows of
// 16 ceil(nin2 / 16) + 1), the D1 rows of the block (16 NQ x 16, NQ = ceil(NS / 4)) and,
// with 8 waves, the partial tiles of up to 3 quartered tiles (12 x 256), FP64.
static size_t mode2_lds(int nin1, int nin2, int nout2) {
    const size_t nq = size_t((mode2_steps(nin1, nin2) + 3) / 4);
    const size_t parts = mode2_waves(nin1, nin2, nout2) == 8 ? size_t(12 * 256) : 0;
    return size_t(8) * (size_t(nin2) * size_t(nin1 | 1) + size_t(16) * size_t(16 * ((nin2 + 15) / 16) + 1) +
                        size_t(256) * nq + parts);
}

bool mode2_fits(int nin1, int nin2, int nout1, int nout2, int64_t slabs) {
    return nin1 >= 1 && nin2 >= 1 && nout1 >= 1 && nout2 >= 1 && slabs >= 1 && slabs < (int64_t(1) << 31) &&
           nin1 <= 4 * kMode2Steps && nin2 <= 4 * kMode2Steps && (nout1 + 15) / 16 <= 65535 &&
           mode2_lds(nin1, nin2, nout2) <= size_t(kMode2MaxLds);
}

template <typename TI, typename TO, int NS>
static void launch_mode2_ns(const Mode2Args &a, dim3 grid, int threads, size_t lds, hipStream_t s) {
    // once per process (thread-safe initialisation of a function-local static)
    static const bool attr = [] {
        (void)hipFuncSetAttribute(reinterpret_cast<const void *>(&mode2_kernel<TI, TO, NS>),
                                  hipFuncAttributeMaxDynamicSharedMemorySize, kMode2MaxLds);
        return true;
    }();
    (void)attr;
    hipLaunchKernelGGL((mode2_kernel<TI, TO, NS>), grid, dim3(threads), lds, s, a);
}

template <typename TI, typename TO, int NS>
static void launch_mode2_steps(int steps, const Mode2Args &a, dim3 grid, int threads, size_t lds, hipStream_t s) {
    if constexpr (NS < kMode2Steps) {
        if (steps > NS) return launch_mode2_steps<TI, TO, NS + 1>(steps, a, grid, threads, lds, s);
    }
    launch_mode2_ns<TI, TO, NS>(a, grid, threads, lds, s);
}

template <typename TI, typename TO>
static void launch_mode2_t(const Mode2Args &a, dim3 grid, int threads, size_t lds, hipStream_t s) {
    launch_mode2_steps<TI, TO, 1>(mode2_steps(a.nin1, a.nin2), a, grid, threads, lds, s);
}

void launch_mode2(const Mode2Args &a, bool in_f32, int out_kind, hipStream_t s) {
    const int waves = mode2_waves(a.nin1, a.nin2, a.nout2);
    const dim3 grid(unsigned(int64_t(a.Clo) * a.nvec), unsigned((a.nout1 + 15) / 16));
    const size_t lds = mode2_lds(a.nin1, a.nin2, a.nout2);
    if (in_f32) launch_mode2_t<float, double>(a, grid, 64 * waves, lds, s);
    else if (out_kind == 1) launch_mode2_t<double, float>(a, grid, 64 * waves, lds, s);
    else if (out_kind == 2) launch_mode2_t<double, __bf16>(a, grid, 64 * waves, lds, s);
    else launch_mode2_t<double, double>(a, grid, 64 * waves, lds, s);
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
