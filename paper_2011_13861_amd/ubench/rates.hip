// Issue-rate microbenchmark of the units the covariance kernel uses on this chip: FP32 and
// FP64 FMA, the FP32 base-2 exponential and square root, the three matrix-core forms of the
// stage-5 kernels, and whether matrix-core and vector-ALU instructions overlap (in one wave,
// and across two waves sharing a SIMD).  The roofline of the covariance kernel is priced
// against these measured rates (the transcendental rate is not published).
//
// Every kernel runs independent dependency chains (so that issue, not latency, is measured)
// for a fixed number of iterations and stores its chains, so nothing is optimised away.
// Output: one JSON object per test on stdout.
//
// Build: hipcc -O3 --offload-arch=gfx950 -Xclang -target-feature -Xclang -packed-fp32-ops
//        rates.hip -o klrates
#include <hip/hip_runtime.h>

#include <cstdio>
#include <algorithm>
#include <cstdlib>
#include <vector>

typedef float floatx16 __attribute__((ext_vector_type(16)));
typedef double doublex4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

#define CHECK(x)                                                                       \
    do {                                                                               \
        hipError_t e_ = (x);                                                           \
        if (e_ != hipSuccess) {                                                        \
            fprintf(stderr, "%s: %s\n", #x, hipGetErrorString(e_));                    \
            exit(1);                                                                   \
        }                                                                              \
    } while (0)

constexpr int kChains = 8;

// VALU chains: FP32 FMA, FP64 FMA, v_exp_f32, v_sqrt_f32 (kChains per lane, iters steps).
template <int OP>
__global__ __launch_bounds__(256) void valu_kernel(float *out32, double *out64, int iters, float a) {
    float v[kChains];
    double w[kChains];
#pragma unroll
    for (int c = 0; c < kChains; ++c) {
        v[c] = 0.25f + 0.01f * float(c + threadIdx.x % 7);
        w[c] = double(v[c]);
    }
    // four steps of every chain per loop trip (iters is a multiple of 4), so that the loop
    // control is a small part of the issue slots
    for (int it = 0; it < iters; it += 4) {
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
            for (int c = 0; c < kChains; ++c) {
                if constexpr (OP == 0) v[c] = fmaf(v[c], a, 0.5f);
                else if constexpr (OP == 1) w[c] = fma(w[c], double(a), 0.5);
                else if constexpr (OP == 2) v[c] = __builtin_amdgcn_exp2f(-v[c]);
                else v[c] = __builtin_amdgcn_sqrtf(v[c]);
            }
    }
    float s = 0.f;
    double t = 0.0;
#pragma unroll
    for (int c = 0; c < kChains; ++c) { s += v[c]; t += w[c]; }
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    out32[g] = s;
    out64[g] = t;
}

// Matrix-core chains: 4 independent accumulators per wave.  KIND 0: FP32 32x32x2,
// 1: BF16 32x32x16, 2: FP64 16x16x4.  MODE 0: every wave issues the matrix instructions,
// each followed by NVALU FP32 FMAs on independent chains (none with NVALU = 0); MODE 1: the
// waves of the upper half of the 512-thread workgroup (one per SIMD, next to a lower-half
// wave on the same SIMD) issue only the FMAs, the lower half only the matrix instructions;
// MODE 2: every wave issues only the FMAs (4 NVALU per iteration).
template <int KIND, int NVALU, int MODE>
__global__ __launch_bounds__(512) void mfma_kernel(float *out32, double *out64, int iters, float a) {
    const int lane = threadIdx.x & 63;
    const bool valu_wave = MODE == 2 || (MODE == 1 && threadIdx.x >= 256);
    floatx16 acc[4];
    doublex4 dacc[4];
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int r = 0; r < 16; ++r) { acc[q][r] = 0.f; if (r < 4) dacc[q][r] = 0.0; }
    float v[kChains];
#pragma unroll
    for (int c = 0; c < kChains; ++c) v[c] = 0.25f + 0.01f * float(c + lane % 5);
    const float fa = 1e-3f * float(lane);
    const double da = 1e-3 * double(lane);
    bf16x8 ba;
#pragma unroll
    for (int e = 0; e < 8; ++e) ba[e] = __bf16(fa + 0.01f * float(e));
    if (!valu_wave) {
        for (int it = 0; it < iters; ++it) {
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                if constexpr (KIND == 0) acc[q] = __builtin_amdgcn_mfma_f32_32x32x2f32(fa, fa, acc[q], 0, 0, 0);
                else if constexpr (KIND == 1) acc[q] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ba, ba, acc[q], 0, 0, 0);
                else dacc[q] = __builtin_amdgcn_mfma_f64_16x16x4f64(da, da, dacc[q], 0, 0, 0);
                if constexpr (NVALU > 0 && MODE == 0) {
#pragma unroll
                    for (int c = 0; c < NVALU; ++c) v[c % kChains] = fmaf(v[c % kChains], a, 0.5f);
                }
            }
        }
    } else {
        for (int it = 0; it < iters; ++it)
#pragma unroll
            for (int q = 0; q < 4; ++q)
#pragma unroll
                for (int c = 0; c < NVALU; ++c) v[c % kChains] = fmaf(v[c % kChains], a, 0.5f);
    }
    float s = 0.f;
    double t = 0.0;
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int r = 0; r < 16; ++r) { s += acc[q][r]; if (r < 4) t += dacc[q][r]; }
#pragma unroll
    for (int c = 0; c < kChains; ++c) s += v[c];
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    out32[g] = s;
    out64[g] = t;
}

struct Timer {
    hipEvent_t a, b;
    Timer() { CHECK(hipEventCreate(&a)); CHECK(hipEventCreate(&b)); }
    ~Timer() { (void)hipEventDestroy(a); (void)hipEventDestroy(b); }
};

template <typename F>
double time_ms(F launch) {
    Timer t;
    launch();   // warm
    CHECK(hipDeviceSynchronize());
    double best = 1e30;
    for (int r = 0; r < 5; ++r) {
        CHECK(hipEventRecord(t.a, 0));
        launch();
        CHECK(hipEventRecord(t.b, 0));
        CHECK(hipEventSynchronize(t.b));
        float ms = 0.f;
        CHECK(hipEventElapsedTime(&ms, t.a, t.b));
        if (ms < best) best = ms;
    }
    CHECK(hipGetLastError());
    return best;
}

int main(int argc, char **argv) {
    int dev = 0, ncu = 0, clk_khz = 0;
    CHECK(hipGetDevice(&dev));
    CHECK(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
    CHECK(hipDeviceGetAttribute(&clk_khz, hipDeviceAttributeClockRate, dev));
    const int iters = (argc > 1 ? atoi(argv[1]) : 4096) / 4 * 4;
    // two 256-thread workgroups per CU (two waves per SIMD) for the vector tests; one
    // 512-thread workgroup per CU (two waves per SIMD) for the matrix tests
    const int g256 = 2 * ncu, g512 = ncu;
    float *o32;
    double *o64;
    CHECK(hipMalloc(&o32, sizeof(float) * 512 * g512 * 2));
    CHECK(hipMalloc(&o64, sizeof(double) * 512 * g512 * 2));
    printf("{\"test\": \"device\", \"cus\": %d, \"max_clock_mhz\": %.0f, \"iters\": %d}\n", ncu, clk_khz / 1e3, iters);
    const double simds = 4.0 * ncu;
    auto report = [&](const char *name, double ms, double wave_instr, const char *unit, double per_instr) {
        // wave_instr: wave-level instructions of the measured kind issued chip-wide
        const double per_simd = wave_instr / simds;
        const double rate = wave_instr * per_instr / (ms * 1e-3);
        printf("{\"test\": \"%s\", \"ms\": %.4f, \"wave_instr_per_simd\": %.0f, \"ns_per_wave_instr_per_simd\": %.4f, "
               "\"rate\": %.4e, \"unit\": \"%s\"}\n",
               name, ms, per_simd, ms * 1e6 / per_simd, rate, unit);
    };
    const double vwaves = g256 * 4.0;   // waves in a 256-thread launch
    const double vi = vwaves * iters * kChains;
    report("fma_f32", time_ms([&] { valu_kernel<0><<<g256, 256>>>(o32, o64, iters, 0.999f); }), vi, "FLOP/s", 128.0);
    report("fma_f64", time_ms([&] { valu_kernel<1><<<g256, 256>>>(o32, o64, iters, 0.999f); }), vi, "FLOP/s", 128.0);
    report("exp_f32", time_ms([&] { valu_kernel<2><<<g256, 256>>>(o32, o64, iters, 0.999f); }), vi, "lane-op/s", 64.0);
    report("sqrt_f32", time_ms([&] { valu_kernel<3><<<g256, 256>>>(o32, o64, iters, 0.999f); }), vi, "lane-op/s", 64.0);
    const double mwaves = g512 * 8.0;
    const double mi = mwaves * iters * 4.0;
    const double t_m32 = time_ms([&] { mfma_kernel<0, 0, 0><<<g512, 512>>>(o32, o64, iters, 0.999f); });
    report("mfma_f32_32x32x2", t_m32, mi, "FLOP/s", 32.0 * 32 * 2 * 2);
    report("mfma_bf16_32x32x16", time_ms([&] { mfma_kernel<1, 0, 0><<<g512, 512>>>(o32, o64, iters, 0.999f); }),
           mi, "FLOP/s", 32.0 * 32 * 16 * 2);
    const double t_m64 = time_ms([&] { mfma_kernel<2, 0, 0><<<g512, 512>>>(o32, o64, iters, 0.999f); });
    report("mfma_f64_16x16x4", t_m64, mi, "FLOP/s", 16.0 * 16 * 4 * 2);
    // co-issue: 8 FMAs after each matrix instruction in the same wave, against the matrix
    // instructions alone and the same FMAs alone (serialised: t_both = t_mfma + t_fma;
    // overlapped: t_both = max)
    const double t_v8 = time_ms([&] { mfma_kernel<0, 8, 2><<<g512, 512>>>(o32, o64, iters, 0.999f); });
    report("fma_f32_8_per_mfma_alone", t_v8, mi * 8, "FLOP/s", 128.0);
    const double t_b32 = time_ms([&] { mfma_kernel<0, 8, 0><<<g512, 512>>>(o32, o64, iters, 0.999f); });
    report("mfma_f32_plus_8_fma_same_wave", t_b32, mi, "FLOP/s", 32.0 * 32 * 2 * 2);
    const double t_b64 = time_ms([&] { mfma_kernel<2, 8, 0><<<g512, 512>>>(o32, o64, iters, 0.999f); });
    report("mfma_f64_plus_8_fma_same_wave", t_b64, mi, "FLOP/s", 16.0 * 16 * 4 * 2);
    const double t_mb = time_ms([&] { mfma_kernel<1, 0, 0><<<g512, 512>>>(o32, o64, iters, 0.999f); });
    const double t_bb = time_ms([&] { mfma_kernel<1, 8, 0><<<g512, 512>>>(o32, o64, iters, 0.999f); });
    report("mfma_bf16_plus_8_fma_same_wave", t_bb, mi, "FLOP/s", 32.0 * 32 * 16 * 2);
    const double t_sb = time_ms([&] { mfma_kernel<1, 8, 1><<<g512, 512>>>(o32, o64, iters, 0.999f); });
    report("mfma_bf16_next_to_fma_wave", t_sb, mi / 2, "FLOP/s", 32.0 * 32 * 16 * 2);
    // split: per SIMD one wave of matrix instructions next to one wave of FMAs (half the
    // work of each of the tests above)
    const double t_s32 = time_ms([&] { mfma_kernel<0, 8, 1><<<g512, 512>>>(o32, o64, iters, 0.999f); });
    report("mfma_f32_next_to_fma_wave", t_s32, mi / 2, "FLOP/s", 32.0 * 32 * 2 * 2);
    const double t_s64 = time_ms([&] { mfma_kernel<2, 8, 1><<<g512, 512>>>(o32, o64, iters, 0.999f); });
    report("mfma_f64_next_to_fma_wave", t_s64, mi / 2, "FLOP/s", 16.0 * 16 * 4 * 2);
    printf("{\"test\": \"summary\", \"mfma_f32_ms\": %.4f, \"mfma_f64_ms\": %.4f, \"fma_ms\": %.4f, "
           "\"f32_same_wave_ms\": %.4f, \"f64_same_wave_ms\": %.4f, \"f32_split_ms\": %.4f, \"f64_split_ms\": %.4f, "
           "\"f32_same_wave_overlap\": %.3f, \"f64_same_wave_overlap\": %.3f, \"f32_split_overlap\": %.3f, "
           "\"f64_split_overlap\": %.3f, \"mfma_bf16_ms\": %.4f, \"bf16_same_wave_ms\": %.4f, "
           "\"bf16_split_ms\": %.4f, \"bf16_same_wave_overlap\": %.3f, \"bf16_split_overlap\": %.3f}\n",
           t_m32, t_m64, t_v8, t_b32, t_b64, t_s32, t_s64,
           (t_m32 + t_v8 - t_b32) / std::min(t_m32, t_v8), (t_m64 + t_v8 - t_b64) / std::min(t_m64, t_v8),
           (0.5 * (t_m32 + t_v8) - t_s32) / (0.5 * std::min(t_m32, t_v8)),
           (0.5 * (t_m64 + t_v8) - t_s64) / (0.5 * std::min(t_m64, t_v8)), t_mb, t_bb, t_sb,
           (t_mb + t_v8 - t_bb) / std::min(t_mb, t_v8), (0.5 * (t_mb + t_v8) - t_sb) / (0.5 * std::min(t_mb, t_v8)));
    CHECK(hipFree(o32));
    CHECK(hipFree(o64));
    return 0;
}
