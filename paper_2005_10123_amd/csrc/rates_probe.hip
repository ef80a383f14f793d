// rates_probe.hip -- issue rates of the VALU instructions the pairwise pass is built from, on one
// gfx950 device, for the roofline of the pass (built by paper_2005_10123_amd/build.py into the
// executable paper_2005_10123_amd/rates_probe; prints one JSON object).
//
// Each probe kernel runs, in every lane, kChains independent dependency chains of one instruction
// kind (or a fixed mix) for kIters iterations, so the SIMD's issue rate, not an instruction's
// latency, bounds it.  The grid is exactly `waves` blocks of 256 threads per compute unit (one wave
// per SIMD per block, all resident at once), so each SIMD runs `waves` waves.  Every wave reads the
// device's constant 100 MHz clock (s_memrealtime, common to the whole device) and its own shader
// clock counter (s_memtime, not aligned between compute units) before and after its loop.  The
// probe's span is the largest end minus the smallest start of the 100 MHz clock over all waves; the
// shader clock is the median over the waves of their shader-clock ticks per 100 MHz tick, and
//     cycles per wave64 instruction per SIMD = span * clock / (waves * instructions per wave),
//     lanes per clock per CU = 4 SIMDs * 64 lanes / that.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <vector>

namespace {

constexpr int kThreads = 256;
constexpr int kChains = 8;
constexpr int kIters = 16384;

enum Kind : int {
    kFmaF32 = 0, kAddF32, kMulF32, kExpF32, kFmaF64, kAddF64, kSubU32, kMixExp4Fma, kMixExp4Add, kDppAddF32,
    kNumKinds
};
const char* kName[kNumKinds] = {"v_fma_f32", "v_add_f32", "v_mul_f32", "v_exp_f32", "v_fma_f64", "v_add_f64",
                                "v_sub_u32", "mix: 1 v_exp_f32 + 4 v_fma_f32", "mix: 1 v_exp_f32 + 4 v_add_f32",
                                "v_add_f32 with a DPP row rotation"};
// VALU instructions per chain step of each kind (the mixes count every instruction).
const int kPerStep[kNumKinds] = {1, 1, 1, 1, 1, 1, 1, 5, 5, 1};

template <int KIND>
__global__ __launch_bounds__(kThreads) void probe(float seed, unsigned long long* rec, float* sink)
{
    const unsigned long long r0 = __builtin_amdgcn_s_memrealtime();
    const unsigned long long t0 = __builtin_amdgcn_s_memtime();
    float f[kChains], g[kChains];
    double d[kChains];
    int u[kChains];
#pragma unroll
    for (int c = 0; c < kChains; ++c) {
        f[c] = seed + 0.001f * (float)(threadIdx.x + c);
        g[c] = f[c] + 0.5f;
        d[c] = (double)f[c];
        u[c] = (int)threadIdx.x + c;
    }
    const float a = 0.999f + 1e-7f * seed, b = 1e-6f * seed;
    const double da = (double)a, db = (double)b;
#pragma unroll 1
    for (int it = 0; it < kIters; ++it) {
#pragma unroll
        for (int c = 0; c < kChains; ++c) {
            if (KIND == kFmaF32) f[c] = fmaf(f[c], a, b);
            if (KIND == kAddF32) f[c] = f[c] + b;
            if (KIND == kMulF32) f[c] = f[c] * a;
            if (KIND == kExpF32) f[c] = __builtin_amdgcn_exp2f(-f[c]);
            if (KIND == kFmaF64) d[c] = fma(d[c], da, db);
            if (KIND == kAddF64) d[c] = d[c] + db;
            if (KIND == kSubU32) u[c] = u[c] - (int)threadIdx.x;
            if (KIND == kDppAddF32)
                f[c] += __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, f[c]), 0x121,
                                                                             0xF, 0xF, false));
        }
        if (KIND == kMixExp4Fma || KIND == kMixExp4Add) {
            // Per chain step: chain c's exponential and four operations on the other chains, each of
            // those independent of the exponential issued just before it.
#pragma unroll
            for (int c = 0; c < kChains; ++c) {
                f[c] = __builtin_amdgcn_exp2f(-f[c]);
#pragma unroll
                for (int k = 1; k <= 4; ++k) {
                    const int o = (c + k) % kChains;
                    if (KIND == kMixExp4Fma) g[o] = fmaf(g[o], a, b);
                    else g[o] = g[o] + b;
                }
            }
        }
    }
    const unsigned long long t1 = __builtin_amdgcn_s_memtime();
    const unsigned long long r1 = __builtin_amdgcn_s_memrealtime();
    float acc = 0.0f;
#pragma unroll
    for (int c = 0; c < kChains; ++c) acc += f[c] + g[c] + (float)d[c] + (float)u[c];
    const int gid = blockIdx.x * kThreads + threadIdx.x;
    sink[gid] = acc;
    if ((threadIdx.x & 63) == 0) {
        unsigned long long* w = rec + 4 * (size_t)(gid >> 6);
        w[0] = r0;
        w[1] = r1;
        w[2] = t0;
        w[3] = t1;
    }
}

template <int KIND>
void launch(int blocks, float seed, unsigned long long* rec, float* sink)
{
    probe<KIND><<<blocks, kThreads>>>(seed, rec, sink);
}

using Launcher = void (*)(int, float, unsigned long long*, float*);
const Launcher kLaunch[kNumKinds] = {launch<kFmaF32>, launch<kAddF32>, launch<kMulF32>, launch<kExpF32>,
                                     launch<kFmaF64>, launch<kAddF64>, launch<kSubU32>, launch<kMixExp4Fma>,
                                     launch<kMixExp4Add>, launch<kDppAddF32>};

#define CHECK(x)                                                                          \
    do {                                                                                  \
        hipError_t e_ = (x);                                                              \
        if (e_ != hipSuccess) {                                                           \
            std::fprintf(stderr, "%s: %s\n", #x, hipGetErrorString(e_));                  \
            std::exit(1);                                                                 \
        }                                                                                 \
    } while (0)

}  // namespace

int main()
{
    int cus = 0;
    CHECK(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, 0));
    const int max_waves = 4;  // per SIMD; one block of 4 waves per CU and wave per SIMD
    const size_t max_wave_slots = (size_t)cus * max_waves * 4;
    unsigned long long* d_rec = nullptr;
    float* d_sink = nullptr;
    CHECK(hipMalloc(&d_rec, max_wave_slots * 4 * sizeof(unsigned long long)));
    CHECK(hipMalloc(&d_sink, max_wave_slots * 64 * sizeof(float)));
    hipEvent_t ev0, ev1;
    CHECK(hipEventCreate(&ev0));
    CHECK(hipEventCreate(&ev1));
    std::vector<unsigned long long> rec(max_wave_slots * 4);
    std::printf("{\"compute_units\": %d, \"chains_per_lane\": %d, \"iterations\": %d, \"probes\": [", cus, kChains,
                kIters);
    bool first = true;
    const int wave_counts[3] = {1, 2, 4};
    for (int kind = 0; kind < kNumKinds; ++kind) {
        for (int wi = 0; wi < 3; ++wi) {
            const int waves = wave_counts[wi];
            const int blocks = cus * waves;
            const size_t nw = (size_t)blocks * 4;  // waves of the grid
            kLaunch[kind](blocks, 1.0f, d_rec, d_sink);  // warm-up
            CHECK(hipGetLastError());
            CHECK(hipDeviceSynchronize());
            CHECK(hipEventRecord(ev0, 0));
            kLaunch[kind](blocks, 1.0f, d_rec, d_sink);
            CHECK(hipGetLastError());
            CHECK(hipEventRecord(ev1, 0));
            CHECK(hipEventSynchronize(ev1));
            float ms = 0.0f;
            CHECK(hipEventElapsedTime(&ms, ev0, ev1));
            CHECK(hipMemcpy(rec.data(), d_rec, nw * 4 * sizeof(unsigned long long), hipMemcpyDeviceToHost));
            unsigned long long lo = rec[0], hi = rec[1];
            std::vector<double> ratio(nw);
            for (size_t w = 0; w < nw; ++w) {
                const unsigned long long* r = &rec[4 * w];
                lo = r[0] < lo ? r[0] : lo;
                hi = r[1] > hi ? r[1] : hi;
                ratio[w] = r[1] > r[0] ? (double)(r[3] - r[2]) / (double)(r[1] - r[0]) : 0.0;
            }
            std::sort(ratio.begin(), ratio.end());
            const double clock_hz = ratio[nw / 2] * 100e6;
            const double span_s = (double)(hi - lo) / 100e6;
            const double instr = (double)kIters * kChains * kPerStep[kind];
            const double cyc = span_s * clock_hz / (waves * instr);
            std::printf("%s{\"kind\": \"%s\", \"waves_per_simd\": %d, \"span_us\": %.2f, \"kernel_ms\": %.4f, "
                        "\"clock_ghz\": %.4f, \"cycles_per_wave_instruction\": %.4f, \"lanes_per_clock_per_cu\": %.3f}",
                        first ? "" : ", ", kName[kind], waves, span_s * 1e6, ms, clock_hz * 1e-9, cyc, 4.0 * 64.0 / cyc);
            first = false;
        }
    }
    std::printf("]}\n");
    CHECK(hipFree(d_rec));
    CHECK(hipFree(d_sink));
    return 0;
}
