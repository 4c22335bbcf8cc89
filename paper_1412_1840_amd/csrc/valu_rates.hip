// VALU throughput probe for gfx950: the rates that bound the pair x frequency kernel.
//
//   valu_rates [iterations]
//   valu_rates copy <MiB>   one plain device-to-device copy kernel of MiB mebibytes (to calibrate
//                           memory-traffic counters: it reads and writes exactly MiB each)
//
// Prints one JSON object with lane-operations per second for
//   exp   : v_exp_f32 only (independent chains x <- 2^-x, values stay in (0, 1])
//   fma   : FP32 fused multiply-add only
//   mix K : one v_exp_f32 interleaved with K FP32 FMAs, for K = 0 .. 8, 10, 12.  The exps form
//           their own independent chains and the FMAs theirs (no FMA reads an exp result), so the
//           rate is the issue ceiling of that instruction mix, free of dependences; reported as
//           items (one exp + K FMAs) per second.  K = 6 is the pair body's mix.
//   pair  : the pair kernel's own column body (below) - a multiply and two FMAs for the squared
//           half-angle sine, one v_exp_f32 and three accumulations (add, add, FMA) per item, with
//           its per-column FP64 folds - reported as items per second, as compiled and with the
//           interleaving hint (pair_hint).
// Every kernel runs 512-thread workgroups, the pair kernel's shape, and every launch is sized to
// fill the chip several times over; all loops have fixed trip counts.  clock_mhz is the device's
// reported peak engine clock (hipDeviceProp_t::clockRate), not the clock under load.
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstdlib>
#include <string>

#define CHECK(x)                                                                      \
    do {                                                                              \
        hipError_t e_ = (x);                                                          \
        if (e_ != hipSuccess) {                                                       \
            std::fprintf(stderr, "%s: %s\n", #x, hipGetErrorString(e_));              \
            std::exit(1);                                                             \
        }                                                                             \
    } while (0)

constexpr int kThreads = 512;
constexpr int kChains = 16;

__global__ void __launch_bounds__(kThreads) exp_kernel(float* out, int iters) {
    float x[kChains];
#pragma unroll
    for (int k = 0; k < kChains; ++k) x[k] = 0.01f * (threadIdx.x + k);
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int k = 0; k < kChains; ++k) x[k] = __builtin_amdgcn_exp2f(-x[k]);
    }
    float s = 0.f;
#pragma unroll
    for (int k = 0; k < kChains; ++k) s += x[k];
    out[blockIdx.x * blockDim.x + threadIdx.x] = s;
}

__global__ void __launch_bounds__(kThreads) fma_kernel(float* out, int iters, float a, float b) {
    float x[kChains];
#pragma unroll
    for (int k = 0; k < kChains; ++k) x[k] = 0.01f * (threadIdx.x + k);
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int k = 0; k < kChains; ++k) x[k] = __builtin_fmaf(x[k], a, b);
    }
    float s = 0.f;
#pragma unroll
    for (int k = 0; k < kChains; ++k) s += x[k];
    out[blockIdx.x * blockDim.x + threadIdx.x] = s;
}

// One exp and K FMAs per item: kExpChains independent exp chains x <- 2^-x and kFmaChains
// independent FMA chains y <- y a + b, the K FMAs of each exp spread round robin over the FMA
// chains.  No instruction reads the result of an instruction of the other kind.
constexpr int kExpChains = 8;
constexpr int kFmaChains = 12;

template <int K>
__global__ void __launch_bounds__(kThreads) mix_kernel(float* out, int iters, float a, float b) {
    float x[kExpChains], y[kFmaChains];
#pragma unroll
    for (int k = 0; k < kExpChains; ++k) x[k] = 0.01f * (threadIdx.x + k);
#pragma unroll
    for (int k = 0; k < kFmaChains; ++k) y[k] = 0.02f * (threadIdx.x + k);
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int e = 0; e < kExpChains; ++e) {
            x[e] = __builtin_amdgcn_exp2f(-x[e]);
#pragma unroll
            for (int q = 0; q < K; ++q) {
                const int c = (e * K + q) % kFmaChains;
                y[c] = __builtin_fmaf(y[c], a, b);
            }
        }
    }
    float s = 0.f;
#pragma unroll
    for (int k = 0; k < kExpChains; ++k) s += x[k];
#pragma unroll
    for (int k = 0; k < kFmaChains; ++k) s += y[k];
    out[blockIdx.x * blockDim.x + threadIdx.x] = s;
}

// The pair kernel's straight-line column body, as it runs there: each lane (frequency) reads its
// warp vector of the column from LDS, 32 register rows per wave with their kernel values K(i, j)
// from a per-column table read by the scalar unit (each wave its own run of 32), per item a
// multiply and two FMAs for the squared half-angle sine, one v_exp_f32, and three accumulations
// (the column partials of g and K g in four interleaved chains, the row sum of g); per column the
// FP64 fold of the column partials into LDS (ds_add_f64), per 64 columns the FP64 fold of the row
// sums.  HINT asks the scheduler to interleave every exp between the multiply-adds of its own row
// and the accumulations of the previous one (3 VALU, 1 transcendental, 3 VALU per row) instead of
// issuing each row's chain back to back.
constexpr int kRows = 32;
constexpr int kCols = 64;

__device__ __forceinline__ void lds_add(double* p, double v) {
    __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
}

template <bool HINT>
__global__ void __launch_bounds__(kThreads, 4) pair_kernel(float* out, const float* ktab,
                                                          const float* kstab, const double* rtab,
                                                          int reps) {
    __shared__ float2 ph[kCols][64];
    __shared__ double acc[3][kThreads / 64][64];
    const int lane = threadIdx.x & 63;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    for (int q = w; q < kCols; q += kThreads / 64)
        ph[q][lane] = make_float2(0.3f * q / kCols + 0.002f * lane, -0.2f * q / kCols);
    acc[0][w][lane] = 0.0;
    acc[1][w][lane] = 0.0;
    acc[2][w][lane] = 0.0;
    __syncthreads();
    float ci[kRows], si[kRows], G[kRows];
#pragma unroll
    for (int m = 0; m < kRows; ++m) {
        __sincosf(0.1f * (m + threadIdx.x), &si[m], &ci[m]);
        ci[m] *= 2.f;
        si[m] *= 2.f;
        G[m] = 0.f;
    }
    double* aJ = &acc[0][w][lane];
    double* aT = &acc[1][w][lane];
    double* aC = &acc[2][w][lane];
    for (int r = 0; r < reps; ++r) {
        for (int q = 0; q < kCols; ++q) {
            const float2 u = ph[q][lane];
            const float* kr = ktab + (q * (kThreads / 64) + w) * kRows;
            float kk[kRows];
#pragma unroll
            for (int m = 0; m < kRows; ++m) kk[m] = kr[m];
            float T4[4], J4[4];
#pragma unroll
            for (int m = 0; m < kRows; ++m) {
                const float pr = ci[m] * u.y;
                const float d = __builtin_fmaf(si[m], u.x, -pr);
                const float a = __builtin_fmaf(d, d, 0.f);
                const float g = __builtin_amdgcn_exp2f(-a);
                G[m] += g;
                if (m < 4) {
                    T4[m] = g;
                    J4[m] = kk[m] * g;
                } else {
                    T4[m & 3] += g;
                    J4[m & 3] = __builtin_fmaf(kk[m], g, J4[m & 3]);
                }
            }
            if (HINT) {
#pragma unroll
                for (int m = 0; m < kRows; ++m) {
                    __builtin_amdgcn_sched_group_barrier(0x002, 3, 0);  // VALU
                    __builtin_amdgcn_sched_group_barrier(0x400, 1, 0);  // transcendental
                    __builtin_amdgcn_sched_group_barrier(0x002, 3, 0);
                }
            }
            const float Tq = (T4[0] + T4[1]) + (T4[2] + T4[3]);
            const float Jq = (J4[0] + J4[1]) + (J4[2] + J4[3]);
            const double Td = (double)Tq;
            lds_add(aT, Td);
            lds_add(aJ, (double)(Jq - kstab[q]));
            lds_add(aC, Td * rtab[q]);
        }
        double sca = 0.0;
#pragma unroll
        for (int m = 0; m < kRows; ++m) {
            sca = fma((double)G[m], rtab[m], sca);
            G[m] = 0.f;
        }
        lds_add(aC, sca);
    }
    __syncthreads();
    out[blockIdx.x * blockDim.x + threadIdx.x] = (float)(*aJ + *aT + *aC);
}

__global__ void __launch_bounds__(256) copy_kernel(const float4* __restrict__ src,
                                                  float4* __restrict__ dst, size_t n) {
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (size_t)gridDim.x * blockDim.x)
        dst[i] = src[i];
}

static int copy_mode(size_t mib) {
    const size_t n = mib * (1u << 20) / sizeof(float4);
    float4 *a, *b;
    CHECK(hipMalloc(&a, n * sizeof(float4)));
    CHECK(hipMalloc(&b, n * sizeof(float4)));
    CHECK(hipMemset(a, 0, n * sizeof(float4)));
    CHECK(hipDeviceSynchronize());
    copy_kernel<<<4096, 256>>>(a, b, n);
    CHECK(hipDeviceSynchronize());
    std::printf("{\"copy_mib\": %zu}\n", mib);
    CHECK(hipFree(a));
    CHECK(hipFree(b));
    return 0;
}

int main(int argc, char** argv) {
    if (argc > 2 && std::string(argv[1]) == "copy") return copy_mode((size_t)std::atoi(argv[2]));
    const int iters = argc > 1 ? std::atoi(argv[1]) : 4096;
    hipDeviceProp_t prop;
    CHECK(hipGetDeviceProperties(&prop, 0));
    const int cus = prop.multiProcessorCount;
    const int blocks = cus * 16, threads = kThreads;
    float* out;
    CHECK(hipMalloc(&out, sizeof(float) * blocks * threads));
    // Kernel values (one run of 32 per wave and column), their column sums and FP64 row sums.
    const int nk = kCols * (kThreads / 64) * kRows;
    float* hk = new float[nk];
    for (int i = 0; i < nk; ++i) hk[i] = 0.25f + 0.5f * (float)(i % 977) / 977.f;
    float hks[kCols];
    double hr[kCols];
    for (int q = 0; q < kCols; ++q) {
        hks[q] = 8.f + 0.01f * q;
        hr[q] = 1.5 + 0.01 * q;
    }
    float* ktab;
    float* kstab;
    double* rtab;
    CHECK(hipMalloc(&ktab, sizeof(float) * nk));
    CHECK(hipMalloc(&kstab, sizeof(hks)));
    CHECK(hipMalloc(&rtab, sizeof(hr)));
    CHECK(hipMemcpy(ktab, hk, sizeof(float) * nk, hipMemcpyHostToDevice));
    CHECK(hipMemcpy(kstab, hks, sizeof(hks), hipMemcpyHostToDevice));
    CHECK(hipMemcpy(rtab, hr, sizeof(hr), hipMemcpyHostToDevice));
    delete[] hk;
    hipEvent_t e0, e1;
    CHECK(hipEventCreate(&e0));
    CHECK(hipEventCreate(&e1));
    auto time_ms = [&](auto launch) {
        launch();  // warm-up
        CHECK(hipGetLastError());
        CHECK(hipDeviceSynchronize());
        CHECK(hipEventRecord(e0));
        launch();
        CHECK(hipEventRecord(e1));
        CHECK(hipEventSynchronize(e1));
        float ms = 0.f;
        CHECK(hipEventElapsedTime(&ms, e0, e1));
        return (double)ms;
    };
    const double lanes = (double)blocks * threads;
    const float fa = 0.999f, fb = 1e-3f;
    double ms_exp = time_ms([&] { exp_kernel<<<blocks, threads>>>(out, iters); });
    double ms_fma = time_ms([&] { fma_kernel<<<blocks, threads>>>(out, iters, fa, fb); });
    const int reps = iters / 64 > 0 ? iters / 64 : 1;
    double ms_pair = time_ms([&] { pair_kernel<false><<<blocks, threads>>>(out, ktab, kstab, rtab,
                                                                        reps); });
    double ms_hint = time_ms([&] { pair_kernel<true><<<blocks, threads>>>(out, ktab, kstab, rtab,
                                                                       reps); });
    const double exp_rate = lanes * iters * kChains / (ms_exp * 1e-3);
    const double fma_rate = lanes * iters * kChains / (ms_fma * 1e-3);
    const double pair_rate = lanes * (double)reps * kCols * kRows / (ms_pair * 1e-3);
    const double hint_rate = lanes * (double)reps * kCols * kRows / (ms_hint * 1e-3);
    // Mixed issue: items = exps, each with K FMAs.  Fewer iterations for the longer bodies keep
    // every launch at a few milliseconds.
    const int mix_k[] = {0, 1, 2, 3, 4, 5, 6, 7, 8, 10, 12};
    double mix_rate[11];
    auto mix = [&](int K, int it) {
        switch (K) {
            case 0: return time_ms([&] { mix_kernel<0><<<blocks, threads>>>(out, it, fa, fb); });
            case 1: return time_ms([&] { mix_kernel<1><<<blocks, threads>>>(out, it, fa, fb); });
            case 2: return time_ms([&] { mix_kernel<2><<<blocks, threads>>>(out, it, fa, fb); });
            case 3: return time_ms([&] { mix_kernel<3><<<blocks, threads>>>(out, it, fa, fb); });
            case 4: return time_ms([&] { mix_kernel<4><<<blocks, threads>>>(out, it, fa, fb); });
            case 5: return time_ms([&] { mix_kernel<5><<<blocks, threads>>>(out, it, fa, fb); });
            case 6: return time_ms([&] { mix_kernel<6><<<blocks, threads>>>(out, it, fa, fb); });
            case 7: return time_ms([&] { mix_kernel<7><<<blocks, threads>>>(out, it, fa, fb); });
            case 8: return time_ms([&] { mix_kernel<8><<<blocks, threads>>>(out, it, fa, fb); });
            case 10:
                return time_ms([&] { mix_kernel<10><<<blocks, threads>>>(out, it, fa, fb); });
            default:
                return time_ms([&] { mix_kernel<12><<<blocks, threads>>>(out, it, fa, fb); });
        }
    };
    for (int i = 0; i < 11; ++i) {
        const int K = mix_k[i];
        const int it = iters * 2 / (K + 2) > 0 ? iters * 2 / (K + 2) : 1;
        const double ms = mix(K, it);
        mix_rate[i] = lanes * (double)it * kExpChains / (ms * 1e-3);
    }
    std::printf("{\"device\": \"%s\", \"cus\": %d, \"clock_mhz\": %d, \"exp_per_s\": %.4e, "
                "\"fma_per_s\": %.4e, \"pair_items_per_s\": %.4e, \"pair_hint_items_per_s\": %.4e, "
                "\"exp_vs_fma\": %.3f, \"pair_slots_per_item\": %.3f, \"mix_items_per_s\": {",
                prop.gcnArchName, cus, prop.clockRate / 1000, exp_rate, fma_rate, pair_rate,
                hint_rate, exp_rate / fma_rate, fma_rate / pair_rate);
    for (int i = 0; i < 11; ++i)
        std::printf("%s\"%d\": %.4e", i ? ", " : "", mix_k[i], mix_rate[i]);
    std::printf("}}\n");
    CHECK(hipFree(out));
    CHECK(hipFree(ktab));
    CHECK(hipFree(kstab));
    CHECK(hipFree(rtab));
    return 0;
}
