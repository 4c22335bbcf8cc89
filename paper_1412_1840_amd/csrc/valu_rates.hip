// VALU throughput probe for gfx950: the rates that bound the pair x frequency kernel.
//
//   valu_rates [iterations]
//   valu_rates copy <MiB>   one plain device-to-device copy kernel of MiB mebibytes (to calibrate
//                           memory-traffic counters: it reads and writes exactly MiB each)
//
// Prints one JSON object with lane-operations per second for
//   exp   : v_exp_f32 only (independent chains x <- 2^-x, values stay in (0, 1])
//   fma   : FP32 fused multiply-add only
//   pair  : the pair-sum body itself - a multiply and two FMAs for the squared half-angle sine,
//           one v_exp_f32 and three accumulations (add, add, FMA) per item - reported as items per
//           second.
// Every launch is sized to fill the chip several times over; all loops have fixed trip counts.
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

constexpr int kChains = 16;

__global__ void __launch_bounds__(256) exp_kernel(float* out, int iters) {
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

__global__ void __launch_bounds__(256) fma_kernel(float* out, int iters, float a, float b) {
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

// The pair-sum body over 32 register rows and a stream of columns read from a small table.
__global__ void __launch_bounds__(256) pair_kernel(float* out, const float2* cols, int ncols,
                                                  int reps, float off) {
    constexpr int R = 32;
    float ci[R], si[R], G[R];
#pragma unroll
    for (int m = 0; m < R; ++m) {
        __sincosf(0.1f * (m + threadIdx.x), &si[m], &ci[m]);
        ci[m] *= 2.f;
        si[m] *= 2.f;
        G[m] = 0.f;
    }
    float T = 0.f, J = 0.f;
    for (int r = 0; r < reps; ++r) {
        for (int q = 0; q < ncols; ++q) {
            const float2 u = cols[q];  // uniform
            const float k = 0.5f + 0.001f * q;
            float Tj = 0.f, Jj = 0.f;
#pragma unroll
            for (int m = 0; m < R; ++m) {
                const float pr = ci[m] * u.y;
                const float d = __builtin_fmaf(si[m], u.x, -pr);
                const float a = __builtin_fmaf(d, d, off);
                const float g = __builtin_amdgcn_exp2f(-a);
                Tj += g;
                G[m] += g;
                Jj = __builtin_fmaf(k, g, Jj);
            }
            T += Tj;
            J += Jj;
        }
    }
    float s = T + J;
#pragma unroll
    for (int m = 0; m < R; ++m) s += G[m];
    out[blockIdx.x * blockDim.x + threadIdx.x] = s;
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
    const int blocks = cus * 16, threads = 256;
    float* out;
    CHECK(hipMalloc(&out, sizeof(float) * blocks * threads));
    const int ncols = 64;
    float2 hcols[ncols];
    for (int q = 0; q < ncols; ++q) hcols[q] = make_float2(0.3f * q / ncols, -0.2f * q / ncols);
    float2* cols;
    CHECK(hipMalloc(&cols, sizeof(hcols)));
    CHECK(hipMemcpy(cols, hcols, sizeof(hcols), hipMemcpyHostToDevice));
    hipEvent_t e0, e1;
    CHECK(hipEventCreate(&e0));
    CHECK(hipEventCreate(&e1));
    auto time_ms = [&](auto launch) {
        launch();  // warm-up
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
    double ms_exp = time_ms([&] { exp_kernel<<<blocks, threads>>>(out, iters); });
    double ms_fma = time_ms([&] { fma_kernel<<<blocks, threads>>>(out, iters, 0.999f, 1e-3f); });
    const int reps = iters / 64 > 0 ? iters / 64 : 1;
    double ms_pair =
        time_ms([&] { pair_kernel<<<blocks, threads>>>(out, cols, ncols, reps, 0.f); });
    const double exp_rate = lanes * iters * kChains / (ms_exp * 1e-3);
    const double fma_rate = lanes * iters * kChains / (ms_fma * 1e-3);
    const double pair_rate = lanes * (double)reps * ncols * 32 / (ms_pair * 1e-3);
    std::printf("{\"device\": \"%s\", \"cus\": %d, \"clock_mhz\": %d, \"exp_per_s\": %.4e, "
                "\"fma_per_s\": %.4e, \"pair_items_per_s\": %.4e, \"exp_vs_fma\": %.3f, "
                "\"pair_slots_per_item\": %.3f}\n",
                prop.gcnArchName, cus, prop.clockRate / 1000, exp_rate, fma_rate, pair_rate,
                exp_rate / fma_rate, fma_rate / pair_rate);
    CHECK(hipFree(out));
    CHECK(hipFree(cols));
    return 0;
}
