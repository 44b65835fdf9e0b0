// Device characterization for roofline reporting (not part of the method): the
// sustained rates of the two FP64 pipes the pair kernels can use, measured
// with register-only streams of independent operations at two waves per SIMD
// (the occupancy of the FP64 pair kernel), and the shader clock read from the
// core clock counter against the fixed-frequency real-time counter.
#include <hip/hip_runtime.h>

#include "host.hpp"
#include "mcpt_internal.hpp"

namespace mcpt {

namespace {

typedef double d4 __attribute__((ext_vector_type(4)));

constexpr int kCalThreads = 256;
constexpr int kCalAcc = 8;      // independent MFMA accumulators per wave
constexpr int kCalChains = 16;  // independent FMA chains per lane

// mode 0: v_mfma_f64_16x16x4 only; mode 1: v_fma_f64 only.  out[block * threads + lane]
// keeps the results live; clk[2 block] = core-clock cycles, clk[2 block + 1] =
// real-time (100 MHz) ticks of the block's first wave.
template <int MODE>
__global__ __launch_bounds__(kCalThreads) void rate_kernel(double* out, unsigned long long* clk, int iters,
                                                           double s) {
    d4 acc[kCalAcc];
    double v[kCalChains];
#pragma unroll
    for (int i = 0; i < kCalAcc; ++i) acc[i] = d4(0.0);
#pragma unroll
    for (int i = 0; i < kCalChains; ++i) v[i] = threadIdx.x + i;
    const double a = threadIdx.x * 1e-3;
    const unsigned long long t0 = __builtin_amdgcn_s_memtime(), r0 = __builtin_amdgcn_s_memrealtime();
    for (int it = 0; it < iters; ++it) {
        if (MODE == 0) {
#pragma unroll
            for (int i = 0; i < kCalAcc; ++i) acc[i] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, s, acc[i], 0, 0, 0);
        } else {
#pragma unroll
            for (int r = 0; r < 4; ++r)
#pragma unroll
                for (int i = 0; i < kCalChains; ++i) v[i] = __builtin_fma(v[i], s, 1.0);
        }
    }
    const unsigned long long t1 = __builtin_amdgcn_s_memtime(), r1 = __builtin_amdgcn_s_memrealtime();
    double t = 0.0;
#pragma unroll
    for (int i = 0; i < kCalAcc; ++i) t += acc[i].x + acc[i].y + acc[i].z + acc[i].w;
#pragma unroll
    for (int i = 0; i < kCalChains; ++i) t += v[i];
    out[(int64_t)blockIdx.x * kCalThreads + threadIdx.x] = t;
    if (threadIdx.x == 0) {
        clk[2 * blockIdx.x] = t1 - t0;
        clk[2 * blockIdx.x + 1] = r1 - r0;
    }
}

}  // namespace

}  // namespace mcpt

using namespace mcpt;

extern "C" mcpt_status mcpt_device_rates(int device, mcpt_rates* out) {
    if (!out) return fail(MCPT_ERR_INVALID, "out is NULL");
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess || device < 0 || device >= n)
        return fail(MCPT_ERR_INVALID, "no HIP device " + std::to_string(device));
    if (hipSetDevice(device) != hipSuccess) return fail(MCPT_ERR_DEVICE, "hipSetDevice failed");
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) != hipSuccess) return fail(MCPT_ERR_DEVICE, "device properties");
    const int blocks = prop.multiProcessorCount * 2;   // 4 waves per block, 2 blocks per CU: 2 waves per SIMD
    const int iters = 20000;
    double* d = nullptr;
    unsigned long long* c = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    mcpt_status st = MCPT_OK;
    float ms[2] = {0.f, 0.f};
    unsigned long long h[2] = {0, 0};
    if (hipMalloc(&d, (size_t)blocks * kCalThreads * sizeof(double)) != hipSuccess ||
        hipMalloc(&c, (size_t)2 * blocks * sizeof(unsigned long long)) != hipSuccess ||
        hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
        st = fail(MCPT_ERR_NOMEM, "calibration buffers");
    }
    for (int mode = 0; mode < 2 && st == MCPT_OK; ++mode) {
        for (int rep = 0; rep < 2; ++rep) {   // the first launch warms the clocks up, the second is timed
            if (rep == 1) (void)hipEventRecord(e0, nullptr);
            if (mode == 0)
                hipLaunchKernelGGL(rate_kernel<0>, dim3(blocks), dim3(kCalThreads), 0, nullptr, d, c, iters, 1.0000001);
            else
                hipLaunchKernelGGL(rate_kernel<1>, dim3(blocks), dim3(kCalThreads), 0, nullptr, d, c, iters, 1.0000001);
        }
        (void)hipEventRecord(e1, nullptr);
        if (hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&ms[mode], e0, e1) != hipSuccess ||
            hipMemcpy(h, c, sizeof(h), hipMemcpyDeviceToHost) != hipSuccess)
            st = fail(MCPT_ERR_DEVICE, "calibration run failed");
    }
    if (st == MCPT_OK) {
        const double waves = (double)blocks * (kCalThreads / 64);
        out->mfma_f64_tflops = waves * iters * kCalAcc * 2048.0 / (ms[0] * 1e-3) / 1e12;
        out->valu_f64_tflops = waves * iters * 4 * kCalChains * 64 * 2.0 / (ms[1] * 1e-3) / 1e12;
        out->clock_ghz = h[1] ? (double)h[0] / ((double)h[1] / 100e6) / 1e9 : 0.0;
        out->compute_units = prop.multiProcessorCount;
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (d) (void)hipFree(d);
    if (c) (void)hipFree(c);
    return st;
}
