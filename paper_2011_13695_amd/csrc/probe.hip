// Rate probes of the vector ALU and the matrix cores on the current device:
// the measured peaks behind the roofline figures of the demapper kernels.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "internal.h"

namespace mdgmi {
namespace {

constexpr int kProbeThreads = 256;
constexpr int kProbeChains = 8;  // independent dependency chains per lane

// kIters x kProbeChains base-2 exponentials per lane (v_exp_f32,
// v <- 2^-v: the negation is a source modifier, so the loop holds nothing
// but exponentials); the values stay in [0.5, 1]. Cycle counts of the
// core clock (s_memtime) and of the constant reference clock are recorded by
// lane 0 of block 0.
template <int OP>
__global__ __launch_bounds__(kProbeThreads) void k_probe(int iters, float seed, float* __restrict__ sink,
                                                         unsigned long long* __restrict__ clk) {
    float v[kProbeChains];
#pragma unroll
    for (int c = 0; c < kProbeChains; c++) v[c] = seed * (float)(threadIdx.x + c + 1) * 1e-6f;
    unsigned long long c0 = 0, w0 = 0;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        c0 = clock64();
        w0 = wall_clock64();
    }
    for (int it = 0; it < iters; it++) {
#pragma unroll
        for (int c = 0; c < kProbeChains; c++) {
            if (OP == 0)
                v[c] = __builtin_amdgcn_exp2f(-v[c]);
            else
                v[c] = fmaf(v[c], 0.999999f, 1.0e-7f);        // plain FP32 FMA
        }
    }
    float s = 0.0f;
#pragma unroll
    for (int c = 0; c < kProbeChains; c++) s += v[c];
    if (s == 12345.0f) sink[threadIdx.x] = s;  // keeps the chains alive
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        clk[0] = clock64() - c0;
        clk[1] = wall_clock64() - w0;
    }
}

typedef __bf16 pbf16x8 __attribute__((ext_vector_type(8)));
typedef float pf32x16 __attribute__((ext_vector_type(16)));

// Independent chains of v_mfma_f32_32x32x16_bf16 per wave.
__global__ __launch_bounds__(kProbeThreads) void k_probe_mfma(int iters, float* __restrict__ sink) {
    pbf16x8 a, b;
#pragma unroll
    for (int i = 0; i < 8; i++) {
        a[i] = (__bf16)(1e-3f * (float)(threadIdx.x + i));
        b[i] = (__bf16)(1e-3f * (float)(i + 1));
    }
    pf32x16 acc[4] = {};
    for (int it = 0; it < iters; it++) {
#pragma unroll
        for (int c = 0; c < 4; c++) acc[c] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, acc[c], 0, 0, 0);
    }
    float s = 0.0f;
#pragma unroll
    for (int c = 0; c < 4; c++) s += acc[c][0];
    if (s == 12345.0f) sink[threadIdx.x] = s;
}

// Co-issue: two independent chains of v_mfma_f32_32x32x16_bf16 per wave,
// each MFMA followed by K independent FP32 FMAs (8 chains) of the same
// wave, two waves per SIMD (the fused MLP kernel's shape). The MFMA rate
// with K > 0 against K = 0 shows how many vector instructions issue while
// the matrix core runs.
template <int K>
__global__ __launch_bounds__(kProbeThreads) void k_probe_mix(int iters, float* __restrict__ sink) {
    pbf16x8 a, b;
#pragma unroll
    for (int i = 0; i < 8; i++) {
        a[i] = (__bf16)(1e-3f * (float)(threadIdx.x + i));
        b[i] = (__bf16)(1e-3f * (float)(i + 1));
    }
    pf32x16 acc[2] = {};
    float v[kProbeChains];
#pragma unroll
    for (int c = 0; c < kProbeChains; c++) v[c] = 1e-6f * (float)(threadIdx.x + c + 1);
    for (int it = 0; it < iters; it++) {
#pragma unroll
        for (int m = 0; m < 2; m++) {
            acc[m] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, acc[m], 0, 0, 0);
#pragma unroll
            for (int j = 0; j < K; j++) v[j % kProbeChains] = fmaf(v[j % kProbeChains], 0.999999f, 1.0e-7f);
        }
    }
    float s = acc[0][0] + acc[1][0];
#pragma unroll
    for (int c = 0; c < kProbeChains; c++) s += v[c];
    if (s == 12345.0f) sink[threadIdx.x] = s;
}

// The same across waves: blocks of 8 waves (two per SIMD, waves w and w + 4
// sharing one), waves 0-3 running two MFMA chains and waves 4-7 sixteen FP32
// FMAs per iteration on 8 chains. With MFMA and vector work in different
// waves of one SIMD the time shows whether an MFMA holds up only its own
// wave's vector issue or the whole SIMD's.
__global__ __launch_bounds__(512) void k_probe_split(int iters, float* __restrict__ sink) {
    float s = 0.0f;
    if ((threadIdx.x >> 6) < 4) {
        pbf16x8 a, b;
#pragma unroll
        for (int i = 0; i < 8; i++) {
            a[i] = (__bf16)(1e-3f * (float)(threadIdx.x + i));
            b[i] = (__bf16)(1e-3f * (float)(i + 1));
        }
        pf32x16 acc[2] = {};
        for (int it = 0; it < iters; it++) {
#pragma unroll
            for (int m = 0; m < 2; m++) acc[m] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, acc[m], 0, 0, 0);
        }
        s = acc[0][0] + acc[1][0];
    } else {
        float v[kProbeChains];
#pragma unroll
        for (int c = 0; c < kProbeChains; c++) v[c] = 1e-6f * (float)(threadIdx.x + c + 1);
        for (int it = 0; it < iters; it++) {
#pragma unroll
            for (int j = 0; j < 16; j++) v[j % kProbeChains] = fmaf(v[j % kProbeChains], 0.999999f, 1.0e-7f);
        }
#pragma unroll
        for (int c = 0; c < kProbeChains; c++) s += v[c];
    }
    if (s == 12345.0f) sink[threadIdx.x & (kProbeThreads - 1)] = s;
}

}  // namespace
}  // namespace mdgmi

using namespace mdgmi;

extern "C" int mdgmi_probe_rates(double* out_host) {
    if (!out_host) return MDGMI_E_NULL;
    int dev = 0, wall_khz = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&wall_khz, hipDeviceAttributeWallClockRate, dev) != hipSuccess || wall_khz <= 0)
        return MDGMI_E_HIP;
    const int blocks = device_cu_count() * 8;  // 8 waves per SIMD
    float* sink = nullptr;
    unsigned long long* clk = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    auto release = [&]() {
        if (e0) (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
        if (sink) (void)hipFree(sink);
        if (clk) (void)hipFree(clk);
    };
    if (hipMalloc(&sink, sizeof(float) * kProbeThreads) != hipSuccess ||
        hipMalloc(&clk, 2 * sizeof(unsigned long long)) != hipSuccess || hipEventCreate(&e0) != hipSuccess ||
        hipEventCreate(&e1) != hipSuccess) {
        release();
        return MDGMI_E_HIP;
    }
    int rc = MDGMI_OK;
    const int mix_blocks = device_cu_count() * 2;  // 2 waves per SIMD
    auto run = [&](int op, int iters, double ops_per_lane_iter, double* rate, double* hz) {
        const int nb = op == 6 ? device_cu_count() : op >= 3 ? mix_blocks : blocks;
        for (int rep = 0; rep < 2; rep++) {  // the first launch warms up
            (void)hipEventRecord(e0, nullptr);
            if (op == 0)
                hipLaunchKernelGGL(k_probe<0>, dim3(nb), dim3(kProbeThreads), 0, nullptr, iters, 0.5f, sink, clk);
            else if (op == 1)
                hipLaunchKernelGGL(k_probe<1>, dim3(nb), dim3(kProbeThreads), 0, nullptr, iters, 0.5f, sink, clk);
            else if (op == 2)
                hipLaunchKernelGGL(k_probe_mfma, dim3(nb), dim3(kProbeThreads), 0, nullptr, iters, sink);
            else if (op == 3)
                hipLaunchKernelGGL(k_probe_mix<0>, dim3(nb), dim3(kProbeThreads), 0, nullptr, iters, sink);
            else if (op == 4)
                hipLaunchKernelGGL(k_probe_mix<4>, dim3(nb), dim3(kProbeThreads), 0, nullptr, iters, sink);
            else if (op == 5)
                hipLaunchKernelGGL(k_probe_mix<8>, dim3(nb), dim3(kProbeThreads), 0, nullptr, iters, sink);
            else
                hipLaunchKernelGGL(k_probe_split, dim3(device_cu_count()), dim3(512), 0, nullptr, iters, sink);
            (void)hipEventRecord(e1, nullptr);
        }
        float ms = 0.0f;
        unsigned long long c[2] = {0, 0};
        if (hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&ms, e0, e1) != hipSuccess ||
            hipMemcpy(c, clk, sizeof(c), hipMemcpyDeviceToHost) != hipSuccess) {
            rc = MDGMI_E_HIP;
            return;
        }
        *rate = (double)nb * (op == 6 ? 512 : kProbeThreads) * iters * ops_per_lane_iter / (ms * 1e-3);
        if (hz) *hz = c[1] > 0 ? (double)c[0] / ((double)c[1] / (wall_khz * 1e3)) : 0.0;
    };
    // exponentials and FMAs per lane and iteration; MFMA: 4 per wave and
    // iteration of 2 * 32 * 32 * 16 flops each, counted per lane (/ 64)
    run(0, 4096, kProbeChains, &out_host[0], &out_host[1]);
    run(1, 16384, kProbeChains, &out_host[2], &out_host[3]);
    run(2, 2048, 4.0 * 2 * 32 * 32 * 16 / 64.0, &out_host[4], nullptr);
    // MFMA flops per second at two waves per SIMD with 0, 4 and 8 FMAs per MFMA
    for (int k = 0; k < 3; k++) run(3 + k, 8192, 2.0 * 2 * 32 * 32 * 16 / 64.0, &out_host[5 + k], nullptr);
    // MFMA and FMA waves side by side (k_probe_split): iterations per second
    // of each SIMD, an iteration being two MFMAs in one of its waves and
    // sixteen FMAs in the other
    run(6, 8192, 1.0 / (512.0 * device_cu_count()), &out_host[8], nullptr);
    release();
    return rc;
}
