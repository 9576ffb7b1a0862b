// Calibration kernel for the vector-ALU counters (measurement aid of the
// benchmark, not part of the mapping library): every lane runs 16
// independent FP32 fused multiply-add chains, so the kernel issues a known
// number of VALU instructions (16 v_fma_f32 per wavefront per iteration;
// packed FP32 is disabled in this build) at the rate the SIMDs sustain.
// Profiling it next to the mapping kernels fixes the scale of counters such
// as SQ_INSTS_VALU and SQ_ACTIVE_INST_VALU against the issue rate the
// hardware actually reaches, and its FLOP rate is the measured non-packed
// FP32 vector peak.
#include <hip/hip_runtime.h>

#include <cstdint>

namespace {

constexpr int kChains = 16;

__global__ void __launch_bounds__(256) k_valu_fma(float *out, int iters, float a, float b)
{
    float x[kChains];
#pragma unroll
    for (int c = 0; c < kChains; c++) x[c] = (float)(threadIdx.x + c) * 1e-3f;
    for (int i = 0; i < iters; i++) {
#pragma unroll
        for (int c = 0; c < kChains; c++) x[c] = fmaf(x[c], a, b);
    }
    float s = 0.0f;
#pragma unroll
    for (int c = 0; c < kChains; c++) s += x[c];
    if (s == 1234.5f) out[blockIdx.x] = s;  // keeps the chains live; never true for these inputs
}

}  // namespace

// Runs the calibration kernel `reps` times on `blocks` workgroups of 256
// threads with `iters` iterations; returns the average device time per launch
// (ms) and the FP32 fused multiply-adds of one launch.  0 on success, else a
// HIP error code.
extern "C" int em_calib_valu(int device, int blocks, int iters, int reps, double *ms_per_launch, double *fma_per_launch)
{
    hipError_t e = hipSetDevice(device);
    if (e != hipSuccess) return (int)e;
    float *out = nullptr;
    if ((e = hipMalloc(&out, sizeof(float) * (size_t)blocks)) != hipSuccess) return (int)e;
    hipEvent_t t0, t1;
    (void)hipEventCreate(&t0);
    (void)hipEventCreate(&t1);
    hipLaunchKernelGGL(k_valu_fma, dim3((unsigned)blocks), dim3(256), 0, nullptr, out, iters, 0.9999999f, 1e-7f);
    (void)hipEventRecord(t0, nullptr);
    for (int r = 0; r < reps; r++)
        hipLaunchKernelGGL(k_valu_fma, dim3((unsigned)blocks), dim3(256), 0, nullptr, out, iters, 0.9999999f, 1e-7f);
    (void)hipEventRecord(t1, nullptr);
    e = hipEventSynchronize(t1);
    float ms = 0.0f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, t0, t1);
    (void)hipEventDestroy(t0);
    (void)hipEventDestroy(t1);
    (void)hipFree(out);
    if (e != hipSuccess) return (int)e;
    *ms_per_launch = (double)ms / (double)reps;
    *fma_per_launch = (double)blocks * 256.0 * (double)iters * (double)kChains;
    return 0;
}
