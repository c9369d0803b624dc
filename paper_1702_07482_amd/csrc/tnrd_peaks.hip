// Throughput probes of the units the filter runs on: HBM copy, FP32 and
// BF16/FP16 matrix instructions, FP32 vector FMA and the hardware exp2.  They
// give the measured peaks against which the stage kernels' rates are read
// (the published figures are not re-derived here).
//
// Every probe except the copy works in registers only; each thread writes one
// float of its result to `sink` so that the loop is not removed.  The launch
// shapes are fixed (PK_BLOCKS x PK_THREADS threads) and the caller's `sink`
// holds PK_BLOCKS * PK_THREADS floats.
#include <hip/hip_runtime.h>

#include "tnrd.h"
#include "tnrd_fused_common.hpp"

namespace tnrd {

constexpr int PK_THREADS = 256;   // 4 waves
constexpr int PK_BLOCKS = 2048;   // 8 workgroups per compute unit on 256 CUs
constexpr int PK_CHAINS = 8;      // independent dependency chains per thread

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));

__global__ void __launch_bounds__(PK_THREADS) k_peak_copy(const float4 *__restrict__ src,
                                                          float4 *__restrict__ dst, size_t n)
{
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) dst[i] = src[i];
}

// v_mfma_f32_16x16x4_f32: 2 * 16 * 16 * 4 flop per instruction
__global__ void __launch_bounds__(PK_THREADS) k_peak_mfma_f32(int iters, float *sink)
{
    floatx4 acc[PK_CHAINS];
#pragma unroll
    for (int c = 0; c < PK_CHAINS; ++c) acc[c] = floatx4{0.f, 0.f, 0.f, 0.f};
    const float a = 1e-3f * (threadIdx.x & 63), b = 0.5f;
    for (int i = 0; i < iters; ++i)
#pragma unroll
        for (int c = 0; c < PK_CHAINS; ++c) acc[c] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, acc[c], 0, 0, 0);
    float s = 0.f;
#pragma unroll
    for (int c = 0; c < PK_CHAINS; ++c) s += acc[c][0] + acc[c][3];
    sink[blockIdx.x * blockDim.x + threadIdx.x] = s;
}

// v_mfma_f32_16x16x16_bf16: 2 * 16 * 16 * 16 flop per instruction
__global__ void __launch_bounds__(PK_THREADS) k_peak_mfma_bf16_k16(int iters, float *sink)
{
    floatx4 acc[PK_CHAINS];
#pragma unroll
    for (int c = 0; c < PK_CHAINS; ++c) acc[c] = floatx4{0.f, 0.f, 0.f, 0.f};
    const __bf16 x = (__bf16)(1e-3f * (threadIdx.x & 63));
    const bf16x4 a = {x, x, x, x};
    const short4v av = __builtin_bit_cast(short4v, a);
    for (int i = 0; i < iters; ++i)
#pragma unroll
        for (int c = 0; c < PK_CHAINS; ++c) acc[c] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(av, av, acc[c], 0, 0, 0);
    float s = 0.f;
#pragma unroll
    for (int c = 0; c < PK_CHAINS; ++c) s += acc[c][0] + acc[c][3];
    sink[blockIdx.x * blockDim.x + threadIdx.x] = s;
}

// v_mfma_f32_16x16x32_bf16: 2 * 16 * 16 * 32 flop per instruction
__global__ void __launch_bounds__(PK_THREADS) k_peak_mfma_bf16_k32(int iters, float *sink)
{
    floatx4 acc[PK_CHAINS];
#pragma unroll
    for (int c = 0; c < PK_CHAINS; ++c) acc[c] = floatx4{0.f, 0.f, 0.f, 0.f};
    const __bf16 x = (__bf16)(1e-3f * (threadIdx.x & 63));
    const bf16x8 a = {x, x, x, x, x, x, x, x};
    for (int i = 0; i < iters; ++i)
#pragma unroll
        for (int c = 0; c < PK_CHAINS; ++c) acc[c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, a, acc[c], 0, 0, 0);
    float s = 0.f;
#pragma unroll
    for (int c = 0; c < PK_CHAINS; ++c) s += acc[c][0] + acc[c][3];
    sink[blockIdx.x * blockDim.x + threadIdx.x] = s;
}

// FP32 vector FMA (unpacked): 2 flop per lane per instruction
__global__ void __launch_bounds__(PK_THREADS) k_peak_valu_fma(int iters, float *sink)
{
    float x[PK_CHAINS];
#pragma unroll
    for (int c = 0; c < PK_CHAINS; ++c) x[c] = 1e-3f * (threadIdx.x + c);
    const float a = 0.999f, b = 1e-4f;
    for (int i = 0; i < iters; ++i)
#pragma unroll
        for (int c = 0; c < PK_CHAINS; ++c) x[c] = fmaf(x[c], a, b);
    float s = 0.f;
#pragma unroll
    for (int c = 0; c < PK_CHAINS; ++c) s += x[c];
    sink[blockIdx.x * blockDim.x + threadIdx.x] = s;
}

// hardware exp2 (v_exp_f32): x <- 2^(-x) stays in (0.5, 1) for x in (0, 1)
__global__ void __launch_bounds__(PK_THREADS) k_peak_exp(int iters, float *sink)
{
    float x[PK_CHAINS];
#pragma unroll
    for (int c = 0; c < PK_CHAINS; ++c) x[c] = 0.25f + 1e-3f * ((threadIdx.x + c) & 255);
    for (int i = 0; i < iters; ++i)
#pragma unroll
        for (int c = 0; c < PK_CHAINS; ++c) x[c] = __builtin_amdgcn_exp2f(-x[c]);
    float s = 0.f;
#pragma unroll
    for (int c = 0; c < PK_CHAINS; ++c) s += x[c];
    sink[blockIdx.x * blockDim.x + threadIdx.x] = s;
}

}  // namespace tnrd

using namespace tnrd;

namespace {

// Average seconds of one launch over `reps` launches after one warm-up.
template <typename F>
int time_launch(F launch, int reps, hipStream_t st, double *sec)
{
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess) return TNRD_ERR_HIP;
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return TNRD_ERR_HIP;
    }
    int rc = TNRD_OK;
    launch();
    if (hipGetLastError() != hipSuccess || hipEventRecord(e0, st) != hipSuccess) rc = TNRD_ERR_HIP;
    for (int r = 0; r < reps && rc == TNRD_OK; ++r) launch();
    float ms = 0.f;
    if (rc == TNRD_OK && (hipGetLastError() != hipSuccess || hipEventRecord(e1, st) != hipSuccess ||
                          hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&ms, e0, e1) != hipSuccess))
        rc = TNRD_ERR_HIP;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    *sec = ms * 1e-3 / reps;
    return rc;
}

}  // namespace

extern "C" size_t tnrd_peaks_sink_floats(void) { return (size_t)PK_BLOCKS * PK_THREADS; }

extern "C" int tnrd_measure_peaks(const void *copy_src, void *copy_dst, size_t copy_bytes, float *sink,
                                  tnrd_peaks *out, void *stream)
{
    if (!copy_src || !copy_dst || !sink || !out || copy_bytes < 16 * 1024 * 1024 || copy_bytes % 16)
        return TNRD_ERR_ARG;
    hipStream_t st = (hipStream_t)stream;
    const dim3 grid(PK_BLOCKS), block(PK_THREADS);
    const double waves = (double)PK_BLOCKS * PK_THREADS / 64.0;
    const int it = 4096;  // loop trips per thread (x PK_CHAINS instructions)
    double sec = 0.0;
    int rc;

    const size_t n4 = copy_bytes / 16;
    rc = time_launch([&] {
        hipLaunchKernelGGL(k_peak_copy, dim3(4096), block, 0, st, (const float4 *)copy_src,
                           (float4 *)copy_dst, n4);
    }, 10, st, &sec);
    if (rc) return rc;
    out->copy_gbs = 2.0 * copy_bytes / sec * 1e-9;

    const double instr = waves * it * PK_CHAINS;  // per launch, per wave-instruction
    rc = time_launch([&] { hipLaunchKernelGGL(k_peak_mfma_f32, grid, block, 0, st, it, sink); }, 3, st, &sec);
    if (rc) return rc;
    out->mfma_f32_tflops = instr * 2.0 * 16 * 16 * 4 / sec * 1e-12;

    rc = time_launch([&] { hipLaunchKernelGGL(k_peak_mfma_bf16_k16, grid, block, 0, st, it, sink); }, 3, st, &sec);
    if (rc) return rc;
    out->mfma_bf16_k16_tflops = instr * 2.0 * 16 * 16 * 16 / sec * 1e-12;

    rc = time_launch([&] { hipLaunchKernelGGL(k_peak_mfma_bf16_k32, grid, block, 0, st, it, sink); }, 3, st, &sec);
    if (rc) return rc;
    out->mfma_bf16_k32_tflops = instr * 2.0 * 16 * 16 * 32 / sec * 1e-12;

    rc = time_launch([&] { hipLaunchKernelGGL(k_peak_valu_fma, grid, block, 0, st, 4 * it, sink); }, 3, st, &sec);
    if (rc) return rc;
    out->valu_f32_tflops = waves * 4 * it * PK_CHAINS * 64.0 * 2.0 / sec * 1e-12;

    rc = time_launch([&] { hipLaunchKernelGGL(k_peak_exp, grid, block, 0, st, it, sink); }, 3, st, &sec);
    if (rc) return rc;
    out->exp_per_s = waves * it * PK_CHAINS * 64.0 / sec;
    return TNRD_OK;
}
