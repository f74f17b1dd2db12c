// Attainable-peak probes for the roofline fractions (include/rara_peak.h): a
// streaming device copy for HBM bandwidth, and a loop of independent unpacked
// FP32 FMAs for the vector ALU rate.  Built with packed FP32 disabled, like
// the renderer, so the FMA loop issues v_fma_f32 / v_fmac_f32, one per lane
// and cycle-slot: the ceiling the renderer's kernels can reach.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "rara_peak.h"

namespace {

// Each thread moves kCopyUnroll 16-byte words per step, their loads all issued
// before the stores, so that many loads per wave are in flight.
constexpr int kCopyUnroll = 4;
typedef float v4f __attribute__((ext_vector_type(4)));

__global__ __launch_bounds__(256) void copy_kernel(const v4f* __restrict__ src, v4f* __restrict__ dst, int64_t n4)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (; i + (kCopyUnroll - 1) * stride < n4; i += kCopyUnroll * stride) {
        v4f v[kCopyUnroll];
#pragma unroll
        for (int u = 0; u < kCopyUnroll; ++u) v[u] = __builtin_nontemporal_load(src + i + u * stride);
#pragma unroll
        for (int u = 0; u < kCopyUnroll; ++u) __builtin_nontemporal_store(v[u], dst + i + u * stride);
    }
    for (; i < n4; i += stride) dst[i] = src[i];
}

constexpr int kChains = 16;   // independent FMA chains per lane (hide the FMA latency)

__global__ __launch_bounds__(256) void fma_kernel(float* __restrict__ out, int iters, float a, float b)
{
    float x[kChains];
#pragma unroll
    for (int k = 0; k < kChains; ++k) x[k] = (float)threadIdx.x * 1e-3f + (float)k;
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int k = 0; k < kChains; ++k) x[k] = __builtin_fmaf(x[k], a, b);
    }
    float s = 0.0f;
#pragma unroll
    for (int k = 0; k < kChains; ++k) s += x[k];
    // never true for the arguments the host passes; keeps the chains live
    if (s == -1.0f) out[(int64_t)blockIdx.x * blockDim.x + threadIdx.x] = s;
}

}  // namespace

extern "C" {

int rara_peak_copy(void* dst, const void* src, size_t bytes, int blocks, void* stream)
{
    if (!dst || !src || bytes % 16 != 0 || blocks < 1) return 1;
    hipLaunchKernelGGL(copy_kernel, dim3((unsigned)blocks), dim3(256), 0, static_cast<hipStream_t>(stream),
                       static_cast<const v4f*>(src), static_cast<v4f*>(dst), (int64_t)(bytes / 16));
    return hipGetLastError() == hipSuccess ? 0 : 3;
}

int rara_peak_fma(float* out, int blocks, int iters, void* stream)
{
    if (!out || blocks < 1 || iters < 1) return 1;
    hipLaunchKernelGGL(fma_kernel, dim3((unsigned)blocks), dim3(256), 0, static_cast<hipStream_t>(stream), out,
                       iters, 0.999999f, 1e-6f);
    return hipGetLastError() == hipSuccess ? 0 : 3;
}

double rara_peak_fma_flops(int blocks, int iters) { return 2.0 * kChains * 256.0 * (double)blocks * (double)iters; }

}  // extern "C"
