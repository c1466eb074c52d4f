// Measurements of the device's achievable rates, the denominators of the
// march's rooflines (include/frt.h, frt_microbench): HBM bandwidth from a
// streaming copy, and the rate of FP32 atomic additions whose result is not
// used at random addresses of a buffer (the form of the march's deposits
// into the rate field).
#include "frt.h"
#include "frt_internal.h"

#include <hip/hip_runtime.h>

#include <cstdint>

namespace {

constexpr int MB_BLOCK = 256;

// b[i] = a[i], 16 bytes per lane and iteration, a grid-stride loop.
__global__ void __launch_bounds__(MB_BLOCK) k_mb_copy(const float4* __restrict__ a, float4* __restrict__ b, size_t n)
{
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) b[i] = a[i];
}

// The same with four 16-byte loads in flight per lane before their stores,
// and non-temporal accesses (the copied data is not read again).
typedef float f4v __attribute__((ext_vector_type(4)));
__global__ void __launch_bounds__(MB_BLOCK) k_mb_copy4(const f4v* __restrict__ a, f4v* __restrict__ b, size_t n)
{
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (; i + 3 * stride < n; i += 4 * stride) {
        const f4v v0 = __builtin_nontemporal_load(a + i);
        const f4v v1 = __builtin_nontemporal_load(a + i + stride);
        const f4v v2 = __builtin_nontemporal_load(a + i + 2 * stride);
        const f4v v3 = __builtin_nontemporal_load(a + i + 3 * stride);
        __builtin_nontemporal_store(v0, b + i);
        __builtin_nontemporal_store(v1, b + i + stride);
        __builtin_nontemporal_store(v2, b + i + 2 * stride);
        __builtin_nontemporal_store(v3, b + i + 3 * stride);
    }
    for (; i < n; i += stride) b[i] = a[i];
}

// Each lane adds 1 at `per_lane` addresses drawn by a 32-bit LCG from its
// global index (Numerical Recipes constants), modulo the buffer's slots.
__global__ void __launch_bounds__(MB_BLOCK) k_mb_atomic(float* __restrict__ buf, uint32_t slots, int per_lane, uint32_t seed)
{
    uint32_t s = (uint32_t)(blockIdx.x * blockDim.x + threadIdx.x) * 2654435761u ^ seed;
    for (int k = 0; k < per_lane; k++) {
        s = s * 1664525u + 1013904223u;
        atomicAdd(buf + (s % slots), 1.0f);
    }
}

}  // namespace

namespace frt {

hipError_t microbench_copy(const void* a, void* b, size_t bytes, int variant, hipStream_t s)
{
    const size_t n = bytes / 16;
    if (variant == 0)
        hipLaunchKernelGGL(k_mb_copy, dim3(device_cu_count() * 8), dim3(MB_BLOCK), 0, s, (const float4*)a, (float4*)b, n);
    else
        hipLaunchKernelGGL(k_mb_copy4, dim3(device_cu_count() * 4), dim3(MB_BLOCK), 0, s, (const f4v*)a, (f4v*)b, n);
    return hipGetLastError();
}

hipError_t microbench_atomic(float* buf, uint32_t slots, int per_lane, int grid, uint32_t seed, hipStream_t s)
{
    hipLaunchKernelGGL(k_mb_atomic, dim3(grid), dim3(MB_BLOCK), 0, s, buf, slots, per_lane, seed);
    return hipGetLastError();
}

}  // namespace frt
