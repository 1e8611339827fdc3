// Device probes that measure two roofs of the coarse vote on the GPU it runs
// on: the rate of conflict-free 32-bit LDS atomic adds over all compute units,
// and the HBM bandwidth of a plain streaming copy.  Built into its own small
// library (libaoresp_probe.so) for the benchmark; not part of libaoresp.
#include <hip/hip_runtime.h>

#include <cstdint>

namespace {

constexpr int kThreads = 1024;
constexpr int kWords = 32768;   // 128 KiB of LDS per work-group, like the vote's tiles

// Every lane adds to its own words, `reps` times: thread t hits words
// t + 1024 i, so the 64 lanes of a wave hit 64 consecutive words (distinct
// banks) in every instruction.  The sum of the tile is written out so that
// nothing is optimised away.
__global__ __launch_bounds__(kThreads) void k_lds_add(uint32_t* out, int reps) {
    extern __shared__ uint32_t tile[];
    for (int t = threadIdx.x; t < kWords; t += kThreads) tile[t] = 0u;
    __syncthreads();
    uint32_t* p = tile + threadIdx.x;
#pragma unroll 1
    for (int r = 0; r < reps; ++r) {
#pragma unroll
        for (int i = 0; i < kWords / kThreads; ++i) atomicAdd(p + i * kThreads, 1u);
    }
    __syncthreads();
    uint32_t s = 0;
    for (int t = threadIdx.x; t < kWords; t += kThreads) s += tile[t];
    atomicAdd(out, s);
}

__global__ void k_copy(const float4* __restrict__ src, float4* __restrict__ dst, size_t n4) {
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n4; i += (size_t)gridDim.x * blockDim.x)
        dst[i] = src[i];
}

}  // namespace

extern "C" {

// Conflict-free LDS atomic adds per second over `blocks` work-groups of 1024
// threads (one per CU when blocks = CU count); 0 on a HIP error.
double aoresp_probe_lds_atomics(int blocks, int reps) {
    if (blocks < 1 || reps < 1) return 0.0;
    if (hipFuncSetAttribute((const void*)k_lds_add, hipFuncAttributeMaxDynamicSharedMemorySize,
                            kWords * 4) != hipSuccess)
        return 0.0;
    uint32_t* out = nullptr;
    if (hipMalloc(&out, 4) != hipSuccess) return 0.0;
    hipEvent_t a, b;
    (void)hipEventCreate(&a);
    (void)hipEventCreate(&b);
    hipLaunchKernelGGL(k_lds_add, dim3(blocks), dim3(kThreads), kWords * 4, 0, out, reps);   // warm-up
    (void)hipEventRecord(a, 0);
    hipLaunchKernelGGL(k_lds_add, dim3(blocks), dim3(kThreads), kWords * 4, 0, out, reps);
    (void)hipEventRecord(b, 0);
    float ms = 0.0f;
    const bool ok = hipEventSynchronize(b) == hipSuccess && hipEventElapsedTime(&ms, a, b) == hipSuccess;
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    (void)hipFree(out);
    if (!ok || ms <= 0.0f) return 0.0;
    return (double)blocks * kWords * (double)reps / (ms * 1e-3);
}

// Bytes per second (read + write) of a streaming device copy of `bytes`.
double aoresp_probe_copy(size_t bytes, int reps) {
    const size_t n4 = bytes / 16;
    if (n4 == 0 || reps < 1) return 0.0;
    float4 *src = nullptr, *dst = nullptr;
    if (hipMalloc(&src, n4 * 16) != hipSuccess) return 0.0;
    if (hipMalloc(&dst, n4 * 16) != hipSuccess) {
        (void)hipFree(src);
        return 0.0;
    }
    (void)hipMemset(src, 0, n4 * 16);
    hipEvent_t a, b;
    (void)hipEventCreate(&a);
    (void)hipEventCreate(&b);
    hipLaunchKernelGGL(k_copy, dim3(4096), dim3(256), 0, 0, src, dst, n4);
    (void)hipEventRecord(a, 0);
    for (int r = 0; r < reps; ++r) hipLaunchKernelGGL(k_copy, dim3(4096), dim3(256), 0, 0, src, dst, n4);
    (void)hipEventRecord(b, 0);
    float ms = 0.0f;
    const bool ok = hipEventSynchronize(b) == hipSuccess && hipEventElapsedTime(&ms, a, b) == hipSuccess;
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    (void)hipFree(src);
    (void)hipFree(dst);
    if (!ok || ms <= 0.0f) return 0.0;
    return 2.0 * (double)(n4 * 16) * reps / (ms * 1e-3);
}

}  // extern "C"
