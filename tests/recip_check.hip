// Device check of the library's reciprocal (recip_1_4 in geometry.h) against
// the correctly rounded division of the same build, for every binary32 x in
// [1, 4).  Prints the number of mismatches; test code only.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>

#include "../paper_2502_06337_amd/csrc/geometry.h"

__global__ void k_check(uint32_t base, uint32_t count, unsigned long long* bad) {
    const uint32_t stride = gridDim.x * blockDim.x;
    unsigned long long nbad = 0;
    for (uint32_t t = blockIdx.x * blockDim.x + threadIdx.x; t < count; t += stride) {
        const float x = __uint_as_float(base + t);
        if (__float_as_uint(1.0f / x) != __float_as_uint(aoresp::recip_1_4(x))) ++nbad;
    }
    if (nbad) atomicAdd(bad, nbad);
}

int main() {
    const uint32_t lo = 0x3f800000u, hi = 0x40800000u;   // [1.0f, 4.0f)
    unsigned long long* d_bad = nullptr;
    unsigned long long bad = 0;
    if (hipMalloc(&d_bad, sizeof(bad)) != hipSuccess) return 2;
    if (hipMemcpy(d_bad, &bad, sizeof(bad), hipMemcpyHostToDevice) != hipSuccess) return 2;
    hipLaunchKernelGGL(k_check, dim3(4096), dim3(256), 0, 0, lo, hi - lo, d_bad);
    if (hipDeviceSynchronize() != hipSuccess) return 3;
    if (hipMemcpy(&bad, d_bad, sizeof(bad), hipMemcpyDeviceToHost) != hipSuccess) return 3;
    std::printf("checked %u values in [1, 4): %llu mismatches\n", hi - lo, bad);
    (void)hipFree(d_bad);
    return bad == 0 ? 0 : 1;
}
