// Streaming bandwidth probe: the rate the GPU sustains for plain 16-byte reads
// or copies over a large buffer, the measured ceiling that the hop kernels are
// compared with (they read about eight bytes for every byte they write).
#include <hip/hip_runtime.h>

#include <cstdint>

namespace tmqcd {
namespace {

// xor of every 32-bit word into *xor_out (the result keeps the loads, and lets a test check them)
__global__ __launch_bounds__(256) void probe_read_kernel(const uint4* __restrict__ a, int64_t n, unsigned* xor_out) {
    unsigned acc = 0;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
        const uint4 v = a[i];
        acc ^= v.x ^ v.y ^ v.z ^ v.w;
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) acc ^= __shfl_xor(acc, off, 64);
    if ((threadIdx.x & 63) == 0) atomicXor(xor_out, acc);
}

__global__ __launch_bounds__(256) void probe_copy_kernel(const uint4* __restrict__ a, uint4* __restrict__ b,
                                                         int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) b[i] = a[i];
}

}  // namespace

hipError_t launch_hbm_probe(const void* src, void* dst, int64_t bytes, int grid, unsigned* xor_out, hipStream_t s) {
    const int64_t n = bytes / 16;
    if (dst)
        hipLaunchKernelGGL(probe_copy_kernel, dim3(grid), dim3(256), 0, s, static_cast<const uint4*>(src),
                           static_cast<uint4*>(dst), n);
    else
        hipLaunchKernelGGL(probe_read_kernel, dim3(grid), dim3(256), 0, s, static_cast<const uint4*>(src), n,
                           xor_out);
    return hipGetLastError();
}

}  // namespace tmqcd
