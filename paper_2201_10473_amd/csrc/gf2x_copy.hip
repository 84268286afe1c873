// gf2x_copy.hip -- copies between pinned host memory and device memory done
// by kernels: the GPU reads or writes the host pages over PCIe, so a caller
// that stages its inputs and results in pinned memory (the serving loop)
// issues no DMA copy.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>

#include "gf2x_copy.hpp"

namespace gf2x {

// dst0[0 .. n0) = src0[0 .. n0) and dst1[0 .. n1) = src1[0 .. n1), 64-bit
// words; the sources are device views of pinned host buffers.
__global__ __launch_bounds__(256) void k_pull(const uint64_t *src0, uint64_t *dst0, uint64_t n0,
                                              const uint64_t *src1, uint64_t *dst1, uint64_t n1) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n0 + n1; i += stride) {
        if (i < n0) dst0[i] = src0[i];
        else dst1[i - n0] = src1[i - n0];
    }
}

// dst[0 .. n) = src[0 .. n), 64-bit words, dst a device view of a pinned
// host buffer; each thread's writes reach system scope before it ends, so a
// host that has seen the kernel complete (an event) reads the new values.
__global__ __launch_bounds__(256) void k_push(const uint64_t *src, uint64_t *dst, uint64_t n) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n; i += stride) dst[i] = src[i];
    __threadfence_system();
}

hipError_t launch_push(const uint64_t *src, uint64_t *dst, uint64_t n, hipStream_t s) {
    if (n == 0) return hipSuccess;
    const uint32_t blocks = (uint32_t)std::min<uint64_t>((n + 255) / 256, 1024);
    hipLaunchKernelGGL(k_push, dim3(blocks), dim3(256), 0, s, src, dst, n);
    return hipGetLastError();
}

hipError_t launch_pull(const uint64_t *src0, uint64_t *dst0, uint64_t n0, const uint64_t *src1, uint64_t *dst1,
                       uint64_t n1, hipStream_t s) {
    const uint64_t total = n0 + n1;
    if (total == 0) return hipSuccess;
    const uint32_t blocks = (uint32_t)std::min<uint64_t>((total + 255) / 256, 1024);
    hipLaunchKernelGGL(k_pull, dim3(blocks), dim3(256), 0, s, src0, dst0, n0, src1, dst1, n1);
    return hipGetLastError();
}

}  // namespace gf2x
