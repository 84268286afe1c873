// gf2x_inv.hip -- kernels of the inversion in F2[X]/(X^n - 1): repeated
// squaring as a bit permutation, and the gathers that move operands between
// the caller's buffers and the contiguous working buffers.
//
// In characteristic 2, squaring is linear: (sum a_i X^i)^2 = sum a_i X^(2i),
// so squaring j times modulo X^n - 1 sends coefficient i to i * 2^j mod n.
// Output bit t is input bit t * 2^(-j) mod n; the permutation depends only on
// the public n and j, never on operand bits (constant time).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "gf2x_internal.hpp"

namespace gf2x {

// out item i (W words at out_base + (out_off ? out_off[i] : i * W)) = in item
// i (W words at in + i * W) squared j times, with inv = 2^(-j) mod n.  One
// workgroup per item: the item is staged in LDS (dynamic, W words), then each
// thread builds output words: bit t of the result is bit s_t = t * inv mod n
// of the input, with s_(t+1) = s_t + inv reduced by one conditional
// subtraction.  Bits >= n of the last word are written zero.
__global__ __launch_bounds__(256) void k_frobenius(const uint64_t *in, uint64_t *out_base, const uint64_t *out_off,
                                                   uint32_t n, uint32_t W, uint32_t inv) {
    extern __shared__ uint64_t item[];
    const uint32_t i = blockIdx.x;
    const uint64_t *src = in + (uint64_t)i * W;
    for (uint32_t w = threadIdx.x; w < W; w += blockDim.x) item[w] = src[w];
    __syncthreads();
    uint64_t *dst = out_base + (out_off ? out_off[i] : (uint64_t)i * W);
    for (uint32_t w = threadIdx.x; w < W; w += blockDim.x) {
        uint32_t s = (uint32_t)(((uint64_t)(64u * w) * inv) % n);
        uint64_t v = 0;
        for (uint32_t b = 0; b < 64; ++b) {
            const uint32_t t = 64u * w + b;
            const uint64_t bit = (item[s >> 6] >> (s & 63u)) & 1ull;
            v |= (t < n ? bit : 0ull) << b;
            s += inv;
            s = s >= n ? s - n : s;  // s, inv < n: one subtraction reduces
        }
        dst[w] = v;
    }
}

// out item i (contiguous, W words) = the W words at in_base + in_off[i], bits
// >= n cleared.
__global__ void k_gather_items(const uint64_t *in_base, const uint64_t *in_off, uint64_t *out, uint32_t n, uint32_t W,
                               uint32_t count) {
    const uint64_t g = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
    if (g >= (uint64_t)count * W) return;
    const uint32_t i = (uint32_t)(g / W), w = (uint32_t)(g - (uint64_t)i * W);
    uint64_t v = in_base[in_off[i] + w];
    const uint32_t s = n % 64u;
    if (w == W - 1 && s) v &= (1ull << s) - 1ull;
    out[g] = v;
}

hipError_t launch_frobenius(const uint64_t *in, uint64_t *out_base, const uint64_t *out_off, uint32_t n, uint32_t count,
                            uint32_t inv, hipStream_t s) {
    const uint32_t W = (n + 63u) / 64u;  // at most 2048 words (16 KB of LDS) for n <= 131072
    if (count == 0) return hipSuccess;
    hipLaunchKernelGGL(k_frobenius, dim3(count), dim3(256), W * 8, s, in, out_base, out_off, n, W, inv);
    return hipGetLastError();
}

hipError_t launch_gather_items(const uint64_t *in_base, const uint64_t *in_off, uint64_t *out, uint32_t n,
                               uint32_t count, hipStream_t s) {
    const uint32_t W = (n + 63u) / 64u;
    const uint64_t total = (uint64_t)count * W;
    hipLaunchKernelGGL(k_gather_items, dim3((uint32_t)((total + 255) / 256)), dim3(256), 0, s, in_base, in_off, out, n,
                       W, count);
    return hipGetLastError();
}

}  // namespace gf2x
