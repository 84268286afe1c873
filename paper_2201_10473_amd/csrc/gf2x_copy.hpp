// gf2x_copy.hpp -- launchers of the copy kernels between pinned host memory
// and device memory (gf2x_copy.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace gf2x {

// dst0[0 .. n0) = src0[0 .. n0) and dst1[0 .. n1) = src1[0 .. n1), 64-bit
// words, the sources being device views of pinned host buffers.
hipError_t launch_pull(const uint64_t *src0, uint64_t *dst0, uint64_t n0, const uint64_t *src1, uint64_t *dst1,
                       uint64_t n1, hipStream_t s);

// dst[0 .. n) = src[0 .. n), 64-bit words, dst the device view of a pinned
// host buffer; the values are visible to the host once the kernel has
// completed.
hipError_t launch_push(const uint64_t *src, uint64_t *dst, uint64_t n, hipStream_t s);

}  // namespace gf2x
