// gf2x_launch.hpp -- interface between the kernel translation units: the
// host-side launchers (gf2x_kernels.hip) obtain the handles of the kernels
// instantiated in gf2x_kern_*.hip through these functions.  Internal.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "gf2x_internal.hpp"

namespace gf2x {

// Direct classes are spread over this many translation units by id.
constexpr int kDirectGroups = 4;

// Fill single[id] / batched[id] for the direct classes of group G; returns
// the group's kernel for batches whose classes come from the size table.
const void *direct_kernels_0(const void **single, const void **batched);
const void *direct_kernels_1(const void **single, const void **batched);
const void *direct_kernels_2(const void **single, const void **batched);
const void *direct_kernels_3(const void **single, const void **batched);

// Staged classes (gf2x_kern_staged.hip): LDS limits of their kernels.
hipError_t prepare_staged_kernels();

// Resident workgroups per CU of kernel fn at a dynamic LDS size (cached).
int occupancy(const void *fn, int lds_bytes);

// Descriptors of the np point products of each of count staged items.
hipError_t launch_child_items(uint32_t count, uint32_t S1, uint32_t np, uint32_t child_cls, DevItem *out,
                              hipStream_t s);

}  // namespace gf2x
