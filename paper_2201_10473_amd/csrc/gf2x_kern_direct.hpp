// gf2x_kern_direct.hpp -- the per-class kernels of the direct classes (one
// product inside one workgroup).  The classes are instantiated in several
// translation units (gf2x_kern_d<G>.hip, G = class id mod kDirectGroups) so
// that the library compiles in parallel; each unit exports the handles of its
// kernels through direct_kernels_<G>(), which returns its k_mixed<G>.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "gf2x_launch.hpp"
#include "gf2x_product.hpp"

namespace gf2x {

template <class Sch>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(waves_per_simd<Sch>()))) void k_single(
    const uint64_t *a, const uint64_t *b, uint64_t *c, u32 n, u32 kind) {
    extern __shared__ u32 smem[];
    one_product<Sch>(a, b, c, n, kind, smem);
}

// Persistent workgroups over a batch whose items all use class Sch.
template <class Sch>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(waves_per_simd<Sch>()))) void k_batched(
    const DevItem *items, u32 count, uint64_t *c_base, const uint64_t *a_base, const uint64_t *b_base) {
    extern __shared__ u32 smem[];
    for (u32 i = blockIdx.x; i < count; i += gridDim.x) {
        const DevItem it = items[i];
        one_product<Sch>(a_base + it.a_off, b_base + it.b_off, c_base + it.c_off, it.n, it.kind, smem);
    }
}

// Persistent workgroups over a batch of mixed classes whose items take their
// class from the per-size table (device-resident descriptors): this kernel
// computes the items whose class is in group G and skips the others; the
// host launches the kernel of every group.  A descriptor with an invalid n or
// kind is skipped (its output is not written) and counted in *bad by the
// group-0 kernel.
template <int G>
__global__ __launch_bounds__(NT) void k_mixed(const DevItem *items, u32 count, uint64_t *c_base,
                                              const uint64_t *a_base, const uint64_t *b_base,
                                              const uint8_t *cls_of_w32, u32 *bad) {
    extern __shared__ u32 smem[];
    for (u32 i = blockIdx.x; i < count; i += gridDim.x) {
        const DevItem it = items[i];
        if (it.n == 0 || it.n > kMaxBits || it.kind > kKindFull) {  // invalid device descriptor
            if (G == 0 && tid() == 0) __hip_atomic_fetch_add(bad, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            continue;
        }
        const u32 cls = (u32)cls_of_w32[(it.n + 31u) / 32u];
        const uint64_t *a = a_base + it.a_off;
        const uint64_t *b = b_base + it.b_off;
        uint64_t *c = c_base + it.c_off;
        switch (cls) {
#define GF2X_MIXED_CASE(id, name, T)                                                              \
    case id:                                                                                      \
        if constexpr (id % kDirectGroups == G) one_product<T>(a, b, c, it.n, it.kind, smem); \
        break;
            GF2X_CLASS_LIST(GF2X_MIXED_CASE)
#undef GF2X_MIXED_CASE
            default: break;
        }
    }
}

// Records the kernels of class ID when it belongs to group G.
template <int G, int ID, class Sch>
void direct_handles(const void **single, const void **batched) {
    if constexpr (ID % kDirectGroups == G) {
        single[ID] = reinterpret_cast<const void *>(&k_single<Sch>);
        batched[ID] = reinterpret_cast<const void *>(&k_batched<Sch>);
    }
}

}  // namespace gf2x

#define GF2X_DIRECT_HANDLE(id, name, T) direct_handles<GF2X_GROUP, id, T>(single, batched);
#define GF2X_DIRECT_GROUP_BODY()                                                    \
    namespace gf2x {                                                                \
    const void *GF2X_GROUP_FN(const void **single, const void **batched) {          \
        GF2X_CLASS_LIST(GF2X_DIRECT_HANDLE)                                         \
        return reinterpret_cast<const void *>(&k_mixed<GF2X_GROUP>);                \
    }                                                                               \
    }
