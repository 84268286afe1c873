// gf2x_kern_fused.hip -- one persistent launch over a batch of uneven sizes:
// every workgroup takes the next item from a work queue (items ordered by
// decreasing cost) and runs the item's direct class, whichever of the fused
// set it is.  The fused set is the direct classes that the schedule table
// gives (or has given) the six ring sizes 12323 ... 57637.  A launch takes
// the LDS of the largest class it holds.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>

#include "gf2x_launch.hpp"
#include "gf2x_product.hpp"

namespace gf2x {

// X(fused index, class id, schedule type)
#define GF2X_FUSED_LIST(X) \
    X(0, 7, Class7)        \
    X(1, 10, Class10)      \
    X(2, 13, Class13)      \
    X(3, 14, Class14)      \
    X(4, 15, Class15)      \
    X(5, 17, Class17)      \
    X(6, 25, Class25)      \
    X(7, 26, Class26)      \
    X(8, 33, Class33)      \
    X(9, 35, Class35)      \
    X(10, 36, Class36)     \
    X(11, 37, Class37)     \
    X(12, 39, Class39)

#define GF2X_FUSED_LDS(i, id, T) (lds_words<T>() * 4),
constexpr int kFusedLdsList[] = {GF2X_FUSED_LIST(GF2X_FUSED_LDS)};
constexpr int fused_lds() {
    int m = 0;
    for (int v : kFusedLdsList) m = v > m ? v : m;
    return m;
}
constexpr int kFusedLds = fused_lds();

// queue[0]: next item; queue[1]: workgroups that have left.  Both start at
// zero; the last workgroup to leave sets them back to zero, so the launch can
// be replayed (graphs) without a separate reset.
__global__ __launch_bounds__(NT) void k_fused(const DevItem *items, u32 count, uint64_t *c_base,
                                              const uint64_t *a_base, const uint64_t *b_base, u32 *queue) {
    extern __shared__ u32 smem[];
    __shared__ u32 next;
    for (;;) {
        if (tid() == 0) next = __hip_atomic_fetch_add(&queue[0], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __syncthreads();
        const u32 i = next;
        __syncthreads();  // every thread has read `next` before it is overwritten
        if (i >= count) break;
        const DevItem it = items[i];
        const uint64_t *a = a_base + it.a_off;
        const uint64_t *b = b_base + it.b_off;
        uint64_t *c = c_base + it.c_off;
        switch (it.cls) {
#define GF2X_FUSED_CASE(i, id, T) \
    case id: one_product<T>(a, b, c, it.n, it.kind, smem); break;
            GF2X_FUSED_LIST(GF2X_FUSED_CASE)
#undef GF2X_FUSED_CASE
            default: break;  // the host admits only classes of the fused set
        }
    }
    if (tid() == 0) {
        // every workgroup has made its last (failing) fetch on queue[0] before
        // it counts itself out, so the last one out can reset both
        const u32 out = __hip_atomic_fetch_add(&queue[1], 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
        if (out == gridDim.x - 1) {
            __hip_atomic_store(&queue[0], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_store(&queue[1], 0u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        }
    }
}

bool fused_class(int cls) {
    switch (cls) {
#define GF2X_FUSED_IS(i, id, T) case id:
        GF2X_FUSED_LIST(GF2X_FUSED_IS)
#undef GF2X_FUSED_IS
        return true;
        default: return false;
    }
}

hipError_t prepare_fused_kernel() {
    return hipFuncSetAttribute(reinterpret_cast<const void *>(&k_fused), hipFuncAttributeMaxDynamicSharedMemorySize,
                               kFusedLds);
}

hipError_t launch_fused(const DevItem *items, uint32_t count, int lds, uint64_t *c_base, const uint64_t *a_base,
                        const uint64_t *b_base, uint32_t *queue, int num_cu, hipStream_t s) {
    if (lds <= 0 || lds > kFusedLds) return hipErrorInvalidValue;
    const long long cap = (long long)num_cu * occupancy(reinterpret_cast<const void *>(&k_fused), lds);
    const uint32_t grid = (uint32_t)std::min<long long>(count, cap);
    if (grid == 0) return hipSuccess;
    hipLaunchKernelGGL(k_fused, dim3(grid), dim3(NT), lds, s, items, count, c_base, a_base, b_base, queue);
    return hipGetLastError();
}

}  // namespace gf2x
