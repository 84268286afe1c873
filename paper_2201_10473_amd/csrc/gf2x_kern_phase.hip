// gf2x_kern_phase.hip -- a batch of mixed sizes in three launches, whatever
// classes it holds: (1) the evaluation of every item whose class is staged,
// (2) every product computed inside one workgroup -- the point products of
// the staged items and the items of direct classes -- in one persistent
// launch, (3) the interpolation and fold of every staged item.  Kernel
// boundaries order the phases; nothing waits inside a kernel.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>

#include "gf2x_launch.hpp"
#include "gf2x_product.hpp"

namespace gf2x {

// Direct classes of the product phase: the child classes of every staged
// class, and the candidate direct classes of the six ring sizes (Toom-3 and
// Toom-4 over Karatsuba).  X(class id, type)
#define GF2X_PHASE_LIST(X) \
    X(7, Class7)           \
    X(9, Class9)           \
    X(10, Class10)         \
    X(13, Class13)         \
    X(14, Class14)         \
    X(15, Class15)         \
    X(17, Class17)         \
    X(21, Class21)         \
    X(22, Class22)         \
    X(23, Class23)         \
    X(24, Class24)         \
    X(25, Class25)         \
    X(26, Class26)         \
    X(33, Class33)         \
    X(34, Class34)         \
    X(35, Class35)         \
    X(36, Class36)         \
    X(37, Class37)         \
    X(38, Class38)         \
    X(39, Class39)         \
    X(40, Class40)

// (1) evaluation: staged item i reads its operands from a_base / b_base and
// writes its point operand pairs at ws + ws_off[2 i] (32-bit words).
__global__ __launch_bounds__(NT) void k_phase_eval(const DevItem *items, const uint64_t *ws_off, u32 count,
                                                   const uint64_t *a_base, const uint64_t *b_base, u32 *ws) {
    extern __shared__ u32 smem[];
    for (u32 i = blockIdx.x; i < count; i += gridDim.x) {
        const DevItem it = items[i];
        u32 *dst = ws + ws_off[2 * i];
        switch (it.cls) {
#define GF2X_PHASE_EVAL(id, name, T, c, C) \
    case id: staged_eval_item<T>(it, a_base, b_base, dst, smem); break;
            GF2X_STAGED_LIST(GF2X_PHASE_EVAL)
#undef GF2X_PHASE_EVAL
            default: break;
        }
    }
}

// (2) products: item i runs its direct class; items with pad == 1 are point
// products whose operands and result live in the workspace (offsets in
// uint64 words from ws), the others read a_base / b_base and write c_base.
__global__ __launch_bounds__(NT) void k_phase_products(const DevItem *items, u32 count, uint64_t *c_base,
                                                       const uint64_t *a_base, const uint64_t *b_base, uint64_t *ws) {
    extern __shared__ u32 smem[];
    for (u32 i = blockIdx.x; i < count; i += gridDim.x) {
        const DevItem it = items[i];
        const bool in_ws = it.pad != 0;
        const uint64_t *a = (in_ws ? ws : a_base) + it.a_off;
        const uint64_t *b = (in_ws ? ws : b_base) + it.b_off;
        uint64_t *c = (in_ws ? ws : c_base) + it.c_off;
        switch (it.cls) {
#define GF2X_PHASE_PRODUCT(id, T) \
    case id: one_product<T>(a, b, c, it.n, it.kind, smem); break;
            GF2X_PHASE_LIST(GF2X_PHASE_PRODUCT)
#undef GF2X_PHASE_PRODUCT
            default: break;
        }
    }
}

// (3) interpolation: staged item i reads its point products at
// ws + ws_off[2 i + 1] (32-bit words) and writes its result at c_base.
__global__ __launch_bounds__(NT) void k_phase_interp(const DevItem *items, const uint64_t *ws_off, u32 count,
                                                     uint64_t *c_base, const u32 *ws) {
    extern __shared__ u32 smem[];
    for (u32 i = blockIdx.x; i < count; i += gridDim.x) {
        const DevItem it = items[i];
        const u32 *src = ws + ws_off[2 * i + 1];
        switch (it.cls) {
#define GF2X_PHASE_INTERP(id, name, T, c, C) \
    case id: staged_interp_item<T>(it, c_base, src, smem); break;
            GF2X_STAGED_LIST(GF2X_PHASE_INTERP)
#undef GF2X_PHASE_INTERP
            default: break;
        }
    }
}

bool phase_product_class(int cls) {
    switch (cls) {
#define GF2X_PHASE_IS(id, T) case id:
        GF2X_PHASE_LIST(GF2X_PHASE_IS)
#undef GF2X_PHASE_IS
        return true;
        default: return false;
    }
}

// Largest LDS the three kernels may be launched with.
static int max_eval_lds() {
    int m = 0;
#define GF2X_EVAL_LDS(id, name, T, c, C) m = std::max(m, 2 * T::S * 4);
    GF2X_STAGED_LIST(GF2X_EVAL_LDS)
#undef GF2X_EVAL_LDS
    return m;
}
static int max_interp_lds() {
    int m = 0;
#define GF2X_INTERP_LDS(id, name, T, c, C) m = std::max(m, T::INTERP_SCRATCH * 4);
    GF2X_STAGED_LIST(GF2X_INTERP_LDS)
#undef GF2X_INTERP_LDS
    return m;
}
static int max_product_lds() {
    int m = 0;
#define GF2X_PRODUCT_LDS(id, T) m = std::max(m, lds_words<T>() * 4);
    GF2X_PHASE_LIST(GF2X_PRODUCT_LDS)
#undef GF2X_PRODUCT_LDS
    return m;
}

int phase_eval_lds(int cls) {
    switch (cls) {
#define GF2X_EVAL_LDS_OF(id, name, T, c, C) \
    case id: return 2 * T::S * 4;
        GF2X_STAGED_LIST(GF2X_EVAL_LDS_OF)
#undef GF2X_EVAL_LDS_OF
        default: return 0;
    }
}

int phase_interp_lds(int cls) {
    switch (cls) {
#define GF2X_INTERP_LDS_OF(id, name, T, c, C) \
    case id: return T::INTERP_SCRATCH * 4;
        GF2X_STAGED_LIST(GF2X_INTERP_LDS_OF)
#undef GF2X_INTERP_LDS_OF
        default: return 0;
    }
}

hipError_t prepare_phase_kernels() {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(&k_phase_eval),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, max_eval_lds());
    if (e == hipSuccess)
        e = hipFuncSetAttribute(reinterpret_cast<const void *>(&k_phase_products),
                                hipFuncAttributeMaxDynamicSharedMemorySize, max_product_lds());
    if (e == hipSuccess)
        e = hipFuncSetAttribute(reinterpret_cast<const void *>(&k_phase_interp),
                                hipFuncAttributeMaxDynamicSharedMemorySize, max_interp_lds());
    return e;
}

static uint32_t phase_grid(const void *fn, int lds, uint32_t count, int num_cu) {
    const long long cap = (long long)num_cu * occupancy(fn, lds);
    return (uint32_t)std::min<long long>(count, cap);
}

hipError_t launch_phase_eval(const DevItem *items, const uint64_t *ws_off, uint32_t count, int lds,
                             const uint64_t *a_base, const uint64_t *b_base, uint32_t *ws, int num_cu,
                             hipStream_t s) {
    if (count == 0) return hipSuccess;
    const uint32_t grid = phase_grid(reinterpret_cast<const void *>(&k_phase_eval), lds, count, num_cu);
    hipLaunchKernelGGL(k_phase_eval, dim3(grid), dim3(NT), lds, s, items, ws_off, count, a_base, b_base, ws);
    return hipGetLastError();
}

hipError_t launch_phase_products(const DevItem *items, uint32_t count, int lds, uint64_t *c_base,
                                 const uint64_t *a_base, const uint64_t *b_base, uint64_t *ws, int num_cu,
                                 hipStream_t s) {
    if (count == 0) return hipSuccess;
    const uint32_t grid = phase_grid(reinterpret_cast<const void *>(&k_phase_products), lds, count, num_cu);
    hipLaunchKernelGGL(k_phase_products, dim3(grid), dim3(NT), lds, s, items, count, c_base, a_base, b_base, ws);
    return hipGetLastError();
}

hipError_t launch_phase_interp(const DevItem *items, const uint64_t *ws_off, uint32_t count, int lds,
                               uint64_t *c_base, const uint32_t *ws, int num_cu, hipStream_t s) {
    if (count == 0) return hipSuccess;
    const uint32_t grid = phase_grid(reinterpret_cast<const void *>(&k_phase_interp), lds, count, num_cu);
    hipLaunchKernelGGL(k_phase_interp, dim3(grid), dim3(NT), lds, s, items, ws_off, count, c_base, ws);
    return hipGetLastError();
}

}  // namespace gf2x
