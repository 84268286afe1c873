// gf2x_kern_staged.hip -- staged classes: the top Toom-3 or Toom-4 level is
// spread over workgroups through HBM (evaluation kernel, one batched launch
// of the NP * count point products, interpolation kernel).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

#include "gf2x_launch.hpp"
#include "gf2x_product.hpp"

namespace gf2x {

// Point operands of every item: word w of operand x of point e of item i goes
// to ws_in[((NP i + e) * 2 + x) * S1 + w] (persistent workgroups, one item
// at a time).
template <class Top>
__global__ __launch_bounds__(NT) void k_stage_eval(const DevItem *items, u32 count, const uint64_t *a_base,
                                                   const uint64_t *b_base, u32 *ws_in) {
    extern __shared__ u32 smem[];
    for (u32 i = blockIdx.x; i < count; i += gridDim.x)
        staged_eval_item<Top>(items[i], a_base, b_base, ws_in + (size_t)i * 2 * Top::NP * Top::S1, smem);
}

// Interpolation of the NP point products of each item, then the ring fold
// or the full store (persistent workgroups).
// Waves per SIMD the interpolation kernel of Top must allow (a register
// budget for the compiler): Top::INTERP_WAVES where a Top declares it.
template <class T, class = void>
struct InterpWaves {
    static constexpr int value = 1;
};
template <class T>
struct InterpWaves<T, std::void_t<decltype(T::INTERP_WAVES)>> {
    static constexpr int value = T::INTERP_WAVES;
};

template <class Top>
__global__ __launch_bounds__(NT, InterpWaves<Top>::value) void k_stage_interp(const DevItem *items, u32 count, uint64_t *c_base,
                                                     const u32 *ws_out) {
    extern __shared__ u32 smem[];
    for (u32 i = blockIdx.x; i < count; i += gridDim.x)
        staged_interp_item<Top>(items[i], c_base, ws_out + (size_t)i * 2 * Top::NP * Top::S1, smem);
}

hipError_t prepare_staged_kernels() {
#define GF2X_INTERP_ATTR(id, name, T, c, C)                                                                    \
    {                                                                                                          \
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(&k_stage_interp<T>),                   \
                                           hipFuncAttributeMaxDynamicSharedMemorySize, T::INTERP_SCRATCH * 4); \
        if (e != hipSuccess) return e;                                                                         \
        e = hipFuncSetAttribute(reinterpret_cast<const void *>(&k_stage_eval<T>),                               \
                                hipFuncAttributeMaxDynamicSharedMemorySize, 2 * T::S * 4);                     \
        if (e != hipSuccess) return e;                                                                         \
    }
    GF2X_STAGED_LIST(GF2X_INTERP_ATTR)
    return hipSuccess;
}

template <class T, int CHILD>
static hipError_t staged_impl(const DevItem *items, uint32_t count, uint64_t *c_base, const uint64_t *a_base,
                              const uint64_t *b_base, void *ws, int num_cu, hipStream_t s) {
    constexpr int S1 = T::S1, NP = T::NP;
    // point operand b sits S1 / 2 uint64 words after a (k_child_items)
    static_assert(S1 % 2 == 0, "child operands start on a uint64 word");
    const size_t in_bytes = ((size_t)count * 2 * NP * S1 * 4 + 255) / 256 * 256;
    u32 *ws_in = reinterpret_cast<u32 *>(ws);
    u32 *ws_out = reinterpret_cast<u32 *>(reinterpret_cast<char *>(ws) + in_bytes);
    DevItem *child = reinterpret_cast<DevItem *>(reinterpret_cast<char *>(ws) + 2 * in_bytes);
    const void *efn = reinterpret_cast<const void *>(&k_stage_eval<T>);
    const int elds = 2 * T::S * 4;
    const long long ecap = (long long)num_cu * occupancy(efn, elds);
    const uint32_t eval_grid = (uint32_t)(count < ecap ? count : ecap);
    hipLaunchKernelGGL(k_stage_eval<T>, dim3(eval_grid), dim3(NT), elds, s, items, count, a_base, b_base, ws_in);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    e = launch_child_items(count, (u32)S1, (u32)NP, (u32)CHILD, child, s);
    if (e != hipSuccess) return e;
    e = launch_batched(CHILD, child, NP * count, reinterpret_cast<uint64_t *>(ws_out),
                       reinterpret_cast<const uint64_t *>(ws_in), reinterpret_cast<const uint64_t *>(ws_in), num_cu,
                       s);
    if (e != hipSuccess) return e;
    const void *fn = reinterpret_cast<const void *>(&k_stage_interp<T>);
    const int lds = T::INTERP_SCRATCH * 4;
    const long long cap = (long long)num_cu * occupancy(fn, lds);
    const uint32_t grid = (uint32_t)(count < cap ? count : cap);
    hipLaunchKernelGGL(k_stage_interp<T>, dim3(grid), dim3(NT), lds, s, items, count, c_base, ws_out);
    return hipGetLastError();
}

hipError_t launch_staged(int cls, const DevItem *items, uint32_t count, uint64_t *c_base, const uint64_t *a_base,
                         const uint64_t *b_base, void *ws, int num_cu, hipStream_t s) {
    switch (cls) {
#define GF2X_STAGED_CASE(id, name, T, c, C) \
    case id: return staged_impl<T, c>(items, count, c_base, a_base, b_base, ws, num_cu, s);
        GF2X_STAGED_LIST(GF2X_STAGED_CASE)
        default: return hipErrorInvalidValue;
    }
}

}  // namespace gf2x
