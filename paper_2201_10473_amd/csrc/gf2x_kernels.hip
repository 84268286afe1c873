// gf2x_kernels.hip -- kernels of the bit-packed path and their launchers.
// The per-product work and the size classes live in gf2x_product.hpp.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <map>
#include <mutex>

#include "gf2x_product.hpp"

namespace gf2x {

template <class Sch>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(waves_per_simd<Sch>()))) void k_single(const uint64_t *a, const uint64_t *b, uint64_t *c, u32 n,
                                               u32 kind) {
    extern __shared__ u32 smem[];
    one_product<Sch>(a, b, c, n, kind, smem);
}

// Persistent workgroups over a batch whose items all use class Sch.
template <class Sch>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(waves_per_simd<Sch>()))) void k_batched(const DevItem *items, u32 count, uint64_t *c_base,
                                                const uint64_t *a_base, const uint64_t *b_base) {
    extern __shared__ u32 smem[];
    for (u32 i = blockIdx.x; i < count; i += gridDim.x) {
        const DevItem it = items[i];
        one_product<Sch>(a_base + it.a_off, b_base + it.b_off, c_base + it.c_off, it.n, it.kind, smem);
    }
}

// Persistent workgroups over a batch of mixed classes; the class of each item
// comes from its descriptor (host items) or from the per-size table.
__global__ __launch_bounds__(NT) void k_mixed(const DevItem *items, u32 count, uint64_t *c_base,
                                              const uint64_t *a_base, const uint64_t *b_base,
                                              const uint8_t *cls_of_w32, u32 use_table) {
    extern __shared__ u32 smem[];
    for (u32 i = blockIdx.x; i < count; i += gridDim.x) {
        const DevItem it = items[i];
        if (it.n == 0 || it.n > kMaxBits || it.kind > kKindFull) continue;  // invalid device descriptor
        const u32 cls = use_table ? (u32)cls_of_w32[(it.n + 31u) / 32u] : it.cls;
        const uint64_t *a = a_base + it.a_off;
        const uint64_t *b = b_base + it.b_off;
        uint64_t *c = c_base + it.c_off;
        switch (cls) {
#define GF2X_CASE(id, name, T) \
    case id: one_product<T>(a, b, c, it.n, it.kind, smem); break;
            GF2X_CLASS_LIST(GF2X_CASE)
            default: break;
        }
    }
}

// ----------------------------------------------------------- staged Toom-3
// Point operands of every item: word w of operand x of point e of item i goes
// to ws_in[((5 i + e) * 2 + x) * S1 + w].  The parent's words are read from
// HBM (masked to n bits, zero beyond), split in three parts of m words.
template <class Top>
__global__ __launch_bounds__(256) void k_t3_eval(const DevItem *items, u32 count, const uint64_t *a_base,
                                                 const uint64_t *b_base, u32 *ws_in) {
    const size_t total = (size_t)count * 10 * Top::S1;
    for (size_t idx = blockIdx.x * (size_t)blockDim.x + threadIdx.x; idx < total;
         idx += (size_t)gridDim.x * blockDim.x)
        ws_in[idx] = t3_eval_word<Top>(items, a_base, b_base, idx);
}

// Descriptors of the 5 * count point products: full products of S1-word
// operands (n = 32 S1 bits), operands [a | b] at (5 i + e) * S1 uint64 words
// of ws_in, results at (5 i + e) * S1 words of ws_out.
__global__ void k_child_items(u32 count, u32 S1, u32 child_cls, DevItem *out) {
    const u32 j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j < 5 * count) {
        const uint64_t base = (uint64_t)j * S1;
        out[j] = DevItem{32u * S1, kKindFull, child_cls, 0u, base, base + S1 / 2, base};
    }
}

// Interpolation of the five point products of each item, then the ring fold
// or the full store (persistent workgroups).
template <class Top>
__global__ __launch_bounds__(NT) void k_t3_interp(const DevItem *items, u32 count, uint64_t *c_base,
                                                  const u32 *ws_out) {
    extern __shared__ u32 smem[];
    for (u32 i = blockIdx.x; i < count; i += gridDim.x) t3_interp_item<Top>(items[i], c_base, ws_out + (size_t)i * 10 * Top::S1, smem);
}

// Device descriptors (public layout) -> internal layout; the class is taken
// from the size table inside k_mixed.
__global__ void k_convert_items(const gf2x_item *items, u32 count, DevItem *out) {
    const u32 i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) {
        const gf2x_item it = items[i];
        out[i] = DevItem{it.n_bits, it.kind, 0u, 0u, it.a_off, it.b_off, it.c_off};
    }
}

// Pseudo-random words for timing runs (SplitMix64 finaliser of seed + index).
__global__ void k_fill_words(uint64_t *dst, size_t count, uint64_t seed) {
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < count; i += (size_t)gridDim.x * blockDim.x) {
        uint64_t z = seed + (i + 1) * 0x9E3779B97F4A7C15ull;
        z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
        z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
        dst[i] = z ^ (z >> 31);
    }
}

// ------------------------------------------------------------ host side
#define GF2X_INFO(id, name, T) \
    {id, name, T::S, lds_words<T>() * 4, T::BASE, T::OPS, -1, id},
#define GF2X_STAGED_INFO(id, name, T, c, C)                                                             \
    {id, name, T::S, (lds_words<C>() > T::INTERP_SCRATCH ? lds_words<C>() : T::INTERP_SCRATCH) * 4, T::BASE, \
     T::OPS, c, -2},
static ClassInfo kClassInfo[] = {GF2X_CLASS_LIST(GF2X_INFO) GF2X_STAGED_LIST(GF2X_STAGED_INFO)};

// the direct class of each staged class is the one with the same top schedule
static int find_direct(int id) {
    const ClassInfo &ci = kClassInfo[id];
    if (ci.direct != -2) return ci.direct;
    for (int c = 0; c < kNumDirect; ++c)
        if (kClassInfo[c].S == ci.S && kClassInfo[c].ops == ci.ops) return c;
    return -1;
}
static bool init_direct() {
    for (int c = 0; c < kNumClasses; ++c) kClassInfo[c].direct = find_direct(c);
    return true;
}
static const bool kDirectReady = init_direct();

const ClassInfo &class_info(int cls) { return kClassInfo[cls]; }

typedef void (*SingleFn)(const uint64_t *, const uint64_t *, uint64_t *, u32, u32);
typedef void (*BatchedFn)(const DevItem *, u32, uint64_t *, const uint64_t *, const uint64_t *);

#define GF2X_SINGLE_PTR(id, name, T) reinterpret_cast<const void *>(&k_single<T>),
#define GF2X_BATCHED_PTR(id, name, T) reinterpret_cast<const void *>(&k_batched<T>),
static const void *kSingle[] = {GF2X_CLASS_LIST(GF2X_SINGLE_PTR)};
static const void *kBatched[] = {GF2X_CLASS_LIST(GF2X_BATCHED_PTR)};

static hipError_t set_lds_limit(const void *fn, int bytes) {
    return hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
}

#define GF2X_INTERP_PTR(id, name, T, c, C) reinterpret_cast<const void *>(&k_t3_interp<T>),
static const void *kInterp[] = {GF2X_STAGED_LIST(GF2X_INTERP_PTR)};

hipError_t prepare_kernels() {
    (void)kDirectReady;
#define GF2X_INTERP_ATTR(id, name, T, c, C)                                                               \
    {                                                                                                     \
        hipError_t e = set_lds_limit(reinterpret_cast<const void *>(&k_t3_interp<T>), T::INTERP_SCRATCH * 4); \
        if (e != hipSuccess) return e;                                                                    \
    }
    GF2X_STAGED_LIST(GF2X_INTERP_ATTR)
    (void)kInterp;
    for (int c = 0; c < kNumDirect; ++c) {
        hipError_t e = set_lds_limit(kSingle[c], kClassInfo[c].lds_bytes);
        if (e != hipSuccess) return e;
        e = set_lds_limit(kBatched[c], kClassInfo[c].lds_bytes);
        if (e != hipSuccess) return e;
    }
    return set_lds_limit(reinterpret_cast<const void *>(&k_mixed), 160 * 1024);
}

hipError_t launch_single(int cls, const uint64_t *a, const uint64_t *b, uint64_t *c, uint32_t n, uint32_t kind,
                         hipStream_t s) {
    SingleFn fn = reinterpret_cast<SingleFn>(const_cast<void *>(kSingle[cls]));
    hipLaunchKernelGGL(fn, dim3(1), dim3(NT), kClassInfo[cls].lds_bytes, s, a, b, c, n, kind);
    return hipGetLastError();
}

// Resident workgroups per CU of a kernel at a given dynamic LDS size (cached:
// the runtime query is not free and the answer never changes).
static int occupancy(const void *fn, int lds_bytes) {
    static std::mutex mu;
    static std::map<std::pair<const void *, int>, int> cache;
    std::lock_guard<std::mutex> lk(mu);
    auto it = cache.find({fn, lds_bytes});
    if (it != cache.end()) return it->second;
    int blocks = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, fn, NT, lds_bytes) != hipSuccess || blocks < 1)
        blocks = 1;
    cache[{fn, lds_bytes}] = blocks;
    return blocks;
}

hipError_t launch_batched(int cls, const DevItem *items, uint32_t count, uint64_t *c_base, const uint64_t *a_base,
                          const uint64_t *b_base, int num_cu, hipStream_t s) {
    const void *fnp = kBatched[cls];
    const int lds = kClassInfo[cls].lds_bytes;
    const long long cap = (long long)num_cu * occupancy(fnp, lds);
    const uint32_t grid = (uint32_t)(count < cap ? count : cap);
    BatchedFn fn = reinterpret_cast<BatchedFn>(const_cast<void *>(fnp));
    hipLaunchKernelGGL(fn, dim3(grid), dim3(NT), lds, s, items, count, c_base, a_base, b_base);
    return hipGetLastError();
}

size_t staged_workspace_bytes(int cls, uint32_t count) {
    const ClassInfo &ci = kClassInfo[cls];
    if (ci.child < 0) return 0;
    const size_t S1 = (size_t)kClassInfo[ci.child].S;
    const size_t in = (size_t)count * 10 * S1 * 4, items = (size_t)count * 5 * sizeof(DevItem);
    return 2 * ((in + 255) / 256 * 256) + items;
}

template <class T, int CHILD>
static hipError_t staged_impl(const DevItem *items, uint32_t count, uint64_t *c_base, const uint64_t *a_base,
                              const uint64_t *b_base, void *ws, int num_cu, hipStream_t s) {
    constexpr int S1 = T::S1;
    const size_t in_bytes = ((size_t)count * 10 * S1 * 4 + 255) / 256 * 256;
    u32 *ws_in = reinterpret_cast<u32 *>(ws);
    u32 *ws_out = reinterpret_cast<u32 *>(reinterpret_cast<char *>(ws) + in_bytes);
    DevItem *child = reinterpret_cast<DevItem *>(reinterpret_cast<char *>(ws) + 2 * in_bytes);
    const size_t total = (size_t)count * 10 * S1;
    const uint32_t eval_grid = (uint32_t)std::min<size_t>((total + 255) / 256, (size_t)num_cu * 16);
    hipLaunchKernelGGL(k_t3_eval<T>, dim3(eval_grid), dim3(256), 0, s, items, count, a_base, b_base, ws_in);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_child_items, dim3((5 * count + 255) / 256), dim3(256), 0, s, count, (u32)S1, (u32)CHILD,
                       child);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    e = launch_batched(CHILD, child, 5 * count, reinterpret_cast<uint64_t *>(ws_out),
                       reinterpret_cast<const uint64_t *>(ws_in), reinterpret_cast<const uint64_t *>(ws_in), num_cu,
                       s);
    if (e != hipSuccess) return e;
    const void *fn = reinterpret_cast<const void *>(&k_t3_interp<T>);
    const int lds = T::INTERP_SCRATCH * 4;
    const long long cap = (long long)num_cu * occupancy(fn, lds);
    const uint32_t grid = (uint32_t)(count < cap ? count : cap);
    hipLaunchKernelGGL(k_t3_interp<T>, dim3(grid), dim3(NT), lds, s, items, count, c_base, ws_out);
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

hipError_t launch_fill_words(uint64_t *dst, size_t count, uint64_t seed, hipStream_t s) {
    hipLaunchKernelGGL(k_fill_words, dim3(1024), dim3(256), 0, s, dst, count, seed);
    return hipGetLastError();
}

hipError_t launch_convert_items(const gf2x_item *items, uint32_t count, DevItem *out, hipStream_t s) {
    hipLaunchKernelGGL(k_convert_items, dim3((count + 255) / 256), dim3(256), 0, s, items, count, out);
    return hipGetLastError();
}

hipError_t launch_mixed(const DevItem *items, uint32_t count, uint64_t *c_base, const uint64_t *a_base,
                        const uint64_t *b_base, const uint8_t *cls_of_w32, bool use_table, int lds_bytes,
                        int num_cu, hipStream_t s) {
    const void *fnp = reinterpret_cast<const void *>(&k_mixed);
    const long long cap = (long long)num_cu * occupancy(fnp, lds_bytes);
    const uint32_t grid = (uint32_t)(count < cap ? count : cap);
    hipLaunchKernelGGL(k_mixed, dim3(grid), dim3(NT), lds_bytes, s, items, count, c_base, a_base, b_base,
                       cls_of_w32, use_table ? 1u : 0u);
    return hipGetLastError();
}

}  // namespace gf2x
