// gf2x_kernels.hip -- kernels of the bit-packed path and their launchers.
// The per-product work and the size classes live in gf2x_product.hpp.
#include <hip/hip_runtime.h>
#include <stdint.h>

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
    {id, name, T::S, lds_words<T>() * 4, T::BASE, T::OPS},
static const ClassInfo kClassInfo[] = {GF2X_CLASS_LIST(GF2X_INFO)};

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

hipError_t prepare_kernels() {
    for (int c = 0; c < kNumClasses; ++c) {
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
