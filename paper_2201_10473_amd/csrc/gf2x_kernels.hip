// gf2x_kernels.hip -- host side of the bit-packed path: the size-class table,
// the launchers, and the small helper kernels.  The per-product kernels are
// instantiated in gf2x_kern_d<G>.hip (direct classes and the mixed-class
// kernels) and gf2x_kern_staged.hip; the per-product work lives in
// gf2x_product.hpp.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <map>
#include <mutex>

#include "gf2x_launch.hpp"
#include "gf2x_product.hpp"

namespace gf2x {

// Descriptors of the np * count point products: full products of S1-word
// operands (n = 32 S1 bits), operands [a | b] at (np i + e) * S1 uint64 words
// of ws_in, results at (np i + e) * S1 words of ws_out.
__global__ void k_child_items(u32 count, u32 S1, u32 np, u32 child_cls, DevItem *out) {
    const u32 j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j < np * count) {
        const uint64_t base = (uint64_t)j * S1;
        out[j] = DevItem{32u * S1, kKindFull, child_cls, 0u, base, base + S1 / 2, base};
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

// ------------------------------------------------- allocation-free scratch
// Device memory of gf2x_mul_batched_noalloc: the descriptors of one call
// (first kScratchItemBytes) and the workspace of its staged groups (the
// rest).  Every device the library runs on holds its own copy, loaded with
// the code object, until the process ends.  Host code never passes this name
// to a kernel: it uses the per-device address from scratch_for_device.
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

hipError_t scratch_for_device(int device, void **ptr) {
    static std::mutex mu;
    static std::map<int, void *> addr;
    std::lock_guard<std::mutex> lk(mu);
    auto it = addr.find(device);
    if (it != addr.end()) {
        *ptr = it->second;
        return hipSuccess;
    }
    // with `device` current: the address of this device's copy of the array
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    addr[device] = p;
    *ptr = p;
    return hipSuccess;
}

// ------------------------------------------------------------ host side
#define GF2X_INFO(id, name, T) \
    {id, name, T::S, lds_words<T>() * 4, T::BASE, T::OPS, -1, id, 0},
#define GF2X_STAGED_INFO(id, name, T, c, C)                                                             \
    {id, name, T::S, (lds_words<C>() > T::INTERP_SCRATCH ? lds_words<C>() : T::INTERP_SCRATCH) * 4, T::BASE, \
     T::OPS, c, -2, T::NP},
static ClassInfo kClassInfo[] = {GF2X_CLASS_LIST(GF2X_INFO) GF2X_STAGED_LIST(GF2X_STAGED_INFO)};

// The direct class of a staged class is one with the same top schedule (the
// one with the least LDS when a from-memory form exists); a top level without
// such a class takes the cheapest direct class that holds its size.
static int find_direct(int id) {
    const ClassInfo &ci = kClassInfo[id];
    if (ci.direct != -2) return ci.direct;
    int same = -1;
    for (int c = 0; c < kNumDirect; ++c)
        if (kClassInfo[c].S == ci.S && kClassInfo[c].ops == ci.ops &&
            (same < 0 || kClassInfo[c].lds_bytes < kClassInfo[same].lds_bytes))
            same = c;
    if (same >= 0) return same;
    int best = -1;
    for (int c = 0; c < kNumDirect; ++c)
        if (kClassInfo[c].S >= ci.S && (best < 0 || kClassInfo[c].ops < kClassInfo[best].ops)) best = c;
    return best;
}
static bool init_direct() {
    for (int c = 0; c < kNumClasses; ++c) kClassInfo[c].direct = find_direct(c);
    return true;
}
static const bool kDirectReady = init_direct();

// The sparse size classes as class-table rows: S is the largest ceil(n/32)
// the class holds, lds_bytes one wavefront's buffer; ops and base are not
// modelled here (the product is not a Karatsuba schedule).
static ClassInfo kSparseInfo[8];
static bool init_sparse_info() {
    static const char *names[8] = {"SP.R8", "SP.R13", "SP.R18", "SP.R25", "SP.R36", "SP.R41", "SP.R57", "SP.R64"};
    for (int i = 0; i < 8; ++i) {
        const int R = sparse_words_per_lane(i);
        kSparseInfo[i] = ClassInfo{kSparseBase + i, names[i], (64 * R - 2) / 2, 256 * R, 0, 0, -1,
                                   kSparseBase + i, 0};
    }
    return true;
}
static const bool kSparseInfoReady = init_sparse_info();

static const ClassInfo kFusedInfo{kFusedCls, "FUSED", 0, 0, 0, 0, -1, kFusedCls, 0};

const ClassInfo &class_info(int cls) {
    if (cls == kFusedCls) return kFusedInfo;
    return is_sparse_class(cls) ? kSparseInfo[cls - kSparseBase] : kClassInfo[cls];
}

typedef void (*SingleFn)(const uint64_t *, const uint64_t *, uint64_t *, u32, u32);
typedef void (*BatchedFn)(const DevItem *, u32, uint64_t *, const uint64_t *, const uint64_t *);

static const void *kSingle[kNumDirect];
static const void *kBatched[kNumDirect];
static const void *kMixed[kDirectGroups];
static int kMixedLds[kDirectGroups];  // largest LDS of the classes of each group
static bool collect_handles() {
    kMixed[0] = direct_kernels_0(kSingle, kBatched);
    kMixed[1] = direct_kernels_1(kSingle, kBatched);
    kMixed[2] = direct_kernels_2(kSingle, kBatched);
    kMixed[3] = direct_kernels_3(kSingle, kBatched);
    for (int c = 0; c < kNumDirect; ++c)
        kMixedLds[c % kDirectGroups] = std::max(kMixedLds[c % kDirectGroups], kClassInfo[c].lds_bytes);
    return true;
}
static const bool kHandlesReady = collect_handles();

static hipError_t set_lds_limit(const void *fn, int bytes) {
    return hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
}

hipError_t prepare_kernels() {
    (void)kDirectReady;
    (void)kHandlesReady;
    (void)kSparseInfoReady;
    hipError_t e = prepare_staged_kernels();
    if (e != hipSuccess) return e;
    e = prepare_sparse_kernels();
    if (e != hipSuccess) return e;
    e = prepare_fused_kernel();
    if (e != hipSuccess) return e;
    e = prepare_phase_kernels();
    if (e != hipSuccess) return e;
    for (int c = 0; c < kNumDirect; ++c) {
        e = set_lds_limit(kSingle[c], kClassInfo[c].lds_bytes);
        if (e != hipSuccess) return e;
        e = set_lds_limit(kBatched[c], kClassInfo[c].lds_bytes);
        if (e != hipSuccess) return e;
    }
    for (int g = 0; g < kDirectGroups; ++g) {
        e = set_lds_limit(kMixed[g], kMixedLds[g]);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t launch_single(int cls, const uint64_t *a, const uint64_t *b, uint64_t *c, uint32_t n, uint32_t kind,
                         hipStream_t s) {
    SingleFn fn = reinterpret_cast<SingleFn>(const_cast<void *>(kSingle[cls]));
    hipLaunchKernelGGL(fn, dim3(1), dim3(NT), kClassInfo[cls].lds_bytes, s, a, b, c, n, kind);
    return hipGetLastError();
}

// Resident workgroups per CU of a kernel at a given dynamic LDS size (cached:
// the runtime query is not free and the answer never changes).
int occupancy(const void *fn, int lds_bytes) {
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
    if (is_sparse_class(cls)) return launch_sparse(cls - kSparseBase, items, count, c_base, a_base, b_base, num_cu, s);
    const void *fnp = kBatched[cls];
    const int lds = kClassInfo[cls].lds_bytes;
    const long long cap = (long long)num_cu * occupancy(fnp, lds);
    const uint32_t grid = (uint32_t)(count < cap ? count : cap);
    BatchedFn fn = reinterpret_cast<BatchedFn>(const_cast<void *>(fnp));
    hipLaunchKernelGGL(fn, dim3(grid), dim3(NT), lds, s, items, count, c_base, a_base, b_base);
    return hipGetLastError();
}

size_t staged_workspace_bytes(int cls, uint32_t count) {
    const ClassInfo &ci = class_info(cls);
    if (ci.child < 0) return 0;
    const size_t S1 = (size_t)kClassInfo[ci.child].S;
    const size_t np = (size_t)ci.points;
    const size_t in = (size_t)count * 2 * np * S1 * 4, items = (size_t)count * np * sizeof(DevItem);
    return 2 * ((in + 255) / 256 * 256) + items;
}

hipError_t launch_child_items(uint32_t count, uint32_t S1, uint32_t np, uint32_t child_cls, DevItem *out,
                              hipStream_t s) {
    hipLaunchKernelGGL(k_child_items, dim3((np * count + 255) / 256), dim3(256), 0, s, count, S1, np, child_cls,
                       out);
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

// One launch per class group, in order on stream s; each skips the items of
// the other groups.
hipError_t launch_mixed(const DevItem *items, uint32_t count, uint64_t *c_base, const uint64_t *a_base,
                        const uint64_t *b_base, const uint8_t *cls_of_w32, uint32_t *bad, int num_cu, hipStream_t s) {
    typedef void (*MixedFn)(const DevItem *, u32, uint64_t *, const uint64_t *, const uint64_t *, const uint8_t *,
                            u32 *);
    for (int g = 0; g < kDirectGroups; ++g) {
        const long long cap = (long long)num_cu * occupancy(kMixed[g], kMixedLds[g]);
        const uint32_t grid = (uint32_t)(count < cap ? count : cap);
        MixedFn fn = reinterpret_cast<MixedFn>(const_cast<void *>(kMixed[g]));
        hipLaunchKernelGGL(fn, dim3(grid), dim3(NT), kMixedLds[g], s, items, count, c_base, a_base, b_base,
                           cls_of_w32, bad);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace gf2x
