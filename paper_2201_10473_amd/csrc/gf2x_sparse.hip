// gf2x_sparse.hip -- dense x sparse ring products (gf2x_sparse_device.hpp):
// one wavefront per product, persistent workgroups of one wavefront over the
// items of one sparse size class.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <map>
#include <mutex>

#include "gf2x_internal.hpp"
#include "gf2x_sparse_device.hpp"

namespace gf2x {

// Items of kind GF2X_KIND_SPARSE: a (W(n) words) at a_base + a_off, the
// weight w = kind >> 8 positions (uint32) at b_base + b_off, the ring
// product at c_base + c_off.  NW waves per product (workgroups of NW waves).
template <int R, int NW>
__global__ __launch_bounds__(sparse::WAVE * NW) void k_sparse(const DevItem *items, uint32_t count, uint64_t *c_base,
                                                              const uint64_t *a_base, const uint64_t *b_base) {
    extern __shared__ uint32_t buf[];
    for (uint32_t i = blockIdx.x; i < count; i += gridDim.x) {
        const DevItem it = items[i];
        const uint32_t *pos = reinterpret_cast<const uint32_t *>(b_base + it.b_off);
        sparse::product<R, NW>(a_base + it.a_off, pos, it.kind >> 8, c_base + it.c_off, it.n, buf);
    }
}

namespace {

// Waves per product of the second kernel of each class (for batches that
// would fill the device with one wave per product only up to a fraction).
constexpr int kMultiWave = 4;

#define GF2X_SPARSE_FN(idx, R) reinterpret_cast<const void *>(&k_sparse<R, 1>),
const void *const kSparseFn[] = {GF2X_SPARSE_LIST(GF2X_SPARSE_FN)};
#define GF2X_SPARSE_FN_MW(idx, R) reinterpret_cast<const void *>(&k_sparse<R, kMultiWave>),
const void *const kSparseFnMw[] = {GF2X_SPARSE_LIST(GF2X_SPARSE_FN_MW)};
#define GF2X_SPARSE_R(idx, R) R,
const int kSparseR[] = {GF2X_SPARSE_LIST(GF2X_SPARSE_R)};

int sparse_occupancy(int idx, int nw) {
    static std::mutex mu;
    static std::map<std::pair<int, int>, int> cache;
    std::lock_guard<std::mutex> lk(mu);
    auto it = cache.find({idx, nw});
    if (it != cache.end()) return it->second;
    const void *fn = nw == 1 ? kSparseFn[idx] : kSparseFnMw[idx];
    int blocks = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, fn, sparse::WAVE * nw, 256 * kSparseR[idx]) !=
            hipSuccess ||
        blocks < 1)
        blocks = 1;
    cache[{idx, nw}] = blocks;
    return blocks;
}

}  // namespace

int sparse_class_for(uint32_t n) {
    if (n == 0 || n > sparse::kSparseMaxBits) return -1;
    const int need = sparse::words_per_lane_needed(n);
    for (int i = 0; i < sparse::kSparseClasses; ++i)
        if (kSparseR[i] >= need) return i;
    return -1;
}

int sparse_words_per_lane(int idx) { return kSparseR[idx]; }

hipError_t prepare_sparse_kernels() {
    for (int i = 0; i < sparse::kSparseClasses; ++i) {
        hipError_t e =
            hipFuncSetAttribute(kSparseFn[i], hipFuncAttributeMaxDynamicSharedMemorySize, 256 * kSparseR[i]);
        if (e == hipSuccess)
            e = hipFuncSetAttribute(kSparseFnMw[i], hipFuncAttributeMaxDynamicSharedMemorySize, 256 * kSparseR[i]);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t launch_sparse(int idx, const DevItem *items, uint32_t count, uint64_t *c_base, const uint64_t *a_base,
                         const uint64_t *b_base, int num_cu, hipStream_t s) {
    if (idx < 0 || idx >= sparse::kSparseClasses) return hipErrorInvalidValue;
    // one wave per product when the batch fills the device that way; else
    // several waves share each product's positions
    const long long waves1 = (long long)num_cu * sparse_occupancy(idx, 1);
    const int nw = 2LL * kMultiWave * count <= 3 * waves1 ? kMultiWave : 1;
    const long long cap = (long long)num_cu * sparse_occupancy(idx, nw);
    const uint32_t grid = (uint32_t)(count < cap ? count : cap);
    typedef void (*Fn)(const DevItem *, uint32_t, uint64_t *, const uint64_t *, const uint64_t *);
    Fn fn = reinterpret_cast<Fn>(const_cast<void *>(nw == 1 ? kSparseFn[idx] : kSparseFnMw[idx]));
    hipLaunchKernelGGL(fn, dim3(grid), dim3(sparse::WAVE * nw), 256 * kSparseR[idx], s, items, count, c_base, a_base,
                       b_base);
    return hipGetLastError();
}

}  // namespace gf2x
