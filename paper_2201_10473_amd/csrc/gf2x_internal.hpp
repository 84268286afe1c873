// gf2x_internal.hpp -- interface between the C ABI layer (gf2x_api.cpp) and
// the kernel translation units (gf2x_kernels.hip, gf2x_kern_*.hip).  Not part
// of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "gf2x.h"

namespace gf2x {

constexpr int kNumDirect = 41;   // classes computed inside one workgroup
constexpr int kNumClasses = 52;  // plus the staged classes
constexpr uint32_t kKindCyclic = 0;
constexpr uint32_t kKindFull = 1;
constexpr uint32_t kKindSparse = 2;  // low byte of the kind; the weight is kind >> 8
static_assert(kKindSparse == GF2X_KIND_SPARSE, "kind code as declared in gf2x.h");
// Size classes of dense x sparse products get the ids kSparseBase + index.
constexpr int kSparseBase = 64;
inline bool is_sparse_class(int cls) { return cls >= kSparseBase && cls < kSparseBase + 8; }
// The group id of a fused launch (every item in its direct class, one kernel).
constexpr int kFusedCls = 1000;
constexpr uint32_t kMaxBits = 131072;
constexpr uint32_t kMaxWords32 = kMaxBits / 32;

// Device-side descriptor of one batch item (offsets in uint64 words).
struct DevItem {
    uint32_t n;
    uint32_t kind;
    uint32_t cls;
    uint32_t pad;
    uint64_t a_off, b_off, c_off;
};

struct ClassInfo {
    int id;
    const char *name;
    int S;                   // padded operand size, 32-bit words
    int lds_bytes;           // LDS of one workgroup (largest kernel of a staged class)
    long long base;          // 32x32 word products per multiplication
    long long ops;           // algorithmic VALU lane-ops per multiplication
    int child;               // staged: class of the five point products; else -1
    int direct;              // class computing the same size inside one workgroup
    int points;              // staged: point products per item (5 or 7); else 0
};

// Scratch of the allocation-free batched entry point (a static device array
// per device): descriptors of up to kScratchMaxItems items, then the staged
// workspace.
constexpr size_t kScratchBytes = (size_t)32 << 20;
constexpr uint32_t kScratchMaxItems = 65536;
constexpr size_t kScratchItemBytes = (size_t)kScratchMaxItems * sizeof(DevItem);
static_assert(kScratchItemBytes % 256 == 0, "workspace region starts 256-byte aligned");
static_assert(kScratchBytes == GF2X_NOALLOC_SCRATCH_BYTES && kScratchMaxItems == GF2X_NOALLOC_MAX_ITEMS,
              "scratch limits as declared in gf2x.h");
// Address of the current device's copy of the scratch array (looked up once
// per device; call with that device current).
hipError_t scratch_for_device(int device, void **ptr);

const ClassInfo &class_info(int cls);

// Dense x sparse products (gf2x_sparse.hip): the sparse size class of n
// (index into the class list, -1 if n is too large), its words per lane,
// and the launcher of a batch of one class.
int sparse_class_for(uint32_t n);
int sparse_words_per_lane(int idx);
hipError_t prepare_sparse_kernels();

// One persistent launch over items of the fused class set (gf2x_kern_fused.hip):
// whether a direct class belongs to it, and the launcher; queue: two uint32
// counters, zero before the first launch (the kernel leaves them zero).
bool fused_class(int cls);

// A batch of mixed sizes in three launches (gf2x_kern_phase.hip): the
// evaluations of its staged items, all one-workgroup products (the staged
// items' point products, flagged by pad = 1 and addressed in the workspace,
// and the direct items), the interpolations.  ws_off holds two 32-bit-word
// offsets per staged item (its point operands, its point products).
bool phase_product_class(int cls);
int phase_eval_lds(int cls);
int phase_interp_lds(int cls);
hipError_t prepare_phase_kernels();
hipError_t launch_phase_eval(const DevItem *items, const uint64_t *ws_off, uint32_t count, int lds,
                             const uint64_t *a_base, const uint64_t *b_base, uint32_t *ws, int num_cu,
                             hipStream_t s);
hipError_t launch_phase_products(const DevItem *items, uint32_t count, int lds, uint64_t *c_base,
                                 const uint64_t *a_base, const uint64_t *b_base, uint64_t *ws, int num_cu,
                                 hipStream_t s);
hipError_t launch_phase_interp(const DevItem *items, const uint64_t *ws_off, uint32_t count, int lds,
                               uint64_t *c_base, const uint32_t *ws, int num_cu, hipStream_t s);
hipError_t prepare_fused_kernel();
hipError_t launch_fused(const DevItem *items, uint32_t count, int lds, uint64_t *c_base, const uint64_t *a_base,
                        const uint64_t *b_base, uint32_t *queue, int num_cu, hipStream_t s);
hipError_t launch_sparse(int idx, const DevItem *items, uint32_t count, uint64_t *c_base, const uint64_t *a_base,
                         const uint64_t *b_base, int num_cu, hipStream_t s);
hipError_t prepare_kernels();
// Staged classes need a device workspace: bytes for `count` products.
size_t staged_workspace_bytes(int cls, uint32_t count);
hipError_t launch_staged(int cls, const DevItem *items, uint32_t count, uint64_t *c_base, const uint64_t *a_base,
                         const uint64_t *b_base, void *ws, int num_cu, hipStream_t s);
hipError_t launch_single(int cls, const uint64_t *a, const uint64_t *b, uint64_t *c, uint32_t n, uint32_t kind,
                         hipStream_t s);
hipError_t launch_batched(int cls, const DevItem *items, uint32_t count, uint64_t *c_base, const uint64_t *a_base,
                          const uint64_t *b_base, int num_cu, hipStream_t s);
hipError_t launch_fill_words(uint64_t *dst, size_t count, uint64_t seed, hipStream_t s);
hipError_t launch_convert_items(const struct gf2x_item *items, uint32_t count, DevItem *out, hipStream_t s);
// Items whose classes come from the device table cls_of_w32 (direct classes).
// Invalid descriptors are skipped and counted in *bad (device memory).
hipError_t launch_mixed(const DevItem *items, uint32_t count, uint64_t *c_base, const uint64_t *a_base,
                        const uint64_t *b_base, const uint8_t *cls_of_w32, uint32_t *bad, int num_cu, hipStream_t s);

// Inversion helpers (gf2x_inv.hip): items of W(n) words.
// out item i = in item i (contiguous) squared j times, inv = 2^(-j) mod n;
// written at out_base + out_off[i] (device array) or contiguously if null.
hipError_t launch_frobenius(const uint64_t *in, uint64_t *out_base, const uint64_t *out_off, uint32_t n, uint32_t count,
                            uint32_t inv, hipStream_t s);
// out item i (contiguous) = in_base + in_off[i] (device array), bits >= n cleared.
hipError_t launch_gather_items(const uint64_t *in_base, const uint64_t *in_off, uint64_t *out, uint32_t n,
                               uint32_t count, hipStream_t s);

}  // namespace gf2x
