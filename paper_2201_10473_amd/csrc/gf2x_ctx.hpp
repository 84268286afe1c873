// gf2x_ctx.hpp -- the context object behind the opaque gf2x_ctx handle
// (shared by the C ABI layer and the serving loop).  Not part of the ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <map>
#include <vector>
#include <tuple>

#include "gf2x.h"
#include "gf2x_internal.hpp"
#include "gf2x_toeplitz.hpp"

namespace gf2x {

// A recorded launch sequence of one batch: its graph, the private copy of
// the descriptors and the private workspace of its staged groups.  `done`
// is recorded after every launch, so the entry can be released safely.
struct GraphEntry {
    hipGraphExec_t exec = nullptr;
    hipGraph_t graph = nullptr;
    DevItem *items = nullptr;  // private copy of the descriptors
    uint32_t *queue = nullptr; // work-queue counters of a fused launch (inside the items allocation)
    void *staged_ws = nullptr; // private workspace of the staged groups
    size_t bytes = 0;          // device bytes of items + staged_ws (counted in the budget)
    hipEvent_t done = nullptr;
    bool launched = false;
    uint64_t checksum = 0;
    uint64_t last_use = 0;
};

}  // namespace gf2x

// A batch recorded once by gf2x_plan_create and replayed by gf2x_plan_launch.
struct gf2x_plan {
    gf2x_ctx *ctx = nullptr;
    gf2x::GraphEntry g;
    // A batch of one size class is replayed by launching its kernels directly
    // (the graph adds dispatch latency and overlaps nothing); its class group:
    bool one_group = false;
    int cls = -1;
    uint32_t first = 0, count = 0;
    int lds = 0;
    uint64_t *c = nullptr;
    const uint64_t *a = nullptr, *b = nullptr;
};

struct gf2x_ctx {
    int device = 0;
    int num_cu = 0;
    void *scratch = nullptr;  // this device's copy of the allocation-free scratch array
    size_t budget = 0;
    size_t allocated = 0;
    int cls_of_w32[gf2x::kMaxWords32 + 1];     // batch schedule per size (direct or staged)
    int direct_of_w32[gf2x::kMaxWords32 + 1];  // best direct class per size (device-resident
                                               // items, serving)
    int single_of_w32[gf2x::kMaxWords32 + 1];  // lowest-latency class of one product (direct or
                                               // staged)
    uint8_t *d_cls = nullptr;                  // device copy of direct_of_w32
    gf2x::DevItem *d_items = nullptr;    // workspace for host item descriptors
    uint32_t *d_queue = nullptr;         // work-queue counters of fused launches (same guard)
    size_t d_items_cap = 0;
    hipEvent_t ws_free = nullptr;  // recorded after the last launch reading d_items / staged_ws
    void *staged_ws = nullptr;     // workspace of staged classes (point operands and products)
    size_t staged_ws_bytes = 0;
    void *inv_ws = nullptr;        // working buffers of gf2x_inv_cyclic_batched (same guard)
    size_t inv_ws_bytes = 0;
    bool ws_used = false;
    // GF2X_USE_GRAPH cache, keyed by (items, count, bases, flags, stream);
    // at most kMaxGraphs entries, the least recently used one is released
    // first.
    static constexpr size_t kMaxGraphs = 64;
    std::map<std::tuple<const void *, uint32_t, const void *, const void *, const void *, uint32_t, void *>,
             gf2x::GraphEntry>
        graphs;
    uint64_t graph_clock = 0;
    gf2x::toeplitz::Workspace tz;
    std::map<uint32_t, int> tuned;         // w32 -> class chosen by gf2x_tune or the cache file
    std::map<uint32_t, int> tuned_direct;  // w32 -> fastest direct class measured for that size
    std::map<uint32_t, int> tuned_single;  // w32 -> lowest single-product latency measured
    // w32 -> every candidate the tuner measured: (class, batch ms, single-product ms)
    std::map<uint32_t, std::vector<std::tuple<int, float, float>>> tune_log;
    // Device descriptors of single products run in a staged class, one per
    // (n, kind), written once and never overwritten (enqueued work may read
    // them); grown in chunks.
    std::map<std::pair<uint32_t, uint32_t>, gf2x::DevItem *> single_items;
    std::vector<gf2x::DevItem *> single_chunks;
    size_t single_used = 0;                // descriptors used in the last chunk
    // internal streams (default priority) for concurrent per-class launches,
    // forked from and joined back to the caller's stream with events
    static constexpr int kForks = 4;
    hipStream_t fork_stream[kForks] = {};
    hipEvent_t fork_event[kForks + 1] = {};
};
