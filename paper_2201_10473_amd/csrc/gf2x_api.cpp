// gf2x_api.cpp -- the C ABI declared in include/gf2x.h: argument checks,
// per-size schedule table, workspace and graph cache, launches.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "gf2x.h"
#include "gf2x_internal.hpp"
#include "gf2x_ctx.hpp"
#include "gf2x_toeplitz.hpp"

using namespace gf2x;

namespace {

thread_local std::string g_last_device_error;

int device_error(hipError_t e) {
    g_last_device_error = hipGetErrorName(e);
    g_last_device_error += ": ";
    g_last_device_error += hipGetErrorString(e);
    return GF2X_EDEVICE;
}

#define HIP_TRY(expr)                              \
    do {                                           \
        hipError_t _e = (expr);                    \
        if (_e != hipSuccess) return device_error(_e); \
    } while (0)

uint64_t words64(uint32_t n) { return ((uint64_t)n + 63u) / 64u; }

// In the context's 256-byte counter block: words 0 and 1 are the fused
// launch's work queue, this word counts skipped device-resident descriptors.
constexpr int kBadCounter = 16;

}  // namespace


namespace {

// Default schedule choice: among the classes whose padded size holds w
// 32-bit words, the one with the fewest modelled lane-ops.
int default_class(uint32_t w) {
    int best = -1;
    long long best_ops = 0;
    for (int c = 0; c < kNumClasses; ++c) {
        const ClassInfo &ci = class_info(c);
        if ((uint32_t)ci.S < std::max<uint32_t>(w, 1)) continue;
        if (best < 0 || ci.ops < best_ops) {
            best = c;
            best_ops = ci.ops;
        }
    }
    return best;
}

void default_table(gf2x_ctx *ctx) {
    for (uint32_t w = 0; w <= kMaxWords32; ++w) ctx->cls_of_w32[w] = default_class(w);
}

// The direct class of each size: the one measured fastest by the tuner when
// the table has it, else the direct form of the batch schedule.  The class
// of a single product: the one with the lowest measured latency, else the
// direct class.
void direct_table(gf2x_ctx *ctx) {
    for (uint32_t w = 0; w <= kMaxWords32; ++w) {
        auto it = ctx->tuned_direct.find(w);
        ctx->direct_of_w32[w] = it != ctx->tuned_direct.end() ? it->second : class_info(ctx->cls_of_w32[w]).direct;
        auto is = ctx->tuned_single.find(w);
        ctx->single_of_w32[w] = is != ctx->tuned_single.end() ? is->second : ctx->direct_of_w32[w];
    }
}

int upload_direct_table(gf2x_ctx *ctx) {
    uint8_t tab[kMaxWords32 + 1];
    for (uint32_t w = 0; w <= kMaxWords32; ++w) tab[w] = (uint8_t)ctx->direct_of_w32[w];
    if (!ctx->d_cls) {
        HIP_TRY(hipMalloc(&ctx->d_cls, sizeof tab));
        ctx->allocated += sizeof tab;
    }
    HIP_TRY(hipMemcpy(ctx->d_cls, tab, sizeof tab, hipMemcpyHostToDevice));
    return GF2X_OK;
}

// Tuner cache: text lines "w32 batch_class [direct_class [single_class]]"
// override the default per size: the batch schedule, the fastest direct
// class, and the class with the lowest single-product latency.
int load_tune_cache(gf2x_ctx *ctx, const char *path) {
    FILE *f = std::fopen(path, "r");
    if (!f) return GF2X_OK;  // no cache yet: defaults
    char line[512];
    while (std::fgets(line, sizeof line, f)) {
        unsigned w = 0;
        char name[128], dname[128], sname[128];
        if (line[0] == '#') continue;
        const int got = std::sscanf(line, "%u %127s %127s %127s", &w, name, dname, sname);
        if (got < 2 || w == 0 || w > kMaxWords32) continue;
        for (int c = 0; c < kNumClasses; ++c) {
            if ((uint32_t)class_info(c).S < w) continue;
            if (std::strcmp(class_info(c).name, name) == 0) {
                ctx->cls_of_w32[w] = c;
                ctx->tuned[w] = c;
            }
            if (got >= 3 && c < kNumDirect && std::strcmp(class_info(c).name, dname) == 0) ctx->tuned_direct[w] = c;
            if (got >= 4 && std::strcmp(class_info(c).name, sname) == 0) ctx->tuned_single[w] = c;
        }
    }
    std::fclose(f);
    return GF2X_OK;
}

bool aligned8(const void *p) { return ((uintptr_t)p & 7u) == 0; }

bool overlap(const void *x, uint64_t xw, const void *y, uint64_t yw) {
    const uintptr_t a0 = (uintptr_t)x, a1 = a0 + xw * 8, b0 = (uintptr_t)y, b1 = b0 + yw * 8;
    return a0 < b1 && b0 < a1;
}

int check_single(gf2x_ctx *ctx, uint64_t *c, const uint64_t *a, const uint64_t *b, uint32_t n, uint64_t cw) {
    if (!ctx || !c || !a || !b) return GF2X_EINVAL;
    if (n == 0 || n > kMaxBits) return GF2X_EINVAL;
    if (!aligned8(c) || !aligned8(a) || !aligned8(b)) return GF2X_EINVAL;
    const uint64_t W = words64(n);
    if (overlap(c, cw, a, W) || overlap(c, cw, b, W)) return GF2X_EINVAL;
    return GF2X_OK;
}

// Host items of a batch: every output range is disjoint from every other
// output range and from every operand range (operands may be shared).
// Output spans are sorted by address (a pass when they already are), so an
// overlap shows between neighbours; an operand span is checked in O(1) when
// it lies outside the outputs' hull, else by binary search.  Offsets that
// would wrap the address space are refused.
int check_ranges(const gf2x_item *items, uint32_t count, const uint64_t *c_base, const uint64_t *a_base,
                 const uint64_t *b_base) {
    struct Span {
        uintptr_t lo, hi;
    };
    thread_local std::vector<Span> outs;
    outs.resize(count);
    auto span = [](const void *base, uint64_t off, uint64_t words, Span &sp) -> bool {
        const uintptr_t b = (uintptr_t)base, room = (UINTPTR_MAX - b) / 8;
        if (off > room || words > room - off) return false;
        sp.lo = b + off * 8;
        sp.hi = sp.lo + words * 8;
        return true;
    };
    bool sorted = true;
    for (uint32_t i = 0; i < count; ++i) {
        const gf2x_item &it = items[i];
        const uint64_t W = words64(it.n_bits);
        if (!span(c_base, it.c_off, it.kind == GF2X_KIND_FULL ? 2 * W : W, outs[i])) return GF2X_EINVAL;
        if (i && outs[i].lo < outs[i - 1].lo) sorted = false;
    }
    if (!sorted) std::sort(outs.begin(), outs.end(), [](const Span &x, const Span &y) { return x.lo < y.lo; });
    for (uint32_t i = 1; i < count; ++i)
        if (outs[i].lo < outs[i - 1].hi) return GF2X_EINVAL;
    const uintptr_t hull_lo = outs[0].lo, hull_hi = outs[count - 1].hi;
    auto clash = [&](const Span &sp) -> bool {
        if (sp.hi <= hull_lo || sp.lo >= hull_hi || sp.lo == sp.hi) return false;
        // first output span ending after sp.lo (ends increase with starts)
        auto k = std::upper_bound(outs.begin(), outs.end(), sp.lo,
                                  [](uintptr_t v, const Span &o) { return v < o.hi; });
        return k != outs.end() && k->lo < sp.hi;
    };
    for (uint32_t i = 0; i < count; ++i) {
        const gf2x_item &it = items[i];
        const uint64_t W = words64(it.n_bits);
        const bool sparse = (it.kind & 0xFFu) == GF2X_KIND_SPARSE;
        Span sa, sb;
        if (!span(a_base, it.a_off, W, sa) || !span(b_base, it.b_off, sparse ? ((it.kind >> 8) + 1) / 2 : W, sb))
            return GF2X_EINVAL;
        if (clash(sa) || clash(sb)) return GF2X_EINVAL;
    }
    return GF2X_OK;
}

int ensure_items(gf2x_ctx *ctx, size_t count) {
    if (count <= ctx->d_items_cap) return GF2X_OK;
    size_t cap = std::max<size_t>(count, 2 * ctx->d_items_cap);
    const size_t bytes = cap * sizeof(DevItem);
    if (ctx->allocated - ctx->d_items_cap * sizeof(DevItem) + bytes > ctx->budget) return GF2X_ENOMEM;
    if (ctx->d_items) {
        // the old buffer may still be read by enqueued work
        HIP_TRY(hipEventSynchronize(ctx->ws_free));
        HIP_TRY(hipFree(ctx->d_items));
        ctx->allocated -= ctx->d_items_cap * sizeof(DevItem);
        ctx->d_items = nullptr;
        ctx->d_items_cap = 0;
    }
    if (hipMalloc(&ctx->d_items, bytes) != hipSuccess) return GF2X_ENOMEM;
    ctx->d_items_cap = cap;
    ctx->allocated += bytes;
    return GF2X_OK;
}

// Change detector for the host descriptors behind a cached graph: a
// multiply-rotate mix over their 64-bit words in four independent lanes (not
// cryptographic; it only has to notice an edited descriptor array).
uint64_t checksum(const gf2x_item *items, uint32_t count) {
    const unsigned char *p = reinterpret_cast<const unsigned char *>(items);
    const size_t nw = (size_t)count * sizeof(gf2x_item) / 8;  // 4 words per item
    uint64_t h[4] = {0x9E3779B97F4A7C15ull ^ count, 0xC2B2AE3D27D4EB4Full, 0x165667B19E3779F9ull, 0x27D4EB2F165667C5ull};
    for (size_t i = 0; i < nw; ++i) {
        uint64_t w;
        std::memcpy(&w, p + 8 * i, 8);
        uint64_t &x = h[i & 3];
        x ^= w * 0xC2B2AE3D27D4EB4Full;
        x = ((x << 29) | (x >> 35)) * 0x9E3779B97F4A7C15ull;
    }
    return h[0] ^ ((h[1] << 16) | (h[1] >> 48)) ^ ((h[2] << 32) | (h[2] >> 32)) ^ ((h[3] << 48) | (h[3] >> 16));
}

// Host descriptors -> validated DevItems grouped by class, classes ordered
// by decreasing size, items in each group in submission order.  groups:
// (class, first index, count).
struct Group {
    int cls;
    uint32_t first, count;
    int lds = 0;  // fused launch: LDS bytes of its largest class
};

int build_items(gf2x_ctx *ctx, const gf2x_item *items, uint32_t count, std::vector<DevItem> &out,
                std::vector<Group> &groups, bool fused = false) {
    out.resize(count);
    for (uint32_t i = 0; i < count; ++i) {
        const gf2x_item &it = items[i];
        if (it.n_bits == 0 || it.n_bits > kMaxBits) return GF2X_EINVAL;
        int cls;
        if ((it.kind & 0xFFu) == GF2X_KIND_SPARSE) {  // weight in the upper 24 bits
            const int idx = sparse_class_for(it.n_bits);
            if (idx < 0) return GF2X_EINVAL;
            cls = kSparseBase + idx;
        } else if (it.kind == GF2X_KIND_CYCLIC || it.kind == GF2X_KIND_FULL) {
            cls = fused ? ctx->direct_of_w32[(it.n_bits + 31u) / 32u] : ctx->cls_of_w32[(it.n_bits + 31u) / 32u];
        } else {
            return GF2X_EINVAL;
        }
        if (fused && (is_sparse_class(cls) || !fused_class(cls))) return GF2X_ENOTSUP;
        out[i] = DevItem{it.n_bits, it.kind, (uint32_t)cls, 0u, it.a_off, it.b_off, it.c_off};
    }
    if (fused) {
        // one launch; the work queue hands out the most expensive items first
        std::stable_sort(out.begin(), out.end(), [](const DevItem &x, const DevItem &y) {
            return class_info((int)x.cls).ops > class_info((int)y.cls).ops;
        });
        int lds = 0;
        for (const DevItem &d : out) lds = std::max(lds, class_info((int)d.cls).lds_bytes);
        groups.assign(1, Group{kFusedCls, 0, count, lds});
        return GF2X_OK;
    }
    std::stable_sort(out.begin(), out.end(), [](const DevItem &x, const DevItem &y) {
        const int sx = class_info((int)x.cls).S, sy = class_info((int)y.cls).S;
        return sx != sy ? sx > sy : x.cls < y.cls;
    });
    groups.clear();
    for (uint32_t i = 0; i < count; ++i) {
        if (groups.empty() || groups.back().cls != (int)out[i].cls) groups.push_back(Group{(int)out[i].cls, i, 0});
        groups.back().count++;
    }
    return GF2X_OK;
}

int ensure_forks(gf2x_ctx *ctx) {
    if (ctx->fork_stream[0]) return GF2X_OK;
    for (int i = 0; i < gf2x_ctx::kForks; ++i) HIP_TRY(hipStreamCreateWithFlags(&ctx->fork_stream[i], hipStreamNonBlocking));
    for (int i = 0; i <= gf2x_ctx::kForks; ++i) HIP_TRY(hipEventCreateWithFlags(&ctx->fork_event[i], hipEventDisableTiming));
    return GF2X_OK;
}

// Workspace bytes of the staged groups of a launch (each group gets its own
// region, since groups may run concurrently).
size_t staged_bytes(const std::vector<Group> &groups) {
    size_t total = 0;
    for (const Group &g : groups) total += (staged_workspace_bytes(g.cls, g.count) + 255) / 256 * 256;
    return total;
}

// Grow a workspace owned by the context (ws/ws_bytes) to `need` bytes within
// the budget; the old buffer is freed after the device is done with it.
int ensure_ws(gf2x_ctx *ctx, void *&ws, size_t &ws_bytes, size_t need, hipEvent_t guard, bool guard_used) {
    if (need <= ws_bytes) return GF2X_OK;
    if (ctx->allocated - ws_bytes + need > ctx->budget) return GF2X_ENOMEM;
    if (ws) {
        if (guard_used) HIP_TRY(hipEventSynchronize(guard));
        HIP_TRY(hipFree(ws));
        ctx->allocated -= ws_bytes;
        ws = nullptr;
        ws_bytes = 0;
    }
    if (hipMalloc(&ws, need) != hipSuccess) return GF2X_ENOMEM;
    ws_bytes = need;
    ctx->allocated += need;
    return GF2X_OK;
}

// Staged groups whose workspace does not fit the budget run their direct class.
void fit_staged(gf2x_ctx *ctx, std::vector<Group> &groups, size_t have) {
    size_t total = staged_bytes(groups);
    const size_t avail = ctx->budget > ctx->allocated ? ctx->budget - ctx->allocated + have : have;
    for (Group &g : groups) {
        if (total <= avail) break;
        if (class_info(g.cls).child >= 0) {
            total -= (staged_workspace_bytes(g.cls, g.count) + 255) / 256 * 256;
            g.cls = class_info(g.cls).direct;
        }
    }
}

int launch_one(gf2x_ctx *ctx, const Group &g, const DevItem *d_items, char *&ws, uint64_t *c, const uint64_t *a,
               const uint64_t *b, hipStream_t s, uint32_t *queue = nullptr) {
    hipError_t e;
    if (g.cls == kFusedCls) {
        e = launch_fused(d_items + g.first, g.count, g.lds, c, a, b, queue, ctx->num_cu, s);
    } else if (class_info(g.cls).child >= 0) {
        e = launch_staged(g.cls, d_items + g.first, g.count, c, a, b, ws, ctx->num_cu, s);
        ws += (staged_workspace_bytes(g.cls, g.count) + 255) / 256 * 256;
    } else {
        e = launch_batched(g.cls, d_items + g.first, g.count, c, a, b, ctx->num_cu, s);
    }
    return e == hipSuccess ? GF2X_OK : device_error(e);
}

// One launch per class group.  A single group goes straight onto s; several
// groups are spread over the context's internal streams, forked from s and
// joined back to it with events, so that different sizes overlap.  Staged
// groups carve their regions out of ws in group order.
int launch_groups(gf2x_ctx *ctx, const DevItem *d_items, const std::vector<Group> &groups, uint64_t *c,
                  const uint64_t *a, const uint64_t *b, void *ws, hipStream_t s, uint32_t *queue = nullptr) {
    char *wp = reinterpret_cast<char *>(ws);
    if (groups.size() == 1) return launch_one(ctx, groups[0], d_items, wp, c, a, b, s, queue);
    int rc = ensure_forks(ctx);
    if (rc) return rc;
    const int K = std::min<int>(gf2x_ctx::kForks, (int)groups.size());
    HIP_TRY(hipEventRecord(ctx->fork_event[gf2x_ctx::kForks], s));
    for (int k = 0; k < K; ++k) HIP_TRY(hipStreamWaitEvent(ctx->fork_stream[k], ctx->fork_event[gf2x_ctx::kForks], 0));
    for (size_t i = 0; i < groups.size(); ++i) {
        rc = launch_one(ctx, groups[i], d_items, wp, c, a, b, ctx->fork_stream[i % K]);
        if (rc) return rc;
    }
    for (int k = 0; k < K; ++k) {
        HIP_TRY(hipEventRecord(ctx->fork_event[k], ctx->fork_stream[k]));
        HIP_TRY(hipStreamWaitEvent(s, ctx->fork_event[k], 0));
    }
    return GF2X_OK;
}

// Release a recorded batch: wait for its last launch, then free its graph,
// descriptors and workspace and return their bytes to the budget.
void release_entry(gf2x_ctx *ctx, GraphEntry &g) {
    if (g.done && g.launched) hipEventSynchronize(g.done);
    if (g.exec) hipGraphExecDestroy(g.exec);
    if (g.graph) hipGraphDestroy(g.graph);
    if (g.items) hipFree(g.items);
    if (g.staged_ws) hipFree(g.staged_ws);
    if (g.done) hipEventDestroy(g.done);
    ctx->allocated -= g.bytes;
    g = GraphEntry{};
}

// Record the launch sequence of a validated batch (host descriptors `host`,
// class groups `groups`) into g: private descriptor and workspace buffers
// within the budget, the launches captured on a private stream.  The
// descriptors are copied on copy_stream (ordered before the first replay on
// that stream), or synchronously when copy_stream is null.
int record_graph(gf2x_ctx *ctx, const std::vector<DevItem> &host, std::vector<Group> &groups, uint64_t *c_base,
                 const uint64_t *a_base, const uint64_t *b_base, GraphEntry &g, hipStream_t copy_stream,
                 bool use_copy_stream) {
    g = GraphEntry{};
    fit_staged(ctx, groups, 0);
    const size_t sb = staged_bytes(groups);
    const size_t ib = (host.size() * sizeof(DevItem) + 255) / 256 * 256 + 256;  // + fused queue counters
    if (ctx->allocated + sb + ib > ctx->budget) return GF2X_ENOMEM;
    if (hipMalloc(&g.items, ib) != hipSuccess) {
        g.items = nullptr;
        return GF2X_ENOMEM;
    }
    if (sb && hipMalloc(&g.staged_ws, sb) != hipSuccess) {
        g.staged_ws = nullptr;
        hipFree(g.items);
        g.items = nullptr;
        return GF2X_ENOMEM;
    }
    g.bytes = ib + sb;
    ctx->allocated += g.bytes;
    g.queue = reinterpret_cast<uint32_t *>(reinterpret_cast<char *>(g.items) + ib - 256);
    hipError_t e = use_copy_stream ? hipMemsetAsync(g.queue, 0, 256, copy_stream) : hipMemset(g.queue, 0, 256);
    if (e == hipSuccess)
        e = use_copy_stream
                       ? hipMemcpyAsync(g.items, host.data(), host.size() * sizeof(DevItem), hipMemcpyHostToDevice,
                                        copy_stream)
                : hipMemcpy(g.items, host.data(), host.size() * sizeof(DevItem), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&g.done, hipEventDisableTiming);
    hipStream_t cap = nullptr;
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&cap, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
        int lrc = launch_groups(ctx, g.items, groups, c_base, a_base, b_base, g.staged_ws, cap, g.queue);
        hipError_t e2 = hipStreamEndCapture(cap, &g.graph);
        e = lrc ? hipErrorLaunchFailure : e2;
    }
    if (e == hipSuccess) e = hipGraphInstantiate(&g.exec, g.graph, nullptr, nullptr, 0);
    if (cap) hipStreamDestroy(cap);
    if (e != hipSuccess) {
        release_entry(ctx, g);
        return device_error(e);
    }
    return GF2X_OK;
}

int replay(GraphEntry &g, hipStream_t s) {
    HIP_TRY(hipGraphLaunch(g.exec, s));
    HIP_TRY(hipEventRecord(g.done, s));
    g.launched = true;
    return GF2X_OK;
}

constexpr size_t kSingleChunk = 256;       // descriptors per device chunk
constexpr size_t kMaxSingleItems = 4096;  // distinct (n, kind) kept on the device

// One product: a direct class runs in one workgroup; a staged class spreads
// it over the workgroups of its point products (lower latency for large n),
// through the same descriptor and workspace path as a batch of one.
int single_product(gf2x_ctx *ctx, uint64_t *c, const uint64_t *a, const uint64_t *b, uint32_t n_bits,
                   uint32_t kind, hipStream_t s, int force_cls = -1) {
    HIP_TRY(hipSetDevice(ctx->device));
    const int cls = force_cls >= 0 ? force_cls : ctx->single_of_w32[(n_bits + 31u) / 32u];
    if (class_info(cls).child < 0) {
        HIP_TRY(launch_single(cls, a, b, c, n_bits, kind, s));
        return GF2X_OK;
    }
    // Under stream capture the product stays one launch of the direct class:
    // the staged path waits on the context's workspace event and may write a
    // descriptor synchronously, neither of which belongs in a captured graph.
    hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
    HIP_TRY(hipStreamIsCapturing(s, &cap));
    if (cap != hipStreamCaptureStatusNone) {
        HIP_TRY(launch_single(class_info(cls).direct, a, b, c, n_bits, kind, s));
        return GF2X_OK;
    }
    // the descriptor of (n, kind) lives on the device once written: no copy per call
    DevItem *d_item = nullptr;
    auto found = ctx->single_items.find({n_bits, kind});
    if (found != ctx->single_items.end()) {
        d_item = found->second;
    } else if (ctx->single_items.size() < kMaxSingleItems) {
        if (ctx->single_chunks.empty() || ctx->single_used == kSingleChunk) {
            if (ctx->allocated + kSingleChunk * sizeof(DevItem) > ctx->budget) return GF2X_ENOMEM;
            DevItem *chunk = nullptr;
            HIP_TRY(hipMalloc(&chunk, kSingleChunk * sizeof(DevItem)));
            ctx->allocated += kSingleChunk * sizeof(DevItem);
            ctx->single_chunks.push_back(chunk);
            ctx->single_used = 0;
        }
        d_item = ctx->single_chunks.back() + ctx->single_used;
        const DevItem item{n_bits, kind, (uint32_t)cls, 0u, 0u, 0u, 0u};
        HIP_TRY(hipMemcpy(d_item, &item, sizeof item, hipMemcpyHostToDevice));
        ++ctx->single_used;
        ctx->single_items[{n_bits, kind}] = d_item;
    } else {  // table full: one workgroup
        HIP_TRY(launch_single(class_info(cls).direct, a, b, c, n_bits, kind, s));
        return GF2X_OK;
    }
    const size_t need = (staged_workspace_bytes(cls, 1) + 255) / 256 * 256;
    int rc = ensure_ws(ctx, ctx->staged_ws, ctx->staged_ws_bytes, need, ctx->ws_free, ctx->ws_used);
    if (rc == GF2X_ENOMEM) {  // no room for the workspace within the budget: one workgroup
        HIP_TRY(launch_single(class_info(cls).direct, a, b, c, n_bits, kind, s));
        return GF2X_OK;
    }
    if (rc) return rc;
    if (ctx->ws_used) HIP_TRY(hipStreamWaitEvent(s, ctx->ws_free, 0));
    HIP_TRY(launch_staged(cls, d_item, 1, c, a, b, ctx->staged_ws, ctx->num_cu, s));
    HIP_TRY(hipEventRecord(ctx->ws_free, s));
    ctx->ws_used = true;
    return GF2X_OK;
}

// n an odd prime: X^n - 1 is then (X + 1) times irreducibles of degree
// ord_n(2), which divides n - 1, so every unit u of F2[X]/(X^n - 1) has
// u^(2^(n-1) - 1) = 1.
bool odd_prime(uint32_t n) {
    if (n < 3 || n % 2 == 0) return false;
    for (uint32_t d = 3; (uint64_t)d * d <= n; d += 2)
        if (n % d == 0) return false;
    return true;
}

// 2^(-j) mod the prime n (2^(n-1) = 1).
uint32_t inv_pow2(uint32_t n, uint64_t j) {
    uint64_t e = (n - 1) - j % (n - 1), r = 1, b = 2 % n;
    while (e) {
        if (e & 1) r = r * b % n;
        b = b * b % n;
        e >>= 1;
    }
    return (uint32_t)r;
}

}  // namespace

extern "C" {

int gf2x_version(void) { return 10000; }

const char *gf2x_strerror(int code) {
    switch (code) {
        case GF2X_OK: return "success";
        case GF2X_EINVAL: return "invalid argument";
        case GF2X_ENOMEM: return "device workspace exceeds the budget or could not be allocated";
        case GF2X_EDEVICE: return "HIP runtime error";
        case GF2X_EAGAIN: return "queue full or timed out; try again later";
        case GF2X_ENOTSUP: return "unsupported combination of flags";
        default: return "unknown error code";
    }
}

const char *gf2x_last_device_error(void) { return g_last_device_error.c_str(); }

int gf2x_create(gf2x_ctx **out, const gf2x_opts *opts) {
    if (!out) return GF2X_EINVAL;
    *out = nullptr;
    gf2x_opts o{};
    if (opts) o = *opts;
    if (o.flags != 0) return GF2X_EINVAL;
    int ndev = 0;
    HIP_TRY(hipGetDeviceCount(&ndev));
    if (o.device < 0 || o.device >= ndev) return GF2X_EINVAL;
    HIP_TRY(hipSetDevice(o.device));
    gf2x_ctx *ctx = new (std::nothrow) gf2x_ctx();
    if (!ctx) return GF2X_ENOMEM;
    ctx->device = o.device;
    ctx->budget = o.hbm_budget_bytes ? o.hbm_budget_bytes : ((size_t)1 << 30);
    hipDeviceProp_t prop;
    hipError_t e = hipGetDeviceProperties(&prop, o.device);
    if (e == hipSuccess) e = prepare_kernels();
    // this device's copy of the allocation-free scratch array (device current)
    if (e == hipSuccess) e = scratch_for_device(o.device, &ctx->scratch);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&ctx->ws_free, hipEventDisableTiming);
    if (e != hipSuccess) {
        delete ctx;
        return device_error(e);
    }
    ctx->num_cu = prop.multiProcessorCount;
    default_table(ctx);
    if (o.tune_cache) load_tune_cache(ctx, o.tune_cache);
    direct_table(ctx);
    int rc = upload_direct_table(ctx);
    if (rc == GF2X_OK) {
        e = hipMalloc(&ctx->d_queue, 256);
        if (e == hipSuccess) e = hipMemset(ctx->d_queue, 0, 256);
        if (e == hipSuccess) ctx->allocated += 256;
        else rc = device_error(e);
    }
    if (rc) {
        gf2x_destroy(ctx);
        return rc;
    }
    *out = ctx;
    return GF2X_OK;
}

void gf2x_destroy(gf2x_ctx *ctx) {
    if (!ctx) return;
    hipSetDevice(ctx->device);
    for (auto &kv : ctx->graphs) release_entry(ctx, kv.second);
    if (ctx->staged_ws) hipFree(ctx->staged_ws);
    if (ctx->inv_ws) hipFree(ctx->inv_ws);
    toeplitz::release(ctx->tz);
    for (int i = 0; i < gf2x_ctx::kForks; ++i)
        if (ctx->fork_stream[i]) hipStreamDestroy(ctx->fork_stream[i]);
    for (int i = 0; i <= gf2x_ctx::kForks; ++i)
        if (ctx->fork_event[i]) hipEventDestroy(ctx->fork_event[i]);
    if (ctx->d_items) hipFree(ctx->d_items);
    for (gf2x::DevItem *chunk : ctx->single_chunks) hipFree(chunk);
    if (ctx->d_cls) hipFree(ctx->d_cls);
    if (ctx->d_queue) hipFree(ctx->d_queue);
    if (ctx->ws_free) hipEventDestroy(ctx->ws_free);
    delete ctx;
}

int gf2x_mul(gf2x_ctx *ctx, uint64_t *c, const uint64_t *a, const uint64_t *b, uint32_t n_bits,
             gf2x_stream_t stream) {
    int rc = check_single(ctx, c, a, b, n_bits, 2 * words64(n_bits));
    if (rc) return rc;
    return single_product(ctx, c, a, b, n_bits, kKindFull, reinterpret_cast<hipStream_t>(stream));
}

int gf2x_mul_cyclic(gf2x_ctx *ctx, uint64_t *c, const uint64_t *a, const uint64_t *b, uint32_t n_bits,
                    gf2x_stream_t stream) {
    int rc = check_single(ctx, c, a, b, n_bits, words64(n_bits));
    if (rc) return rc;
    return single_product(ctx, c, a, b, n_bits, kKindCyclic, reinterpret_cast<hipStream_t>(stream));
}

// The batched calls refuse a stream under capture: they order the context's
// workspace with the context's event, write descriptors into context-owned
// buffers that later calls reuse or reallocate, and copy host descriptors
// from memory that is gone once the call returns.  A graph recorded from
// them could not be replayed safely; GF2X_USE_GRAPH records one that can.
static int refuse_capture(hipStream_t s) {
    hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
    const hipError_t e = hipStreamIsCapturing(s, &cap);
    if (e != hipSuccess) return device_error(e);
    return cap == hipStreamCaptureStatusNone ? GF2X_OK : GF2X_ENOTSUP;
}

int gf2x_mul_batched(gf2x_ctx *ctx, const gf2x_item *items, uint32_t count, uint64_t *c_base,
                     const uint64_t *a_base, const uint64_t *b_base, uint32_t flags, gf2x_stream_t stream) {
    if (!ctx) return GF2X_EINVAL;
    if (count == 0) return GF2X_OK;
    if (!items || !c_base || !a_base || !b_base) return GF2X_EINVAL;
    if (!aligned8(c_base) || !aligned8(a_base) || !aligned8(b_base)) return GF2X_EINVAL;
    const uint32_t known = GF2X_ITEMS_ON_DEVICE | GF2X_SHARED_A | GF2X_FORCE_PACKED | GF2X_FORCE_TOEPLITZ |
                           GF2X_USE_GRAPH | GF2X_FUSED;
    if (flags & ~known) return GF2X_EINVAL;
    const bool fused = (flags & GF2X_FUSED) != 0;
    if (fused && (flags & (GF2X_ITEMS_ON_DEVICE | GF2X_SHARED_A))) return GF2X_ENOTSUP;
    if ((flags & GF2X_FORCE_PACKED) && (flags & GF2X_FORCE_TOEPLITZ)) return GF2X_EINVAL;
    if ((flags & GF2X_FORCE_TOEPLITZ) && !(flags & GF2X_SHARED_A)) return GF2X_ENOTSUP;
    const bool dev_items = (flags & GF2X_ITEMS_ON_DEVICE) != 0;
    if (dev_items && (flags & (GF2X_USE_GRAPH | GF2X_SHARED_A))) return GF2X_ENOTSUP;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    HIP_TRY(hipSetDevice(ctx->device));
    if (int rc = refuse_capture(s)) return rc;

    if (dev_items) {
        // Descriptors stay on the device; the class comes from the size table.
        int rc = ensure_items(ctx, count);
        if (rc) return rc;
        if (ctx->ws_used) HIP_TRY(hipStreamWaitEvent(s, ctx->ws_free, 0));
        HIP_TRY(launch_convert_items(items, count, ctx->d_items, s));
        HIP_TRY(launch_mixed(ctx->d_items, count, c_base, a_base, b_base, ctx->d_cls, ctx->d_queue + kBadCounter,
                             ctx->num_cu, s));
        HIP_TRY(hipEventRecord(ctx->ws_free, s));
        ctx->ws_used = true;
        return GF2X_OK;
    }

    // Host descriptors: validate, order by decreasing n, pick the path.
    if (flags & GF2X_SHARED_A) {
        for (uint32_t i = 0; i < count; ++i)
            if (items[i].a_off != items[0].a_off || items[i].n_bits != items[0].n_bits ||
                items[i].kind != GF2X_KIND_CYCLIC)
                return GF2X_EINVAL;
        if (items[0].n_bits == 0 || items[0].n_bits > kMaxBits) return GF2X_EINVAL;
        if (flags & GF2X_FORCE_TOEPLITZ) {
            if (int rc = check_ranges(items, count, c_base, a_base, b_base)) return rc;
            int rc = toeplitz::run(ctx->tz, ctx->budget, ctx->allocated, items, count, c_base, a_base, b_base,
                                   ctx->num_cu, s);
            if (rc == GF2X_EDEVICE) g_last_device_error = toeplitz::last_error();
            return rc;
        }
    }
    if (flags & GF2X_USE_GRAPH) {
        // A cache hit costs one pass over the descriptor words (the change
        // check) and the replay; validation and grouping ran when the entry
        // was recorded.
        auto key = std::make_tuple((const void *)items, count, (const void *)c_base, (const void *)a_base,
                                   (const void *)b_base, flags, (void *)s);
        const uint64_t sum = checksum(items, count);
        auto it = ctx->graphs.find(key);
        if (it != ctx->graphs.end() && it->second.checksum == sum) {
            it->second.last_use = ++ctx->graph_clock;
            return replay(it->second, s);
        }
        if (it != ctx->graphs.end()) {  // the descriptors changed: record again
            release_entry(ctx, it->second);
            ctx->graphs.erase(it);
        }
        std::vector<DevItem> host;
        std::vector<Group> groups;
        int rc = build_items(ctx, items, count, host, groups, fused);
        if (rc == GF2X_OK) rc = check_ranges(items, count, c_base, a_base, b_base);
        if (rc) return rc;
        while (ctx->graphs.size() >= gf2x_ctx::kMaxGraphs) {
            auto lru = ctx->graphs.begin();
            for (auto j = ctx->graphs.begin(); j != ctx->graphs.end(); ++j)
                if (j->second.last_use < lru->second.last_use) lru = j;
            release_entry(ctx, lru->second);
            ctx->graphs.erase(lru);
        }
        GraphEntry g;
        rc = record_graph(ctx, host, groups, c_base, a_base, b_base, g, s, true);
        if (rc == GF2X_ENOMEM && !ctx->graphs.empty()) {
            // release the cached entries (their budget) and try once more
            for (auto &kv : ctx->graphs) release_entry(ctx, kv.second);
            ctx->graphs.clear();
            rc = build_items(ctx, items, count, host, groups, fused);
            if (rc == GF2X_OK) rc = record_graph(ctx, host, groups, c_base, a_base, b_base, g, s, true);
        }
        if (rc) return rc;
        g.checksum = sum;
        g.last_use = ++ctx->graph_clock;
        it = ctx->graphs.emplace(key, g).first;
        return replay(it->second, s);
    }

    std::vector<DevItem> host;
    std::vector<Group> groups;
    int rc = build_items(ctx, items, count, host, groups, fused);
    if (rc == GF2X_OK) rc = check_ranges(items, count, c_base, a_base, b_base);
    if (rc) return rc;
    rc = ensure_items(ctx, count);
    if (rc) return rc;
    fit_staged(ctx, groups, ctx->staged_ws_bytes);
    rc = ensure_ws(ctx, ctx->staged_ws, ctx->staged_ws_bytes, staged_bytes(groups), ctx->ws_free, ctx->ws_used);
    if (rc) return rc;
    if (ctx->ws_used) HIP_TRY(hipStreamWaitEvent(s, ctx->ws_free, 0));
    HIP_TRY(hipMemcpyAsync(ctx->d_items, host.data(), count * sizeof(DevItem), hipMemcpyHostToDevice, s));
    rc = launch_groups(ctx, ctx->d_items, groups, c_base, a_base, b_base, ctx->staged_ws, s, ctx->d_queue);
    if (rc) return rc;
    HIP_TRY(hipEventRecord(ctx->ws_free, s));
    ctx->ws_used = true;
    return GF2X_OK;
}

// The batch of gf2x_mul_batched (host items) in the static scratch array of
// the context's device: descriptors and staged workspace, no allocation.
// Groups run one after another on the caller's stream; a staged group whose
// workspace does not fit the scratch that is left runs its direct class.
int gf2x_mul_batched_noalloc(gf2x_ctx *ctx, const gf2x_item *items, uint32_t count, uint64_t *c_base,
                             const uint64_t *a_base, const uint64_t *b_base, gf2x_stream_t stream) {
    if (!ctx) return GF2X_EINVAL;
    if (count == 0) return GF2X_OK;
    if (!items || !c_base || !a_base || !b_base) return GF2X_EINVAL;
    if (!aligned8(c_base) || !aligned8(a_base) || !aligned8(b_base)) return GF2X_EINVAL;
    if (count > kScratchMaxItems) return GF2X_ENOMEM;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    HIP_TRY(hipSetDevice(ctx->device));
    if (int rc = refuse_capture(s)) return rc;
    thread_local std::vector<DevItem> host;
    thread_local std::vector<Group> groups;
    int rc = build_items(ctx, items, count, host, groups);
    if (rc == GF2X_OK) rc = check_ranges(items, count, c_base, a_base, b_base);
    if (rc) return rc;
    const size_t cap = kScratchBytes - kScratchItemBytes;
    size_t total = staged_bytes(groups);
    for (Group &g : groups) {
        if (total <= cap) break;
        if (class_info(g.cls).child >= 0) {
            total -= (staged_workspace_bytes(g.cls, g.count) + 255) / 256 * 256;
            g.cls = class_info(g.cls).direct;
        }
    }
    char *base = reinterpret_cast<char *>(ctx->scratch);
    DevItem *desc = reinterpret_cast<DevItem *>(base);
    HIP_TRY(hipMemcpyAsync(desc, host.data(), (size_t)count * sizeof(DevItem), hipMemcpyHostToDevice, s));
    char *wp = base + kScratchItemBytes;
    for (const Group &g : groups) {
        rc = launch_one(ctx, g, desc, wp, c_base, a_base, b_base, s);
        if (rc) return rc;
    }
    return GF2X_OK;
}

int gf2x_device_item_errors(gf2x_ctx *ctx, uint64_t *count) {
    if (!ctx || !count) return GF2X_EINVAL;
    HIP_TRY(hipSetDevice(ctx->device));
    HIP_TRY(hipDeviceSynchronize());
    uint32_t v = 0;
    HIP_TRY(hipMemcpy(&v, ctx->d_queue + kBadCounter, 4, hipMemcpyDeviceToHost));
    HIP_TRY(hipMemset(ctx->d_queue + kBadCounter, 0, 4));
    *count = v;
    return GF2X_OK;
}

int gf2x_plan_create(gf2x_plan **out, gf2x_ctx *ctx, const gf2x_item *items, uint32_t count, uint64_t *c_base,
                     const uint64_t *a_base, const uint64_t *b_base, uint32_t flags) {
    if (!out) return GF2X_EINVAL;
    *out = nullptr;
    if (!ctx || (flags & ~GF2X_FUSED)) return GF2X_EINVAL;
    if (count && (!items || !c_base || !a_base || !b_base)) return GF2X_EINVAL;
    if (!aligned8(c_base) || !aligned8(a_base) || !aligned8(b_base)) return GF2X_EINVAL;
    HIP_TRY(hipSetDevice(ctx->device));
    gf2x_plan *plan = new (std::nothrow) gf2x_plan();
    if (!plan) return GF2X_ENOMEM;
    plan->ctx = ctx;
    if (count) {
        std::vector<DevItem> host;
        std::vector<Group> groups;
        int rc = build_items(ctx, items, count, host, groups, (flags & GF2X_FUSED) != 0);
        if (rc == GF2X_OK) rc = check_ranges(items, count, c_base, a_base, b_base);
        if (rc == GF2X_OK) rc = record_graph(ctx, host, groups, c_base, a_base, b_base, plan->g, nullptr, false);
        if (rc) {
            delete plan;
            return rc;
        }
        if (groups.size() == 1) {  // (after record_graph: a staged group may have become direct)
            plan->one_group = true;
            plan->cls = groups[0].cls;
            plan->first = groups[0].first;
            plan->count = groups[0].count;
            plan->lds = groups[0].lds;
            plan->c = c_base;
            plan->a = a_base;
            plan->b = b_base;
        }
    }
    *out = plan;
    return GF2X_OK;
}

int gf2x_plan_launch(gf2x_plan *plan, gf2x_stream_t stream) {
    if (!plan) return GF2X_EINVAL;
    if (!plan->g.exec) return GF2X_OK;  // empty batch
    HIP_TRY(hipSetDevice(plan->ctx->device));
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    if (!plan->one_group) return replay(plan->g, s);
    // one size class: its kernels (one, or four for a staged class) on the
    // plan's descriptors, workspace and queue, then the plan's event
    const Group g{plan->cls, plan->first, plan->count, plan->lds};
    char *ws = reinterpret_cast<char *>(plan->g.staged_ws);
    const int rc = launch_one(plan->ctx, g, plan->g.items, ws, plan->c, plan->a, plan->b, s, plan->g.queue);
    if (rc) return rc;
    HIP_TRY(hipEventRecord(plan->g.done, s));
    plan->g.launched = true;
    return GF2X_OK;
}

void gf2x_plan_destroy(gf2x_plan *plan) {
    if (!plan) return;
    hipSetDevice(plan->ctx->device);
    release_entry(plan->ctx, plan->g);
    delete plan;
}

// Inversion by exponentiation (the Itoh-Tsujii addition chain): for an odd
// prime n, an invertible a has a^(2^(n-1) - 1) = 1, so a^-1 =
// a^(2^(n-1) - 2) = (a^(2^(n-2) - 1))^2.  b_k = a^(2^k - 1) follows the
// binary digits of m = n - 2 from the top: b_2k = b_k^(2^k) * b_k, and
// b_(k+1) = b_k^2 * a.  Squaring j times is a bit permutation; every step
// runs on all items at once (one permutation launch, one batched product).
int gf2x_inv_cyclic_batched(gf2x_ctx *ctx, const gf2x_item *items, uint32_t count, uint64_t *c_base,
                            const uint64_t *a_base, uint32_t flags, gf2x_stream_t stream) {
    if (!ctx || (count && (!items || !c_base || !a_base))) return GF2X_EINVAL;
    if (flags != 0) return GF2X_EINVAL;
    if (count == 0) return GF2X_OK;
    const uint32_t n = items[0].n_bits;
    for (uint32_t i = 0; i < count; ++i)
        if (items[i].n_bits != n || items[i].kind != GF2X_KIND_CYCLIC) return GF2X_EINVAL;
    if (n > kMaxBits || !odd_prime(n)) return GF2X_EINVAL;
    if (!aligned8(c_base) || !aligned8(a_base)) return GF2X_EINVAL;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    HIP_TRY(hipSetDevice(ctx->device));
    if (int rc = refuse_capture(s)) return rc;
    const uint64_t W = words64(n);
    const uint32_t w32 = (n + 31u) / 32u;
    const int cls = count <= 64 ? ctx->single_of_w32[w32] : ctx->cls_of_w32[w32];
    // working buffers: A (a), X (b_k), Y, Z, then the offsets and descriptors
    const size_t buf = (size_t)count * W * 8;
    const size_t offs = ((size_t)count * 8 + 255) / 256 * 256;
    const size_t need = 4 * ((buf + 255) / 256 * 256) + 2 * offs + (size_t)count * sizeof(DevItem);
    int rc = ensure_ws(ctx, ctx->inv_ws, ctx->inv_ws_bytes, need, ctx->ws_free, ctx->ws_used);
    if (rc) return rc;
    Group g{cls, 0, count};
    if (class_info(cls).child >= 0) {
        rc = ensure_ws(ctx, ctx->staged_ws, ctx->staged_ws_bytes, (staged_workspace_bytes(cls, count) + 255) / 256 * 256,
                       ctx->ws_free, ctx->ws_used);
        if (rc == GF2X_ENOMEM) g.cls = class_info(cls).direct;
        else if (rc) return rc;
    }
    char *p = reinterpret_cast<char *>(ctx->inv_ws);
    const size_t stride = (buf + 255) / 256 * 256;
    uint64_t *A = reinterpret_cast<uint64_t *>(p);
    uint64_t *X = reinterpret_cast<uint64_t *>(p + stride);
    uint64_t *Y = reinterpret_cast<uint64_t *>(p + 2 * stride);
    uint64_t *Z = reinterpret_cast<uint64_t *>(p + 3 * stride);
    uint64_t *d_aoff = reinterpret_cast<uint64_t *>(p + 4 * stride);
    uint64_t *d_coff = reinterpret_cast<uint64_t *>(p + 4 * stride + offs);
    DevItem *d_it = reinterpret_cast<DevItem *>(p + 4 * stride + 2 * offs);
    std::vector<uint64_t> ho(2 * (size_t)count);
    std::vector<DevItem> hi(count);
    for (uint32_t i = 0; i < count; ++i) {
        ho[i] = items[i].a_off;
        ho[count + i] = items[i].c_off;
        hi[i] = DevItem{n, kKindCyclic, (uint32_t)g.cls, 0u, i * W, i * W, i * W};
    }
    if (ctx->ws_used) HIP_TRY(hipStreamWaitEvent(s, ctx->ws_free, 0));
    HIP_TRY(hipMemcpyAsync(d_aoff, ho.data(), count * 8, hipMemcpyHostToDevice, s));
    HIP_TRY(hipMemcpyAsync(d_coff, ho.data() + count, count * 8, hipMemcpyHostToDevice, s));
    HIP_TRY(hipMemcpyAsync(d_it, hi.data(), count * sizeof(DevItem), hipMemcpyHostToDevice, s));
    HIP_TRY(launch_gather_items(a_base, d_aoff, A, n, count, s));
    HIP_TRY(hipMemcpyAsync(X, A, buf, hipMemcpyDeviceToDevice, s));
    const uint32_t m = n - 2;
    int top = 31;
    while (!((m >> top) & 1u)) --top;
    uint64_t k = 1;
    auto product = [&](const uint64_t *f, const uint64_t *h, uint64_t *out) -> int {
        char *ws = reinterpret_cast<char *>(ctx->staged_ws);
        return launch_one(ctx, g, d_it, ws, out, f, h, s);
    };
    for (int bit = top - 1; bit >= 0; --bit) {
        HIP_TRY(launch_frobenius(X, Y, nullptr, n, count, inv_pow2(n, k), s));  // b^(2^k)
        rc = product(Y, X, Z);                                                  // b_2k
        if (rc) return rc;
        std::swap(X, Z);
        k *= 2;
        if ((m >> bit) & 1u) {
            HIP_TRY(launch_frobenius(X, Y, nullptr, n, count, inv_pow2(n, 1), s));  // b^2
            rc = product(Y, A, Z);                                                  // b_(k+1)
            if (rc) return rc;
            std::swap(X, Z);
            k += 1;
        }
    }
    if (k != m) return GF2X_EINVAL;  // cannot happen: the chain follows the digits of m
    HIP_TRY(launch_frobenius(X, c_base, d_coff, n, count, inv_pow2(n, 1), s));  // (b_m)^2
    HIP_TRY(hipEventRecord(ctx->ws_free, s));
    ctx->ws_used = true;
    return GF2X_OK;
}

int gf2x_tune(gf2x_ctx *ctx, const uint32_t *sizes, uint32_t nsizes, uint32_t batch, const char *out_path) {
    if (!ctx || (!sizes && nsizes) || batch == 0) return GF2X_EINVAL;
    for (uint32_t i = 0; i < nsizes; ++i)
        if (sizes[i] == 0 || sizes[i] > kMaxBits) return GF2X_EINVAL;
    HIP_TRY(hipSetDevice(ctx->device));
    uint32_t maxn = 0;
    for (uint32_t i = 0; i < nsizes; ++i) maxn = std::max(maxn, sizes[i]);
    if (nsizes) {
        const uint64_t W = words64(maxn);
        size_t staged = 0;
        for (int c = 0; c < kNumClasses; ++c) staged = std::max(staged, staged_workspace_bytes(c, batch));
        const size_t main_bytes = (size_t)batch * W * 8 * 3 + (size_t)batch * sizeof(DevItem);
        const size_t bytes = (main_bytes + 255) / 256 * 256 + staged;
        if (ctx->allocated + bytes > ctx->budget) return GF2X_ENOMEM;
        uint64_t *buf = nullptr;
        if (hipMalloc(&buf, bytes) != hipSuccess) return GF2X_ENOMEM;
        hipStream_t s = nullptr;
        hipEvent_t e0 = nullptr, e1 = nullptr;
        hipError_t e = hipStreamCreateWithFlags(&s, hipStreamNonBlocking);
        if (e == hipSuccess) e = hipEventCreate(&e0);
        if (e == hipSuccess) e = hipEventCreate(&e1);
        if (e == hipSuccess) e = launch_fill_words(buf, (size_t)batch * W * 2, 0x2201047300ull, s);
        uint64_t *A = buf, *B = buf + (size_t)batch * W, *C = buf + (size_t)2 * batch * W;
        DevItem *d_items = reinterpret_cast<DevItem *>(buf + (size_t)3 * batch * W);
        void *staged_ws = reinterpret_cast<char *>(buf) + (main_bytes + 255) / 256 * 256;
        std::vector<DevItem> host(batch);
        for (uint32_t i = 0; e == hipSuccess && i < nsizes; ++i) {
            const uint32_t n = sizes[i], w32 = (n + 31u) / 32u;
            const uint64_t Wn = words64(n);
            for (uint32_t k = 0; k < batch; ++k) host[k] = DevItem{n, kKindCyclic, 0u, 0u, k * Wn, k * Wn, k * Wn};
            e = hipMemcpyAsync(d_items, host.data(), batch * sizeof(DevItem), hipMemcpyHostToDevice, s);
            // Two passes over the candidates (so that no candidate is only
            // measured while the clocks settle); per pass and candidate, one
            // warm-up launch and three timed ones.  A class's batch time is
            // its minimum over both passes, its single-product latency the
            // median of its nine timed calls in the last pass.
            float batch_ms[kNumClasses], single_ms[kNumClasses];
            for (int c = 0; c < kNumClasses; ++c) batch_ms[c] = single_ms[c] = -1.f;
            for (int pass = 0; pass < 2; ++pass) {
                for (int c = 0; e == hipSuccess && c < kNumClasses; ++c) {
                    const ClassInfo &ci = class_info(c);
                    if ((uint32_t)ci.S < w32 || (double)ci.S > 1.6 * w32 + 8) continue;
                    for (int rep = 0; e == hipSuccess && rep < 4; ++rep) {
                        e = hipEventRecord(e0, s);
                        if (e == hipSuccess) {
                            if (ci.child >= 0) e = launch_staged(c, d_items, batch, C, A, B, staged_ws, ctx->num_cu, s);
                            else e = launch_batched(c, d_items, batch, C, A, B, ctx->num_cu, s);
                        }
                        if (e == hipSuccess) e = hipEventRecord(e1, s);
                        if (e == hipSuccess) e = hipEventSynchronize(e1);
                        float ms = 0.f;
                        if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
                        if (e == hipSuccess && rep > 0 && (batch_ms[c] < 0 || ms < batch_ms[c])) batch_ms[c] = ms;
                    }
                    if (pass == 0) continue;
                    // latency of one product (item 0) through the entry point's
                    // own path (descriptor, workspace, launches)
                    float lat[10] = {};
                    for (int rep = 0; e == hipSuccess && rep < 10; ++rep) {
                        e = hipEventRecord(e0, s);
                        if (e == hipSuccess && single_product(ctx, C, A, B, n, kKindCyclic, s, c) != GF2X_OK)
                            e = hipErrorLaunchFailure;
                        if (e == hipSuccess) e = hipEventRecord(e1, s);
                        if (e == hipSuccess) e = hipEventSynchronize(e1);
                        if (e == hipSuccess) e = hipEventElapsedTime(&lat[rep], e0, e1);
                    }
                    std::sort(lat + 1, lat + 10);
                    single_ms[c] = lat[5];
                }
            }
            int best = -1, best_direct = -1, best_single = -1;
            auto &log = ctx->tune_log[w32];
            log.clear();
            for (int c = 0; c < kNumClasses; ++c)
                if (batch_ms[c] >= 0) log.emplace_back(c, batch_ms[c], single_ms[c]);
            for (int c = 0; c < kNumClasses; ++c) {
                if (batch_ms[c] >= 0 && (best < 0 || batch_ms[c] < batch_ms[best])) best = c;
                if (batch_ms[c] >= 0 && class_info(c).child < 0 &&
                    (best_direct < 0 || batch_ms[c] < batch_ms[best_direct]))
                    best_direct = c;
                if (single_ms[c] >= 0 && (best_single < 0 || single_ms[c] < single_ms[best_single])) best_single = c;
            }
            if (e == hipSuccess && best >= 0) {
                ctx->cls_of_w32[w32] = best;
                ctx->tuned[w32] = best;
            }
            if (e == hipSuccess && best_direct >= 0) ctx->tuned_direct[w32] = best_direct;
            if (e == hipSuccess && best_single >= 0) ctx->tuned_single[w32] = best_single;
        }
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e == hipSuccess) direct_table(ctx);
        if (e0) hipEventDestroy(e0);
        if (e1) hipEventDestroy(e1);
        if (s) hipStreamDestroy(s);
        hipFree(buf);
        if (e != hipSuccess) return device_error(e);
        const int rc = upload_direct_table(ctx);
        if (rc) return rc;
    }
    if (out_path) {
        FILE *f = std::fopen(out_path, "w");
        if (!f) return GF2X_EINVAL;
        std::fprintf(f,
                     "# gf2x schedule table: <ceil(n/32)> <batch class> <fastest direct class> "
                     "<lowest-latency class of one product>, written by gf2x_tune\n");
        for (auto &kv : ctx->tuned)
            std::fprintf(f, "%u %s %s %s\n", kv.first, class_info(kv.second).name,
                         class_info(ctx->direct_of_w32[kv.first]).name, class_info(ctx->single_of_w32[kv.first]).name);
        // the measurements behind the table, as comments
        std::fprintf(f, "# candidates: <ceil(n/32)> <class> <ms per batch> <us per single product>\n");
        for (auto &kv : ctx->tune_log)
            for (auto &c : kv.second)
                std::fprintf(f, "# %u %s %.4f %.1f\n", kv.first, class_info(std::get<0>(c)).name, std::get<1>(c),
                             1000.0f * std::get<2>(c));
        std::fclose(f);
    }
    return GF2X_OK;
}

int gf2x_schedule_info(gf2x_ctx *ctx, uint32_t n_bits, uint32_t *padded_words32, uint64_t *base_products,
                       uint64_t *lane_ops, char *name, size_t name_len) {
    if (n_bits == 0 || n_bits > kMaxBits) return GF2X_EINVAL;
    const uint32_t w = (n_bits + 31u) / 32u;
    const ClassInfo &ci = class_info(ctx ? ctx->cls_of_w32[w] : default_class(w));
    if (padded_words32) *padded_words32 = (uint32_t)ci.S;
    if (base_products) *base_products = (uint64_t)ci.base;
    if (lane_ops) *lane_ops = (uint64_t)ci.ops;
    if (name && name_len) {
        std::strncpy(name, ci.name, name_len - 1);
        name[name_len - 1] = 0;
    }
    return GF2X_OK;
}

}  // extern "C"
