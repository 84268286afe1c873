// gf2x_serve.cpp -- continuous batching of ring products with admission by
// an HBM budget (the serving API of include/gf2x.h).
//
// Requests are ring products of any supported n with host operands.  A
// scheduler thread owns K stream slots; each slot has a pinned host buffer
// and a device buffer sized for `max_batch` requests of the largest n.  The
// device buffers together are the HBM budget: a request is admitted only into
// a free slot, so the budget is never exceeded and waiting requests queue on
// the host (or are refused with GF2X_EAGAIN when the host queue is full).
//
// Loop of the scheduler thread:
//   1. retire: every busy slot whose completion event has fired hands its
//      results back (pinned -> caller's buffer) and stamps the completion time;
//   2. launch: if a slot is free and requests whose arrival time has passed
//      are waiting, pack up to max_batch of them (descriptors, a, b) into the
//      slot's pinned buffer, copy to the device, launch the products, copy the
//      results back, record the event.  A batch of at most a few hundred
//      requests runs as three phase kernels whatever sizes it holds (the
//      evaluations of the sizes whose products are spread over workgroups, all
//      one-workgroup products, the interpolations); a larger batch runs one
//      persistent launch per size class, the classes on sub-streams.
// While one slot's batch runs, the next arrivals form the next batch on
// another slot: new requests join while earlier ones are on the GPU, and
// batches on different streams overlap on the device.
//
// Each request carries its scheduled arrival time; it is not admitted before
// it, so an open-loop arrival process can be replayed exactly and latency is
// measured from the scheduled arrival to the completion stamp.
#include <hip/hip_runtime.h>
#include <sys/prctl.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "gf2x.h"
#include "gf2x_copy.hpp"
#include "gf2x_ctx.hpp"
#include "gf2x_internal.hpp"

using namespace gf2x;

namespace {

uint64_t now_ns() {
    return (uint64_t)std::chrono::duration_cast<std::chrono::nanoseconds>(
               std::chrono::steady_clock::now().time_since_epoch())
        .count();
}

struct Request {
    uint32_t n;
    const uint64_t *a, *b;
    uint64_t *c;
    uint64_t arrival_ns;
    uint64_t ticket;
};

constexpr int kSubStreams = 6;  // one per size class present in a batch
// A batch of at most this many requests runs each product in the class with
// the lowest single-product latency (a staged class spreads a product over
// several workgroups); larger batches use the fastest direct classes.  Up to
// a few hundred requests the device is far from full, so spreading products
// shortens the batch; each slot then holds a staged workspace for this many
// requests (about 14 MB at n = 57637).  Where the budget cannot hold that for
// every slot, the limit is halved until it can.
constexpr uint32_t kSmallBatch = 256;
// While batches run, the scheduler checks their completion events this often.
constexpr uint64_t kBusyPollNs = 5000;

struct Slot {
    uint64_t t_admit = 0, t_issued = 0;  // batch admitted, last HIP call of the batch returned
    bool phased = false;
    hipStream_t stream = nullptr;
    hipEvent_t done = nullptr;
    hipStream_t sub[kSubStreams] = {};   // class groups of one batch run side by side
    hipEvent_t fork = nullptr, join[kSubStreams] = {};
    char *host = nullptr;   // pinned: [items | a | b | c]
    char *host_dev = nullptr;  // the device's view of host
    char *dev = nullptr;    // device: same layout
    char *ws = nullptr;     // device workspace of the staged groups of a small batch
    char *ph_host = nullptr, *ph_dev = nullptr;  // descriptors of a phased batch (pinned, device)
    char *ph_host_dev = nullptr;                 // the device's view of ph_host
    std::vector<Request> reqs;
    std::vector<uint64_t> c_off;  // word offset of each request's result in the c region
    size_t c_region = 0;          // byte offset of the c region
    size_t c_bytes = 0;
    bool busy = false;
};

}  // namespace

struct gf2x_srv {
    gf2x_ctx *ctx = nullptr;
    uint32_t max_bits = 0, max_batch = 0, max_pending = 0;
    size_t slot_bytes = 0;
    size_t ws_bytes = 0;  // per slot; 0 when the budget leaves no room
    size_t ph_bytes = 0;  // per slot: descriptors of a phased batch
    uint32_t small_limit = 0;  // batches up to this size use the staged classes
    std::vector<Slot> slots;
    std::mutex mu;
    std::condition_variable cv;
    std::deque<Request> pending;
    // completion stamps of tickets base_ticket, base_ticket + 1, ...; 0 = not
    // done; bit 63 set once the stamp has been returned by gf2x_srv_completion.
    // Returned stamps at the front are dropped, so the window holds only the
    // tickets the caller has not read yet (plus those behind one it has not).
    std::deque<uint64_t> done_ns;
    uint64_t base_ticket = 0;
    std::atomic<uint64_t> completed{0};
    uint64_t next_ticket = 0;
    std::atomic<bool> stop{false};
    std::thread thread;
    int error = GF2X_OK;
    std::string error_text;
    gf2x_srv_stats stats{};
};

namespace {

size_t round_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

// Run f(i) for i in [0, count), split over up to 8 host threads when the
// batch is large enough for the thread start-up to pay off.
template <class F>
void parallel_for(uint32_t count, F f) {
    const uint32_t threads = count >= 512 ? std::min<uint32_t>(8, count / 256) : 1;
    if (threads <= 1) {
        for (uint32_t i = 0; i < count; ++i) f(i);
        return;
    }
    std::vector<std::thread> pool;
    const uint32_t chunk = (count + threads - 1) / threads;
    for (uint32_t t = 0; t < threads; ++t)
        pool.emplace_back([&, t] {
            const uint32_t lo = t * chunk, hi = std::min(count, lo + chunk);
            for (uint32_t i = lo; i < hi; ++i) f(i);
        });
    for (auto &th : pool) th.join();
}

// Retire finished batches; returns the number of requests completed.
size_t retire(gf2x_srv *srv) {
    size_t done = 0;
    for (Slot &sl : srv->slots) {
        if (!sl.busy) continue;
        const hipError_t q = hipEventQuery(sl.done);
        if (q == hipErrorNotReady) continue;
        const uint64_t t = now_ns();
        if (q != hipSuccess) {
            std::lock_guard<std::mutex> lk(srv->mu);
            srv->error = GF2X_EDEVICE;
            srv->error_text = hipGetErrorName(q);
        }
        parallel_for((uint32_t)sl.reqs.size(), [&](uint32_t i) {
            const Request &r = sl.reqs[i];
            const uint64_t W = (r.n + 63u) / 64u;
            std::memcpy(r.c, sl.host + sl.c_region + sl.c_off[i] * 8, W * 8);
        });
        const uint64_t t_out = now_ns();
        {
            std::lock_guard<std::mutex> lk(srv->mu);
            for (const Request &r : sl.reqs) srv->done_ns[r.ticket - srv->base_ticket] = t;
            srv->completed += sl.reqs.size();
            gf2x_srv_stats &st = srv->stats;
            st.host_retire_ns += t_out - t;
            st.host_retire_max_ns = std::max(st.host_retire_max_ns, t_out - t);
            st.device_max_ns = std::max(st.device_max_ns, t - sl.t_issued);
            st.batch_max_ns = std::max(st.batch_max_ns, t_out - sl.t_admit);
        }
        done += sl.reqs.size();
        sl.reqs.clear();
        sl.busy = false;
    }
    if (done) srv->cv.notify_all();
    return done;
}

// Pack the admissible requests into a free slot and launch; returns true if a
// batch was launched.
bool launch(gf2x_srv *srv) {
    Slot *sl = nullptr;
    for (Slot &s : srv->slots)
        if (!s.busy) {
            sl = &s;
            break;
        }
    if (!sl) return false;
    const uint64_t t = now_ns();
    {
        std::lock_guard<std::mutex> lk(srv->mu);
        while (!srv->pending.empty() && sl->reqs.size() < srv->max_batch && srv->pending.front().arrival_ns <= t) {
            sl->reqs.push_back(srv->pending.front());
            srv->pending.pop_front();
        }
    }
    if (sl->reqs.empty()) return false;
    const uint32_t count = (uint32_t)sl->reqs.size();
    // layout: [DevItem x max_batch | a words | b words (right after the batch's
    // a words) | c words]; the regions are sized for max_batch requests of
    // the largest n
    const uint64_t Wmax = (srv->max_bits + 63u) / 64u;
    const size_t items_bytes = round_up((size_t)srv->max_batch * sizeof(DevItem), 256);
    const size_t region = (size_t)srv->max_batch * Wmax * 8;
    const size_t a_at = items_bytes, c_at = a_at + 2 * region;
    sl->c_off.resize(count);
    uint64_t off = 0;
    const bool small = count <= srv->small_limit && srv->ws_bytes > 0;
    std::vector<int> cls_of(count);
    bool phased = true;  // every class the batch needs is held by the phase kernels
    for (uint32_t i = 0; i < count; ++i) {
        const Request &r = sl->reqs[i];
        const uint32_t w32 = (r.n + 31u) / 32u;
        const int cls = small ? srv->ctx->single_of_w32[w32] : srv->ctx->direct_of_w32[w32];
        cls_of[i] = cls;
        const ClassInfo &ci = class_info(cls);
        if (!phase_product_class(ci.child >= 0 ? ci.child : cls)) phased = false;
        sl->c_off[i] = off;
        off += (r.n + 63u) / 64u;
    }
    const size_t b_at = a_at + off * 8;
    parallel_for(count, [&](uint32_t i) {
        const Request &r = sl->reqs[i];
        const uint64_t W = (r.n + 63u) / 64u;
        std::memcpy(sl->host + a_at + sl->c_off[i] * 8, r.a, W * 8);
        std::memcpy(sl->host + b_at + sl->c_off[i] * 8, r.b, W * 8);
    });
    sl->c_region = c_at;
    sl->c_bytes = off * 8;
    uint64_t *dc = reinterpret_cast<uint64_t *>(sl->dev + c_at);
    const uint64_t *da = reinterpret_cast<const uint64_t *>(sl->dev + a_at);
    const uint64_t *db = reinterpret_cast<const uint64_t *>(sl->dev + b_at);
    hipError_t e = hipSuccess;
    uint64_t t_packed = now_ns();
    uint64_t t_copied = 0;
    uint32_t launches = 0;
    if (phased) {
        // three phase kernels: descriptors of the staged items (with their two
        // workspace offsets, in 32-bit words) and of every one-workgroup product
        std::vector<DevItem> st, pr;
        std::vector<uint64_t> wso;
        st.reserve(count);
        wso.reserve(2 * count);
        pr.reserve(8 * (size_t)count);
        uint64_t wsw = 0;
        int eval_lds = 0, prod_lds = 0, interp_lds = 0;
        for (uint32_t i = 0; i < count; ++i) {
            const Request &r = sl->reqs[i];
            const int cls = cls_of[i];
            const ClassInfo &ci = class_info(cls);
            const DevItem it{r.n, kKindCyclic, (uint32_t)cls, 0u, sl->c_off[i], sl->c_off[i], sl->c_off[i]};
            if (ci.child >= 0) {
                const uint64_t S1 = (uint64_t)class_info(ci.child).S, per = 2 * (uint64_t)ci.points * S1;
                const uint64_t in = wsw, out = wsw + per;
                wsw += 2 * per;
                st.push_back(it);
                wso.push_back(in);
                wso.push_back(out);
                for (int e2 = 0; e2 < ci.points; ++e2)
                    pr.push_back(DevItem{(uint32_t)(32 * S1), kKindFull, (uint32_t)ci.child, 1u, in / 2 + e2 * S1,
                                         in / 2 + e2 * S1 + S1 / 2, out / 2 + e2 * S1});
                eval_lds = std::max(eval_lds, phase_eval_lds(cls));
                interp_lds = std::max(interp_lds, phase_interp_lds(cls));
                prod_lds = std::max(prod_lds, class_info(ci.child).lds_bytes);
            } else {
                pr.push_back(it);
                prod_lds = std::max(prod_lds, ci.lds_bytes);
            }
        }
        // the most expensive products first
        std::stable_sort(pr.begin(), pr.end(), [](const DevItem &x, const DevItem &y) {
            return class_info((int)x.cls).ops > class_info((int)y.cls).ops;
        });
        const size_t st_at = 0, wso_at = round_up(st.size() * sizeof(DevItem), 256);
        const size_t pr_at = wso_at + round_up(wso.size() * 8, 256);
        const size_t ph_used = pr_at + pr.size() * sizeof(DevItem);
        // a small batch's descriptors go to the phase region; a larger one has
        // direct classes only (no staged items), in the slot's item region
        char *dh = small ? sl->ph_host : sl->host;
        const char *dh_dev = small ? sl->ph_host_dev : sl->host_dev;
        char *dd = small ? sl->ph_dev : sl->dev;
        const size_t cap = small ? srv->ph_bytes : items_bytes;
        if (ph_used > cap || wsw * 4 > srv->ws_bytes || (!small && !st.empty())) {
            e = hipErrorInvalidValue;  // cannot happen: the regions are sized for these batches
        } else {
            std::memcpy(dh + st_at, st.data(), st.size() * sizeof(DevItem));
            std::memcpy(dh + wso_at, wso.data(), wso.size() * 8);
            std::memcpy(dh + pr_at, pr.data(), pr.size() * sizeof(DevItem));
            t_packed = now_ns();
            const DevItem *d_st = reinterpret_cast<const DevItem *>(dd + st_at);
            const uint64_t *d_wso = reinterpret_cast<const uint64_t *>(dd + wso_at);
            const DevItem *d_pr = reinterpret_cast<const DevItem *>(dd + pr_at);
            const int ncu = srv->ctx->num_cu;
            // descriptors and operands pulled from the pinned buffers by one
            // kernel (no DMA copy call; sizes are multiples of 8 bytes)
            e = launch_pull(reinterpret_cast<const uint64_t *>(dh_dev), reinterpret_cast<uint64_t *>(dd), ph_used / 8,
                            reinterpret_cast<const uint64_t *>(sl->host_dev + a_at),
                            reinterpret_cast<uint64_t *>(sl->dev + a_at), 2 * off, sl->stream);
            t_copied = now_ns();
            if (e == hipSuccess)
                e = launch_phase_eval(d_st, d_wso, (uint32_t)st.size(), eval_lds, da, db,
                                      reinterpret_cast<uint32_t *>(sl->ws), ncu, sl->stream);
            if (e == hipSuccess)
                e = launch_phase_products(d_pr, (uint32_t)pr.size(), prod_lds, dc, da, db,
                                          reinterpret_cast<uint64_t *>(sl->ws), ncu, sl->stream);
            if (e == hipSuccess)
                e = launch_phase_interp(d_st, d_wso, (uint32_t)st.size(), interp_lds, dc,
                                        reinterpret_cast<const uint32_t *>(sl->ws), ncu, sl->stream);
            launches = st.empty() ? 1 : 3;
        }
    } else {
        DevItem *items = reinterpret_cast<DevItem *>(sl->host);
        std::vector<DevItem> tmp(count);
        for (uint32_t i = 0; i < count; ++i)
            tmp[i] = DevItem{sl->reqs[i].n, kKindCyclic, (uint32_t)cls_of[i], 0u, sl->c_off[i], sl->c_off[i],
                             sl->c_off[i]};
        // group by class (largest first) so that each class is one launch
        std::stable_sort(tmp.begin(), tmp.end(), [](const DevItem &x, const DevItem &y) {
            return class_info((int)x.cls).S > class_info((int)y.cls).S ||
                   (class_info((int)x.cls).S == class_info((int)y.cls).S && x.cls < y.cls);
        });
        std::memcpy(items, tmp.data(), count * sizeof(DevItem));
        t_packed = now_ns();
        e = launch_pull(reinterpret_cast<const uint64_t *>(sl->host_dev), reinterpret_cast<uint64_t *>(sl->dev),
                        count * sizeof(DevItem) / 8, reinterpret_cast<const uint64_t *>(sl->host_dev + a_at),
                        reinterpret_cast<uint64_t *>(sl->dev + a_at), 2 * off, sl->stream);
        t_copied = now_ns();
        const DevItem *d_items = reinterpret_cast<const DevItem *>(sl->dev);
        // one launch per class group; with several groups they go to the slot's
        // sub-streams (forked after the copies, joined before the copy back), a
        // single group runs on the slot's stream
        int groups = 0;
        for (uint32_t i = 0; i < count; ++i) groups += (i == 0 || tmp[i].cls != tmp[i - 1].cls);
        const bool fork = groups > 1;
        if (e == hipSuccess && fork) e = hipEventRecord(sl->fork, sl->stream);
        uint32_t first = 0;
        int g = 0;
        char *wp = sl->ws;  // staged groups carve their workspace regions in order
        while (e == hipSuccess && first < count) {
            uint32_t last = first;
            while (last < count && tmp[last].cls == tmp[first].cls) ++last;
            hipStream_t sub = fork ? sl->sub[g % kSubStreams] : sl->stream;
            if (fork && g < kSubStreams) e = hipStreamWaitEvent(sub, sl->fork, 0);
            const int cls = (int)tmp[first].cls;
            if (e == hipSuccess && class_info(cls).child >= 0) {
                e = launch_staged(cls, d_items + first, last - first, dc, da, db, wp, srv->ctx->num_cu, sub);
                wp += round_up(staged_workspace_bytes(cls, last - first), 256);
            } else if (e == hipSuccess) {
                e = launch_batched(cls, d_items + first, last - first, dc, da, db, srv->ctx->num_cu, sub);
            }
            ++launches;
            first = last;
            ++g;
        }
        for (int k = 0; fork && e == hipSuccess && k < std::min(g, kSubStreams); ++k) {
            e = hipEventRecord(sl->join[k], sl->sub[k]);
            if (e == hipSuccess) e = hipStreamWaitEvent(sl->stream, sl->join[k], 0);
        }
    }
    const uint64_t t_launched = now_ns();
    if (e == hipSuccess)
        e = launch_push(reinterpret_cast<const uint64_t *>(sl->dev + c_at),
                        reinterpret_cast<uint64_t *>(sl->host_dev + c_at), off, sl->stream);
    if (e == hipSuccess) e = hipEventRecord(sl->done, sl->stream);
    const uint64_t t_issued = now_ns();
    if (t_copied < t_packed) t_copied = t_packed;  // no copy was issued
    if (e != hipSuccess) {
        std::lock_guard<std::mutex> lk(srv->mu);
        srv->error = GF2X_EDEVICE;
        srv->error_text = hipGetErrorName(e);
    }
    sl->busy = true;
    sl->t_admit = t;
    sl->t_issued = t_issued;
    sl->phased = phased;
    uint32_t busy = 0;
    for (const Slot &s2 : srv->slots) busy += s2.busy;
    std::lock_guard<std::mutex> lk(srv->mu);
    gf2x_srv_stats &st = srv->stats;
    st.batches++;
    st.launches += launches;
    st.phased_batches += phased;
    st.admitted += count;
    if (count > st.max_batch_seen) st.max_batch_seen = count;
    if (busy > st.max_slots_busy) st.max_slots_busy = busy;
    st.host_pack_ns += t_packed - t;
    st.host_pack_max_ns = std::max(st.host_pack_max_ns, t_packed - t);
    st.host_issue_ns += t_issued - t_packed;
    st.host_issue_max_ns = std::max(st.host_issue_max_ns, t_issued - t_packed);
    st.host_issue_copy_max_ns = std::max(st.host_issue_copy_max_ns, t_copied - t_packed);
    st.host_issue_launch_max_ns = std::max(st.host_issue_launch_max_ns, t_launched - t_copied);
    st.host_issue_tail_max_ns = std::max(st.host_issue_tail_max_ns, t_issued - t_launched);
    return true;
}

void scheduler(gf2x_srv *srv) {
    const hipError_t dev = hipSetDevice(srv->ctx->device);
    if (dev != hipSuccess) {
        // nothing can run on this thread: report it (waking any drain) and admit nothing
        {
            std::lock_guard<std::mutex> lk(srv->mu);
            srv->error = GF2X_EDEVICE;
            srv->error_text = hipGetErrorName(dev);
        }
        srv->cv.notify_all();
        return;
    }
    // The idle waits below last 2-20 us.  Linux lets a sleeping thread wake up
    // to its timer slack late (50 us by default), which would delay every
    // admission and every completion stamp by up to that much; 1 ns keeps the
    // wake-ups at the requested times.
    prctl(PR_SET_TIMERSLACK, 1UL, 0UL, 0UL, 0UL);
    while (true) {
        const uint64_t t_iter = now_ns();
        const size_t done = retire(srv);
        const bool launched = launch(srv);
        {
            const uint64_t t_end = now_ns(), busy_ns = t_end - t_iter;
            std::lock_guard<std::mutex> lk(srv->mu);
            if (busy_ns > srv->stats.loop_busy_max_ns) {
                srv->stats.loop_busy_max_ns = busy_ns;
                srv->stats.loop_busy_max_at_ns = t_iter;
            }
        }
        if (srv->stop.load()) {
            bool busy = false;
            for (const Slot &s : srv->slots) busy |= s.busy;
            std::lock_guard<std::mutex> lk(srv->mu);
            if (!busy && srv->pending.empty()) break;
        }
        if (!done && !launched) {
            // idle: wait for the next arrival, a completion or a new submission
            uint64_t wait_ns = 20000;
            {
                std::unique_lock<std::mutex> lk(srv->mu);
                if (!srv->pending.empty()) {
                    const uint64_t t = now_ns(), a = srv->pending.front().arrival_ns;
                    if (a > t) wait_ns = std::min<uint64_t>(wait_ns, a - t);
                }
                bool any_busy = false;
                for (const Slot &s : srv->slots) any_busy |= s.busy;
                if (any_busy) wait_ns = std::min<uint64_t>(wait_ns, kBusyPollNs);
                if (wait_ns > 2000) {
                    const uint64_t t_wait = now_ns();
                    srv->cv.wait_for(lk, std::chrono::nanoseconds(wait_ns));
                    const uint64_t slept = now_ns() - t_wait;
                    if (slept > wait_ns)
                        srv->stats.wake_late_max_ns = std::max(srv->stats.wake_late_max_ns, slept - wait_ns);
                }
            }
        }
    }
}

}  // namespace

extern "C" {

uint64_t gf2x_srv_now_ns(void) { return now_ns(); }

int gf2x_srv_create(gf2x_srv **out, gf2x_ctx *ctx, const gf2x_srv_opts *opts) {
    if (!out || !ctx) return GF2X_EINVAL;
    *out = nullptr;
    gf2x_srv_opts o{};
    if (opts) o = *opts;
    if (o.flags != 0) return GF2X_EINVAL;
    const size_t budget = o.hbm_budget_bytes ? o.hbm_budget_bytes : ((size_t)256 << 20);
    const uint32_t streams = o.streams ? o.streams : 4;
    const uint32_t max_bits = o.max_bits ? o.max_bits : 57637;
    if (streams > 16 || max_bits > kMaxBits) return GF2X_EINVAL;
    const uint64_t Wmax = (max_bits + 63u) / 64u;
    const size_t per_req = sizeof(DevItem) + 3 * Wmax * 8;
    // workspace of the staged groups of a small batch: all of its requests in
    // the staged class with the largest workspace, plus rounding per group.
    // The slots' workspaces together take at most half of the budget.
    auto ws_for = [](uint32_t limit) {
        size_t w = 0;
        for (int c = 0; c < kNumClasses; ++c)
            if (class_info(c).child >= 0) w = std::max(w, staged_workspace_bytes(c, limit));
        return round_up(w + (size_t)kNumClasses * 1024, 256);
    };
    // descriptors of a phased batch: staged items, two workspace offsets each,
    // and up to seven point products per staged item plus the direct items
    auto ph_for = [](uint32_t limit) {
        return round_up((size_t)limit * (sizeof(DevItem) + 16 + 8 * sizeof(DevItem)) + 3 * 256, 256);
    };
    uint32_t small_limit = kSmallBatch;
    while (small_limit > 0 && (ws_for(small_limit) + ph_for(small_limit)) * streams * 2 > budget) small_limit /= 2;
    const size_t ph_bytes = small_limit ? ph_for(small_limit) : 0;
    const size_t ws_bytes = small_limit ? ws_for(small_limit) + ph_bytes : 0;  // phase descriptors counted here
    uint64_t max_batch = (budget - ws_bytes * streams) / streams / per_req;
    if (o.max_batch && o.max_batch < max_batch) max_batch = o.max_batch;
    if (max_batch < 1) return GF2X_ENOMEM;  // the budget cannot hold one request per stream
    gf2x_srv *srv = new (std::nothrow) gf2x_srv();
    if (!srv) return GF2X_ENOMEM;
    srv->ctx = ctx;
    srv->max_bits = max_bits;
    srv->max_batch = (uint32_t)std::min<uint64_t>(max_batch, 1u << 20);
    srv->max_pending = o.max_pending ? o.max_pending : (1u << 22);
    srv->slot_bytes = round_up((size_t)srv->max_batch * sizeof(DevItem), 256) + 3 * (size_t)srv->max_batch * Wmax * 8;
    srv->ws_bytes = ws_bytes ? ws_bytes - ph_bytes : 0;
    srv->ph_bytes = ph_bytes;
    srv->small_limit = small_limit;
    srv->slots.resize(streams);
    hipError_t e = hipSetDevice(ctx->device);
    for (Slot &sl : srv->slots) {
        if (e == hipSuccess) e = hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&sl.done, hipEventDisableTiming);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&sl.fork, hipEventDisableTiming);
        for (int k = 0; k < kSubStreams && e == hipSuccess; ++k) {
            e = hipStreamCreateWithFlags(&sl.sub[k], hipStreamNonBlocking);
            if (e == hipSuccess) e = hipEventCreateWithFlags(&sl.join[k], hipEventDisableTiming);
        }
        // coherent pinned memory: the pull kernel reads it over PCIe on every
        // batch, so no device cache may hold a line of an earlier batch
        const unsigned pin = hipHostMallocMapped | hipHostMallocCoherent;
        if (e == hipSuccess) e = hipHostMalloc(reinterpret_cast<void **>(&sl.host), srv->slot_bytes, pin);
        if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void **>(&sl.dev), srv->slot_bytes);
        if (e == hipSuccess && srv->ws_bytes) e = hipMalloc(reinterpret_cast<void **>(&sl.ws), srv->ws_bytes);
        if (e == hipSuccess && srv->ph_bytes)
            e = hipHostMalloc(reinterpret_cast<void **>(&sl.ph_host), srv->ph_bytes, pin);
        if (e == hipSuccess && srv->ph_bytes) e = hipMalloc(reinterpret_cast<void **>(&sl.ph_dev), srv->ph_bytes);
        if (e == hipSuccess) e = hipHostGetDevicePointer(reinterpret_cast<void **>(&sl.host_dev), sl.host, 0);
        if (e == hipSuccess && srv->ph_bytes)
            e = hipHostGetDevicePointer(reinterpret_cast<void **>(&sl.ph_host_dev), sl.ph_host, 0);
    }
    // Touch every page of the slot buffers once, host pages on the CPU and
    // then once each way from the device, through the same pull kernel and
    // copy back as a batch: the first use of fresh pinned and device pages is
    // slower than later uses and would otherwise land on the requests of the
    // first large batches.
    for (Slot &sl : srv->slots) {
        if (e != hipSuccess) break;
        std::memset(sl.host, 0, srv->slot_bytes);
        if (srv->ph_bytes) std::memset(sl.ph_host, 0, srv->ph_bytes);
        e = launch_pull(reinterpret_cast<const uint64_t *>(sl.host_dev), reinterpret_cast<uint64_t *>(sl.dev),
                        srv->slot_bytes / 8, reinterpret_cast<const uint64_t *>(sl.ph_host_dev),
                        reinterpret_cast<uint64_t *>(sl.ph_dev), srv->ph_bytes / 8, sl.stream);
        if (e == hipSuccess)
            e = launch_push(reinterpret_cast<const uint64_t *>(sl.dev), reinterpret_cast<uint64_t *>(sl.host_dev),
                            srv->slot_bytes / 8, sl.stream);
    }
    for (Slot &sl : srv->slots)
        if (e == hipSuccess) e = hipStreamSynchronize(sl.stream);
    if (e != hipSuccess) {
        gf2x_srv_destroy(srv);
        return e == hipErrorOutOfMemory ? GF2X_ENOMEM : GF2X_EDEVICE;
    }
    srv->stats.max_batch = srv->max_batch;
    srv->stats.hbm_bytes = (srv->slot_bytes + srv->ws_bytes + srv->ph_bytes) * streams;
    srv->thread = std::thread(scheduler, srv);
    *out = srv;
    return GF2X_OK;
}

int gf2x_srv_submit(gf2x_srv *srv, uint32_t count, const uint32_t *n_bits, const uint64_t *a_base,
                    const uint64_t *a_off, const uint64_t *b_base, const uint64_t *b_off, uint64_t *c_base,
                    const uint64_t *c_off, const uint64_t *arrival_ns, uint64_t *first_ticket) {
    if (!srv || !first_ticket || (count && (!n_bits || !a_base || !a_off || !b_base || !b_off || !c_base || !c_off)))
        return GF2X_EINVAL;
    for (uint32_t i = 0; i < count; ++i)
        if (n_bits[i] == 0 || n_bits[i] > srv->max_bits) return GF2X_EINVAL;
    {
        std::lock_guard<std::mutex> lk(srv->mu);
        if (srv->error) return srv->error;
        if (srv->pending.size() + count > srv->max_pending) {
            srv->stats.refused += count;
            return GF2X_EAGAIN;
        }
        *first_ticket = srv->next_ticket;
        const uint64_t t = now_ns();
        srv->done_ns.resize(srv->next_ticket + count - srv->base_ticket, 0);
        for (uint32_t i = 0; i < count; ++i) {
            Request r{n_bits[i], a_base + a_off[i], b_base + b_off[i], c_base + c_off[i],
                      arrival_ns ? arrival_ns[i] : t, srv->next_ticket++};
            srv->pending.push_back(r);
        }
        srv->stats.submitted += count;
    }
    srv->cv.notify_all();
    return GF2X_OK;
}

int gf2x_srv_completion(gf2x_srv *srv, uint64_t first_ticket, uint32_t count, uint64_t *done_ns) {
    if (!srv || (count && !done_ns)) return GF2X_EINVAL;
    constexpr uint64_t kReturned = (uint64_t)1 << 63;
    std::lock_guard<std::mutex> lk(srv->mu);
    if (first_ticket + count > srv->next_ticket) return GF2X_EINVAL;
    for (uint32_t i = 0; i < count; ++i) {
        const uint64_t t = first_ticket + i;
        if (t < srv->base_ticket) {
            done_ns[i] = 1;  // completed and read before; its stamp is no longer kept
            continue;
        }
        uint64_t &v = srv->done_ns[t - srv->base_ticket];
        done_ns[i] = v & ~kReturned;
        if (v) v |= kReturned;
    }
    while (!srv->done_ns.empty() && (srv->done_ns.front() & kReturned)) {
        srv->done_ns.pop_front();
        ++srv->base_ticket;
    }
    return srv->error;
}

int gf2x_srv_drain(gf2x_srv *srv, uint64_t timeout_ms) {
    if (!srv) return GF2X_EINVAL;
    std::unique_lock<std::mutex> lk(srv->mu);
    const bool ok = srv->cv.wait_for(lk, std::chrono::milliseconds(timeout_ms ? timeout_ms : 3600000ull), [&] {
        return srv->error != GF2X_OK || srv->completed.load() == srv->next_ticket;
    });
    if (srv->error) return srv->error;
    return ok ? GF2X_OK : GF2X_EAGAIN;
}

int gf2x_srv_get_stats(gf2x_srv *srv, gf2x_srv_stats *st) {
    if (!srv || !st) return GF2X_EINVAL;
    std::lock_guard<std::mutex> lk(srv->mu);
    *st = srv->stats;
    st->completed = srv->completed.load();
    st->pending = srv->pending.size();
    return GF2X_OK;
}

void gf2x_srv_destroy(gf2x_srv *srv) {
    if (!srv) return;
    if (srv->thread.joinable()) {
        srv->stop = true;
        srv->cv.notify_all();
        srv->thread.join();
    }
    // Teardown returns nothing, so failures here have no one to be reported to.
    for (Slot &sl : srv->slots) {
        if (sl.stream) (void)hipStreamSynchronize(sl.stream);
        if (sl.dev) (void)hipFree(sl.dev);
        if (sl.ws) (void)hipFree(sl.ws);
        if (sl.ph_dev) (void)hipFree(sl.ph_dev);
        if (sl.ph_host) (void)hipHostFree(sl.ph_host);
        if (sl.host) (void)hipHostFree(sl.host);
        if (sl.done) (void)hipEventDestroy(sl.done);
        if (sl.fork) (void)hipEventDestroy(sl.fork);
        for (int k = 0; k < kSubStreams; ++k) {
            if (sl.sub[k]) (void)hipStreamSynchronize(sl.sub[k]);
            if (sl.sub[k]) (void)hipStreamDestroy(sl.sub[k]);
            if (sl.join[k]) (void)hipEventDestroy(sl.join[k]);
        }
        if (sl.stream) (void)hipStreamDestroy(sl.stream);
    }
    delete srv;
}

}  // extern "C"
