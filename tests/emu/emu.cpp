// CPU emulation of one workgroup of the library's bit-packed product: runs
// gf2x::one_product<Class> with NT host threads over a heap "LDS" buffer.
// Test infrastructure only (compiled by tests/test_emulation.py).
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#include <vector>

#include "gf2x_product.hpp"
#include "gf2x_sparse_device.hpp"
#include "gf2x_toeplitz_device.hpp"

thread_local EmuIdx threadIdx;

static pthread_barrier_t g_bar;
// lane moves (DPP, ds_bpermute) synchronise the 64 lanes of one wave only
static pthread_barrier_t g_wave_bar[gf2x::NT / 64];
static uint32_t g_xch[gf2x::NT];

void __syncthreads() { pthread_barrier_wait(&g_bar); }

unsigned __shfl_up(unsigned v, int delta, int width) {
    const unsigned t = threadIdx.x;
    g_xch[t] = v;
    pthread_barrier_wait(&g_bar);
    const unsigned lane = t % (unsigned)width;
    const unsigned r = lane >= (unsigned)delta ? g_xch[t - delta] : v;
    pthread_barrier_wait(&g_bar);
    return r;
}

unsigned __shfl_xor(unsigned v, int mask, int width) {
    const unsigned t = threadIdx.x;
    g_xch[t] = v;
    pthread_barrier_wait(&g_bar);
    const unsigned base = t - t % (unsigned)width;
    const unsigned r = g_xch[base + ((t % (unsigned)width) ^ (unsigned)mask)];
    pthread_barrier_wait(&g_bar);
    return r;
}

int emu_ds_bpermute(int addr, int v) {
    const unsigned t = threadIdx.x;
    pthread_barrier_t *bar = &g_wave_bar[t / 64u];
    g_xch[t] = (uint32_t)v;
    pthread_barrier_wait(bar);
    const unsigned base = t - t % 64u;
    const int r = (int)g_xch[base + (((unsigned)addr >> 2) & 63u)];
    pthread_barrier_wait(bar);
    return r;
}

int emu_update_dpp(int old, int v, int ctrl) {
    const unsigned t = threadIdx.x;
    pthread_barrier_t *bar = &g_wave_bar[t / 64u];
    g_xch[t] = (uint32_t)v;
    pthread_barrier_wait(bar);
    const unsigned base = t - t % 64u, l = t % 64u;
    int r = old;
    if (ctrl == 0x13C) r = (int)g_xch[base + ((l + 63u) & 63u)];       // wave_ror:1
    else if (ctrl == 0x134) r = (int)g_xch[base + ((l + 1u) & 63u)];   // wave_rol:1
    pthread_barrier_wait(bar);
    return r;
}

static emu_v4i g_ma[gf2x::NT], g_mb[gf2x::NT];

emu_v4i emu_mfma_i32_16x16x64_i8(emu_v4i a, emu_v4i b, emu_v4i c) {
    const unsigned t = threadIdx.x;
    g_ma[t] = a;
    g_mb[t] = b;
    pthread_barrier_wait(&g_bar);
    const unsigned w = t - t % 64u, l = t % 64u;
    emu_v4i out = c;
    for (int r = 0; r < 4; ++r) {
        const unsigned row = 4 * (l / 16) + r, col = l % 16;
        int sum = 0;
        for (int k = 0; k < 64; ++k) {
            emu_v4i av = g_ma[w + row + 16 * (k / 16)], bv = g_mb[w + col + 16 * (k / 16)];
            const int8_t *ab = reinterpret_cast<const int8_t *>(&av);
            const int8_t *bb = reinterpret_cast<const int8_t *>(&bv);
            sum += (int)ab[k % 16] * (int)bb[k % 16];
        }
        out[r] += sum;
    }
    pthread_barrier_wait(&g_bar);
    return out;
}

namespace {

struct Job {
    int cls;
    const uint64_t *a, *b;
    uint64_t *c;
    uint32_t n, kind;
    uint32_t *smem;
    unsigned tid;
};

void *worker(void *p) {
    Job *j = static_cast<Job *>(p);
    threadIdx.x = j->tid;
    threadIdx.y = threadIdx.z = 0;
    switch (j->cls) {
#define EMU_CASE(id, name, T) \
    case id: gf2x::one_product<gf2x::T>(j->a, j->b, j->c, j->n, j->kind, j->smem); break;
        GF2X_CLASS_LIST(EMU_CASE)
        default: break;
    }
    return nullptr;
}

#define EMU_LDS(id, name, T) gf2x::lds_words<gf2x::T>(),
const int kLds[] = {GF2X_CLASS_LIST(EMU_LDS)};
#define EMU_S(id, name, T) gf2x::T::S,
const int kS[] = {GF2X_CLASS_LIST(EMU_S)};

}  // namespace

extern "C" int emu_num_classes() { return gf2x::kNumClasses; }
extern "C" int emu_class_words(int cls) { return kS[cls]; }

// One product with class `cls`; garbage-fills the LDS stand-in first so that
// a read of never-written scratch shows up as a wrong result.
extern "C" int emu_mul(int cls, const uint64_t *a, const uint64_t *b, uint64_t *c, uint32_t n, uint32_t kind) {
    if (cls < 0 || cls >= gf2x::kNumClasses) return -1;
    std::vector<uint32_t> smem(kLds[cls]);
    uint32_t x = 0x9E3779B9u;
    for (auto &w : smem) w = (x = x * 1664525u + 1013904223u);
    pthread_barrier_init(&g_bar, nullptr, gf2x::NT);
    std::vector<pthread_t> th(gf2x::NT);
    std::vector<Job> jobs(gf2x::NT);
    for (int t = 0; t < gf2x::NT; ++t) {
        jobs[t] = Job{cls, a, b, c, n, kind, smem.data(), (unsigned)t};
        pthread_create(&th[t], nullptr, worker, &jobs[t]);
    }
    for (int t = 0; t < gf2x::NT; ++t) pthread_join(th[t], nullptr);
    pthread_barrier_destroy(&g_bar);
    return 0;
}

// Shared-operand batch through the Toeplitz tiles: h (W words), R (count x W),
// C (count x W) = h * r_i mod (X^n - 1).  Mirrors the host driver's sizing.
namespace {
struct TzJob {
    const uint32_t *hr;
    uint32_t hr_dwords, n, P, count, bx, by;
    const uint64_t *R, *boff;
    uint64_t *C;
    const uint64_t *coff;
    uint32_t *lds;
    unsigned tid;
};
void *tz_worker(void *p) {
    TzJob *j = static_cast<TzJob *>(p);
    threadIdx.x = j->tid;
    gf2x::toeplitz::toeplitz_tile(j->hr, j->hr_dwords, j->n, j->P, j->R, j->boff, j->C, j->coff, j->count, j->bx,
                                  j->by, j->lds);
    return nullptr;
}
}  // namespace

extern "C" int emu_toeplitz(const uint64_t *h, uint32_t n, const uint64_t *R, uint64_t *C, uint32_t count) {
    using namespace gf2x::toeplitz;
    const uint32_t W = (n + 63) / 64;
    const uint32_t steps = (n + kStepBits - 1) / kStepBits;
    const uint32_t rows = (n + kRowsWG - 1) / kRowsWG * kRowsWG;
    const uint32_t P = rows + 64;
    const uint32_t hr_dwords = (P + steps * kStepBits + 128 + 31) / 32 + 2;
    std::vector<uint32_t> hr(hr_dwords);
    for (uint32_t d = 0; d < hr_dwords; ++d) hr[d] = hr_dword(h, n, P, d);
    std::vector<uint64_t> boff(count), coff(count);
    for (uint32_t i = 0; i < count; ++i) boff[i] = coff[i] = (uint64_t)i * W;
    const uint32_t hr_len_max = (kRowsWG + kStepBits * steps + 96 + 64) / 32 + 4;
    const size_t lds_words = ((hr_len_max + 3) & ~3u) + 2 * kTileDwords;
    for (uint32_t bx = 0; bx < rows / kRowsWG; ++bx)
        for (uint32_t by = 0; by < (count + kColsWG - 1) / kColsWG; ++by) {
            std::vector<uint32_t> lds(lds_words, 0xDEADBEEFu);
            pthread_barrier_init(&g_bar, nullptr, gf2x::NT);
            std::vector<pthread_t> th(gf2x::NT);
            std::vector<TzJob> jobs(gf2x::NT);
            for (int t = 0; t < gf2x::NT; ++t) {
                jobs[t] = TzJob{hr.data(), hr_dwords, n, P, count, bx, by, R, boff.data(), C, coff.data(),
                                lds.data(), (unsigned)t};
                pthread_create(&th[t], nullptr, tz_worker, &jobs[t]);
            }
            for (int t = 0; t < gf2x::NT; ++t) pthread_join(th[t], nullptr);
            pthread_barrier_destroy(&g_bar);
        }
    return 0;
}

// Staged class `id` (from the staged list) on one product: evaluation for
// every point word, the NP point products by the child class (emulated
// workgroups, full products), then the interpolation workgroup.
namespace {
struct InterpJob {
    int which;
    gf2x::DevItem it;
    uint64_t *c;
    const uint32_t *products;
    uint32_t *smem;
    unsigned tid;
};
struct EvalJob {
    int which;
    gf2x::DevItem it;
    const uint64_t *a, *b;
    uint32_t *dst;
    uint32_t *smem;
    unsigned tid;
};
void *eval_worker(void *p) {
    EvalJob *j = static_cast<EvalJob *>(p);
    threadIdx.x = j->tid;
    int k = 0;
#define EMU_EVAL_ITEM(id, name, T, cid, C) \
    if (k++ == j->which) gf2x::staged_eval_item<gf2x::T>(j->it, j->a, j->b, j->dst, j->smem);
    GF2X_STAGED_LIST(EMU_EVAL_ITEM)
    return nullptr;
}
void *interp_worker(void *p) {
    InterpJob *j = static_cast<InterpJob *>(p);
    threadIdx.x = j->tid;
    int k = 0;
#define EMU_INTERP(id, name, T, cid, C) \
    if (k++ == j->which) gf2x::staged_interp_item<gf2x::T>(j->it, j->c, j->products, j->smem);
    GF2X_STAGED_LIST(EMU_INTERP)
    return nullptr;
}
}  // namespace

extern "C" int emu_staged(int which, const uint64_t *a, const uint64_t *b, uint64_t *c, uint32_t n, uint32_t kind) {
    int k = 0, S1 = 0, m = 0, np = 0, child = -1, interp_words = 0;
#define EMU_STAGED_INFO(id, name, T, cc, C) \
    if (k++ == which) { S1 = gf2x::T::S1; m = gf2x::T::m; np = gf2x::T::NP; child = cc; interp_words = gf2x::T::INTERP_SCRATCH; }
    GF2X_STAGED_LIST(EMU_STAGED_INFO)
    if (child < 0) return -1;
    (void)m;
    gf2x::DevItem it{n, kind, 0u, 0u, 0, 0, 0};
    std::vector<uint32_t> ws_in(2 * (size_t)np * S1), ws_out(2 * (size_t)np * S1);
    {
        int S = 0;
        k = 0;
#define EMU_STAGED_S2(id, name, T, cc, C) \
        if (k++ == which) S = gf2x::T::S;
        GF2X_STAGED_LIST(EMU_STAGED_S2)
        std::vector<uint32_t> esmem(2 * (size_t)S);
        pthread_barrier_init(&g_bar, nullptr, gf2x::NT);
        std::vector<pthread_t> th(gf2x::NT);
        std::vector<EvalJob> jobs(gf2x::NT);
        for (int t = 0; t < gf2x::NT; ++t) {
            jobs[t] = EvalJob{which, it, a, b, ws_in.data(), esmem.data(), (unsigned)t};
            pthread_create(&th[t], nullptr, eval_worker, &jobs[t]);
        }
        for (int t = 0; t < gf2x::NT; ++t) pthread_join(th[t], nullptr);
        pthread_barrier_destroy(&g_bar);
    }
    for (int e = 0; e < np; ++e) {
        const uint64_t *pa = reinterpret_cast<const uint64_t *>(ws_in.data() + (size_t)e * 2 * S1);
        const uint64_t *pb = pa + S1 / 2;
        uint64_t *pc = reinterpret_cast<uint64_t *>(ws_out.data() + (size_t)e * 2 * S1);
        emu_mul(child, pa, pb, pc, 32u * S1, 1u);
    }
    std::vector<uint32_t> smem(interp_words);
    pthread_barrier_init(&g_bar, nullptr, gf2x::NT);
    std::vector<pthread_t> th(gf2x::NT);
    std::vector<InterpJob> jobs(gf2x::NT);
    for (int t = 0; t < gf2x::NT; ++t) {
        jobs[t] = InterpJob{which, it, c, ws_out.data(), smem.data(), (unsigned)t};
        pthread_create(&th[t], nullptr, interp_worker, &jobs[t]);
    }
    for (int t = 0; t < gf2x::NT; ++t) pthread_join(th[t], nullptr);
    pthread_barrier_destroy(&g_bar);
    return 0;
}

extern "C" int emu_staged_words(int which) {
    int k = 0, S = 0;
#define EMU_STAGED_S(id, name, T, cc, C) \
    if (k++ == which) S = gf2x::T::S;
    GF2X_STAGED_LIST(EMU_STAGED_S)
    return S;
}

// Dense x sparse ring product of one wave (sparse class `which`): a (W(n)
// words) times the w positions, c = W(n) words.
namespace {
struct SparseJob {
    int which, nw;
    const uint64_t *a;
    const uint32_t *pos;
    uint32_t w, n;
    uint64_t *c;
    uint32_t *buf;
    unsigned tid;
};
void *sparse_worker(void *p) {
    SparseJob *j = static_cast<SparseJob *>(p);
    threadIdx.x = j->tid;
    switch (j->which) {
#define EMU_SPARSE(idx, R)                                                                  \
    case idx:                                                                               \
        if (j->nw == 1) gf2x::sparse::product<R, 1>(j->a, j->pos, j->w, j->c, j->n, j->buf); \
        else gf2x::sparse::product<R, 4>(j->a, j->pos, j->w, j->c, j->n, j->buf);            \
        break;
        GF2X_SPARSE_LIST(EMU_SPARSE)
        default: break;
    }
    return nullptr;
}
#define EMU_SPARSE_R(idx, R) R,
const int kSparseR[] = {GF2X_SPARSE_LIST(EMU_SPARSE_R)};
}  // namespace

extern "C" int emu_sparse_words_per_lane(int which) { return kSparseR[which]; }

// nw waves (1 or 4) share the positions of one product.
extern "C" int emu_sparse(int which, int nw, const uint64_t *a, const uint32_t *pos, uint32_t w, uint64_t *c,
                          uint32_t n) {
    if (which < 0 || which >= gf2x::sparse::kSparseClasses || (nw != 1 && nw != 4)) return -1;
    if (64 * kSparseR[which] < 2 * (int)((n + 31) / 32) + 2) return -1;
    std::vector<uint32_t> buf(64 * (size_t)kSparseR[which]);
    uint32_t x = 0x9E3779B9u;
    for (auto &v : buf) v = (x = x * 1664525u + 1013904223u);
    const int threads = 64 * nw;
    pthread_barrier_init(&g_bar, nullptr, threads);
    for (int k = 0; k < nw; ++k) pthread_barrier_init(&g_wave_bar[k], nullptr, 64);
    std::vector<pthread_t> th(threads);
    std::vector<SparseJob> jobs(threads);
    for (int t = 0; t < threads; ++t) {
        jobs[t] = SparseJob{which, nw, a, pos, w, n, c, buf.data(), (unsigned)t};
        pthread_create(&th[t], nullptr, sparse_worker, &jobs[t]);
    }
    for (int t = 0; t < threads; ++t) pthread_join(th[t], nullptr);
    pthread_barrier_destroy(&g_bar);
    for (int k = 0; k < nw; ++k) pthread_barrier_destroy(&g_wave_bar[k]);
    return 0;
}
