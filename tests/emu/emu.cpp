// CPU emulation of one workgroup of the library's bit-packed product: runs
// gf2x::one_product<Class> with NT host threads over a heap "LDS" buffer.
// Test infrastructure only (compiled by tests/test_emulation.py).
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#include <vector>

#include "gf2x_product.hpp"

thread_local EmuIdx threadIdx;

static pthread_barrier_t g_bar;
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
