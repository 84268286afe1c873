// Driver for the emulation harness under AddressSanitizer and
// UndefinedBehaviorSanitizer (built by tests/test_emulation_asan.py, host
// code only): products of several schedule classes, three staged classes, the
// Toeplitz tile and the sparse barrel, each compared with the C oracle.  The
// LDS stand-in is a heap buffer of the class's exact LDS size, so a kernel
// reading or writing past its LDS shows up as a heap overflow.  Test
// infrastructure only.
#include <stdint.h>
#include <stdio.h>
#include <string.h>

#include <vector>

extern "C" {
int emu_mul(int cls, const uint64_t *a, const uint64_t *b, uint64_t *c, uint32_t n, uint32_t kind);
int emu_class_words(int cls);
int emu_staged(int which, const uint64_t *a, const uint64_t *b, uint64_t *c, uint32_t n, uint32_t kind);
int emu_staged_words(int which);
int emu_toeplitz(const uint64_t *h, uint32_t n, const uint64_t *R, uint64_t *C, uint32_t count);
int emu_sparse(int which, int nw, const uint64_t *a, const uint32_t *pos, uint32_t w, uint64_t *c, uint32_t n);
int emu_sparse_words_per_lane(int which);
int gf2x_ref_mul(uint64_t *c, const uint64_t *a, const uint64_t *b, uint32_t n);
int gf2x_ref_mul_cyclic(uint64_t *r, const uint64_t *a, const uint64_t *b, uint32_t n);
}

static uint64_t state = 0x2201047300000001ull;
static uint64_t next() {  // xorshift64*: test data only
    state ^= state >> 12;
    state ^= state << 25;
    state ^= state >> 27;
    return state * 0x2545F4914F6CDD1Dull;
}

static std::vector<uint64_t> rnd(uint32_t n) {
    std::vector<uint64_t> v((n + 63) / 64);
    for (auto &x : v) x = next();
    if (n % 64) v.back() &= (1ull << (n % 64)) - 1;
    return v;
}

static int fails = 0;
static void check(const char *what, int id, uint32_t n, const std::vector<uint64_t> &got,
                  const std::vector<uint64_t> &want) {
    if (got != want) {
        printf("MISMATCH %s %d n=%u\n", what, id, n);
        ++fails;
    } else {
        printf("ok %s %d n=%u\n", what, id, n);
    }
    fflush(stdout);
}

int main() {
    const int classes[] = {0, 2, 10, 23, 25, 28};
    for (int cls : classes) {
        const uint32_t n = 32u * (uint32_t)emu_class_words(cls) - 37u;
        auto a = rnd(n), b = rnd(n);
        const size_t W = a.size();
        std::vector<uint64_t> c(W), f(2 * W), rc(W), rf(2 * W);
        emu_mul(cls, a.data(), b.data(), c.data(), n, 0);
        emu_mul(cls, a.data(), b.data(), f.data(), n, 1);
        gf2x_ref_mul_cyclic(rc.data(), a.data(), b.data(), n);
        gf2x_ref_mul(rf.data(), a.data(), b.data(), n);
        check("class ring", cls, n, c, rc);
        check("class full", cls, n, f, rf);
    }
    for (int which : {3, 8, 10}) {  // staged Toom-3, Toom-4 and Toom-5 classes
        for (uint32_t cut : {0u, 37u}) {
            const uint32_t n = 32u * (uint32_t)emu_staged_words(which) - cut;
            auto a = rnd(n), b = rnd(n);
            std::vector<uint64_t> c(a.size()), rc(a.size()), f(2 * a.size()), rf(2 * a.size());
            emu_staged(which, a.data(), b.data(), c.data(), n, 0);
            emu_staged(which, a.data(), b.data(), f.data(), n, 1);
            gf2x_ref_mul_cyclic(rc.data(), a.data(), b.data(), n);
            gf2x_ref_mul(rf.data(), a.data(), b.data(), n);
            check("staged ring", which, n, c, rc);
            check("staged full", which, n, f, rf);
        }
    }
    {
        const uint32_t n = 300, count = 9;
        auto h = rnd(n);
        const size_t W = h.size();
        std::vector<uint64_t> R(count * W), C(count * W), want(count * W);
        for (uint32_t i = 0; i < count; ++i) {
            auto r = rnd(n);
            memcpy(&R[i * W], r.data(), W * 8);
            gf2x_ref_mul_cyclic(&want[i * W], h.data(), r.data(), n);
        }
        emu_toeplitz(h.data(), n, R.data(), C.data(), count);
        check("toeplitz", 0, n, C, want);
    }
    for (int nw : {1, 4}) {
        const int which = 1;
        const uint32_t n = 8161, w = 9;
        auto a = rnd(n);
        std::vector<uint32_t> pos(w);
        std::vector<uint64_t> s(a.size(), 0), c(a.size()), want(a.size());
        for (uint32_t t = 0; t < w; ++t) {
            pos[t] = (uint32_t)next();
            const uint32_t p = pos[t] % n;
            s[p / 64] ^= 1ull << (p % 64);
        }
        emu_sparse(which, nw, a.data(), pos.data(), w, c.data(), n);
        gf2x_ref_mul_cyclic(want.data(), a.data(), s.data(), n);
        check("sparse", nw, n, c, want);
    }
    printf("%s\n", fails ? "FAILED" : "ALL OK");
    return fails ? 1 : 0;
}
