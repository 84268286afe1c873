/*
 * gf2x_oracle.c -- plain, slow, obviously correct CPU reference for products
 * in F2[X] and in the ring F2[X]/(X^n - 1).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
 * call this file: only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark use it.  It shares no code, header, table or helper
 * with the GPU library.
 *
 * What it computes (Robert & Veron, "Faster Multiplication over F2[X] using
 * AVX512 instruction set and VPCLMULQDQ instruction"):
 *   - Section 2.1 (KaratRec subsection): operands are binary polynomials of
 *     degree at most N-1, packed into ceil(N/64) 64-bit words; their product
 *     has degree at most 2N-2.  The product is the schoolbook definition
 *     c_k = XOR_{i+j=k} a_i AND b_j, written out word by word.
 *   - Section 1 (the circulant / ring discussion): the protocols need the
 *     product in F2[X]/(X^N - 1).  Since X^N = 1 in that ring, bit k+N of the
 *     full product lands on bit k: r_k = c_k XOR c_{k+N}.  One fold suffices
 *     because deg c <= 2N-2.
 *
 * Packing (the paper fixes the word count, not the bit order; this library
 * uses little-endian order): bit i of a polynomial is bit (i mod 64) of
 * word floor(i/64).  Input bits >= n are ignored (masked on entry); output
 * bits beyond the result's degree bound are written as zero.
 *
 * The 64x64 -> 128 carry-less multiply is the plain shift-and-XOR definition
 * (the function PCLMULQDQ computes, Section 2.2.2): for every set bit k of x,
 * XOR y shifted left by k into the 128-bit accumulator.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define WORDS(n) (((uint64_t)(n) + 63u) / 64u)

/* Mask that keeps the n mod 64 valid bits of the top word (all ones when
 * n is a multiple of 64). */
static uint64_t top_mask(uint32_t n)
{
    uint32_t s = n % 64u;
    return s == 0 ? ~(uint64_t)0 : (((uint64_t)1 << s) - 1u);
}

/* 64x64 -> 128 carry-less product, bit by bit.  The k = 0 step is kept
 * apart because a C shift by 64 is undefined. */
void gf2x_ref_clmul64(uint64_t x, uint64_t y, uint64_t *lo, uint64_t *hi)
{
    uint64_t l = 0, h = 0;
    for (unsigned k = 0; k < 64; ++k) {
        uint64_t m = (uint64_t)0 - ((x >> k) & 1u); /* all ones iff bit k of x */
        l ^= (y << k) & m;
        if (k > 0)
            h ^= (y >> (64u - k)) & m;
    }
    *lo = l;
    *hi = h;
}

/* Full product c = a*b in F2[X].  a, b: W(n) words each; c: 2*W(n) words.
 * Word-level schoolbook: c[i+j] ^= lo(a_i*b_j), c[i+j+1] ^= hi(a_i*b_j).
 * Returns 0, or -1 on a null pointer / n == 0. */
int gf2x_ref_mul(uint64_t *c, const uint64_t *a, const uint64_t *b, uint32_t n)
{
    if (!c || !a || !b || n == 0)
        return -1;
    uint64_t W = WORDS(n);
    uint64_t *x = (uint64_t *)malloc(W * sizeof(uint64_t));
    uint64_t *y = (uint64_t *)malloc(W * sizeof(uint64_t));
    if (!x || !y) {
        free(x);
        free(y);
        return -2;
    }
    memcpy(x, a, W * sizeof(uint64_t));
    memcpy(y, b, W * sizeof(uint64_t));
    x[W - 1] &= top_mask(n);
    y[W - 1] &= top_mask(n);
    memset(c, 0, 2 * W * sizeof(uint64_t));
    for (uint64_t i = 0; i < W; ++i)
        for (uint64_t j = 0; j < W; ++j) {
            uint64_t lo, hi;
            gf2x_ref_clmul64(x[i], y[j], &lo, &hi);
            c[i + j] ^= lo;
            c[i + j + 1] ^= hi;
        }
    free(x);
    free(y);
    return 0;
}

/* Fold a full product (2*W(n) words, degree <= 2n-2) into the ring:
 * r_k = c_k XOR c_{k+n} for 0 <= k < n.  Word k of (c >> n) is a funnel
 * shift of words q+k and q+k+1 of c, q = floor(n/64), s = n mod 64; words
 * at index >= 2W read as zero.  r: W(n) words. */
int gf2x_ref_fold(uint64_t *r, const uint64_t *c, uint32_t n)
{
    if (!r || !c || n == 0)
        return -1;
    uint64_t W = WORDS(n);
    uint64_t q = n / 64u, s = n % 64u;
    for (uint64_t k = 0; k < W; ++k) {
        uint64_t w0 = (k + q < 2 * W) ? c[k + q] : 0;
        uint64_t w1 = (k + q + 1 < 2 * W) ? c[k + q + 1] : 0;
        uint64_t h = (s == 0) ? w0 : ((w0 >> s) | (w1 << (64u - s)));
        r[k] = c[k] ^ h;
    }
    r[W - 1] &= top_mask(n);
    return 0;
}

/* Ring product r = a*b mod (X^n - 1): full product, then fold. */
int gf2x_ref_mul_cyclic(uint64_t *r, const uint64_t *a, const uint64_t *b, uint32_t n)
{
    if (!r || !a || !b || n == 0)
        return -1;
    uint64_t W = WORDS(n);
    uint64_t *c = (uint64_t *)malloc(2 * W * sizeof(uint64_t));
    if (!c)
        return -2;
    int rc = gf2x_ref_mul(c, a, b, n);
    if (rc == 0)
        rc = gf2x_ref_fold(r, c, n);
    free(c);
    return rc;
}

/* Many independent ring products of one size, one after another:
 * item i uses a + i*W, b + i*W and writes r + i*W.  Used to time the
 * oracle on a sample of a batch. */
int gf2x_ref_mul_cyclic_many(uint64_t *r, const uint64_t *a, const uint64_t *b,
                             uint32_t n, uint32_t count)
{
    uint64_t W = WORDS(n);
    for (uint32_t i = 0; i < count; ++i) {
        int rc = gf2x_ref_mul_cyclic(r + (uint64_t)i * W, a + (uint64_t)i * W,
                                     b + (uint64_t)i * W, n);
        if (rc)
            return rc;
    }
    return 0;
}

/* One product of a batch on host memory: operand a at a_base + a_off, b at
 * b_base + b_off, result at c_base + c_off (offsets in 64-bit words).  The
 * kind is 0 (ring product, W(n) result words), 1 (full product, 2 W(n)
 * words) or 2 + (w << 8): b then holds w positions as 32-bit values from
 * that offset, the sparse operand being the sum of X^(p mod n) over them
 * (equal positions cancel), and the result is the ring product with it.
 * The layout is the batch descriptor of the library's interface, restated
 * here so that the two share no header. */
typedef struct {
    uint32_t n_bits;
    uint32_t kind;
    uint64_t a_off, b_off, c_off;
} gf2x_ref_item;

int gf2x_ref_mul_batched(uint64_t *c_base, const uint64_t *a_base, const uint64_t *b_base,
                         const gf2x_ref_item *items, uint32_t count)
{
    if (count && (!c_base || !a_base || !b_base || !items))
        return -1;
    for (uint32_t i = 0; i < count; ++i) {
        const gf2x_ref_item *it = &items[i];
        const uint32_t n = it->n_bits;
        const uint64_t *a = a_base + it->a_off;
        uint64_t *c = c_base + it->c_off;
        int rc;
        if (n == 0)
            return -1;
        if (it->kind == 0u) {
            rc = gf2x_ref_mul_cyclic(c, a, b_base + it->b_off, n);
        } else if (it->kind == 1u) {
            rc = gf2x_ref_mul(c, a, b_base + it->b_off, n);
        } else if ((it->kind & 0xFFu) == 2u) {
            const uint32_t w = it->kind >> 8;
            const uint32_t *pos = (const uint32_t *)(b_base + it->b_off);
            uint64_t *s = (uint64_t *)calloc(WORDS(n), sizeof(uint64_t));
            if (!s)
                return -2;
            for (uint32_t t = 0; t < w; ++t) {
                const uint32_t p = pos[t] % n;
                s[p / 64u] ^= (uint64_t)1 << (p % 64u);
            }
            rc = gf2x_ref_mul_cyclic(c, a, s, n);
            free(s);
        } else {
            return -1;
        }
        if (rc)
            return rc;
    }
    return 0;
}

/* ------------------------------------------------------------- fast mode
 * The same ring products with the 64x64 carry-less multiply done by the
 * CPU's PCLMULQDQ instruction (Section 2.2.2 names it), for timing the
 * CPU side only.  The word schoolbook and the fold are the ones above; the
 * result is identical to gf2x_ref_mul_cyclic_many (the tests check it).
 * Returns -3 when the CPU has no PCLMULQDQ. */
#if defined(__x86_64__)
#include <immintrin.h>

__attribute__((target("pclmul,sse2")))
static void clmul64_pclmul(uint64_t x, uint64_t y, uint64_t out[2])
{
    const __m128i p = _mm_clmulepi64_si128(_mm_set_epi64x(0, (long long)x), _mm_set_epi64x(0, (long long)y), 0x00);
    _mm_storeu_si128((__m128i *)out, p);
}

__attribute__((target("pclmul,sse2")))
static int mul_cyclic_pclmul(uint64_t *r, const uint64_t *a, const uint64_t *b, uint32_t n,
                             uint64_t *x, uint64_t *y, uint64_t *full)
{
    const uint64_t W = WORDS(n);
    memcpy(x, a, W * sizeof(uint64_t));
    memcpy(y, b, W * sizeof(uint64_t));
    x[W - 1] &= top_mask(n);
    y[W - 1] &= top_mask(n);
    memset(full, 0, 2 * W * sizeof(uint64_t));
    for (uint64_t u = 0; u < W; ++u)
        for (uint64_t v = 0; v < W; ++v) {
            uint64_t prod[2];
            clmul64_pclmul(x[u], y[v], prod);
            full[u + v] ^= prod[0];
            full[u + v + 1] ^= prod[1];
        }
    return gf2x_ref_fold(r, full, n);
}

int gf2x_ref_mul_cyclic_many_pclmul(uint64_t *r, const uint64_t *a, const uint64_t *b, uint32_t n, uint32_t count)
{
    if (!__builtin_cpu_supports("pclmul"))
        return -3;
    if (!r || !a || !b || n == 0)
        return -1;
    const uint64_t W = WORDS(n);
    uint64_t *x = (uint64_t *)malloc(W * sizeof(uint64_t));
    uint64_t *y = (uint64_t *)malloc(W * sizeof(uint64_t));
    uint64_t *full = (uint64_t *)malloc(2 * W * sizeof(uint64_t));
    int rc = (x && y && full) ? 0 : -2;
    for (uint32_t i = 0; rc == 0 && i < count; ++i)
        rc = mul_cyclic_pclmul(r + (uint64_t)i * W, a + (uint64_t)i * W, b + (uint64_t)i * W, n, x, y, full);
    free(x);
    free(y);
    free(full);
    return rc;
}
#else
int gf2x_ref_mul_cyclic_many_pclmul(uint64_t *r, const uint64_t *a, const uint64_t *b, uint32_t n, uint32_t count)
{
    (void)r; (void)a; (void)b; (void)n; (void)count;
    return -3;
}
#endif
