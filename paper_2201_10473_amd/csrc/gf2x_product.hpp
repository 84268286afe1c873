// gf2x_product.hpp -- one product per workgroup: staging, the size-class
// table of schedules, and the ring / full epilogues.
//
// One workgroup computes one product: it stages both operands (masked to n
// bits) from HBM into LDS as 32-bit words, runs the compile-time schedule of
// its size class (gf2x_device.hpp), then either folds the 2n-1 bit product
// modulo X^n - 1 in LDS and stores n bits (ring product, Section 1) or stores
// the full product (Section 2.1).  The full product of a ring multiplication
// never reaches HBM.
//
// Size classes: every class is a schedule with a fixed padded operand size
// S (32-bit words); a product of n bits runs in any class with S >= ceil(n/32)
// (zero padding does not change the product).  The host picks the class per
// n from a table (default cost model, or the tuner's measurements).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "gf2x_device.hpp"
#include "gf2x_internal.hpp"

namespace gf2x {

// ------------------------------------------------------------ size classes
using Class0 = ParK2<0, 4>;
using Class1 = ParK2<0, 8>;
using Class2 = ParK2<1, 8>;
using Class3 = ParK2<2, 8>;
using Class4 = ParK2<3, 8>;
using Class5 = ParK2<4, 8>;
using Class6 = ParK2<5, 8>;
using Class7 = ParK2<5, 13>;
using Class8 = SeqT3<ParK2<4, 9>>;
using Class9 = SeqT3<ParK2<5, 5>>;
using Class10 = SeqT3<ParK2<5, 6>>;
using Class11 = SeqT3<ParK2<4, 12>>;
using Class12 = SeqT3<SeqT3<ParK2<5, 3>>>;
using Class13 = SeqT3<ParK2<5, 9>>;
using Class14 = SeqT3<SeqT3<ParK2<5, 4>>>;
using Class15 = SeqT3<SeqT3<ParK2<5, 5>>>;
using Class16 = SeqT3<SeqT3<ParK2<4, 13>>>;
using Class17 = SeqT3<SeqT3<ParK2<5, 7>>>;
using Class18 = SeqT3<SeqT3<ParK2<5, 10>>>;
using Class19 = SeqT3<SeqT3<SeqT3<ParK2<5, 4>>>>;
using Class20 = SeqT3<SeqT3<SeqT3<ParK2<5, 5>>>>;
using Class21 = SeqT3<ParK2<5, 7>>;
using Class22 = SeqT3<ParK2<5, 4>>;
using Class23 = ParK2<5, 6>;
using Class24 = ParK2<5, 9>;
using Class25 = SeqT4<Class24>;
using Class26 = SeqT4<Class9>;
using Class27 = SeqT4<Class22>;
using Class28 = SeqKN<3, Class23>;
using Class29 = SeqKN<3, Class24>;
using Class30 = SeqKN<3, Class9>;
using Class31 = SeqKN<5, Class24>;
using Class32 = SeqKN<5, Class23>;
using Class33 = SeqT3<ParK2<5, 6>, true>;
using Class34 = SeqT3<ParK2<5, 5>, true>;
using Class35 = SeqT3<ParK2<5, 9>, true>;
using Class36 = SeqT4<Class24, true>;
using Class37 = SeqT4<Class9, true>;
using Class38 = SeqT4<Class22, true>;
using Class39 = SeqT3<Class9, true>;
using Class40 = SeqT3<Class22, true>;
// top levels that exist only as staged classes
using Top4Class9 = TopT4<Class9>;
using Top4Class22 = TopT4<Class22>;
using Top4Class24 = TopT4<Class24>;
using Top5Class22 = TopT5<Class22>;
using Top5Class24 = TopT5<Class24>;

// X(id, name, schedule type)
#define GF2X_CLASS_LIST(X) \
    X(0, "U4", Class0) \
    X(1, "U8", Class1) \
    X(2, "K2^1.U8", Class2) \
    X(3, "K2^2.U8", Class3) \
    X(4, "K2^3.U8", Class4) \
    X(5, "K2^4.U8", Class5) \
    X(6, "K2^5.U8", Class6) \
    X(7, "K2^5.U13", Class7) \
    X(8, "T3.K2^4.U9", Class8) \
    X(9, "T3.K2^5.U5", Class9) \
    X(10, "T3.K2^5.U6", Class10) \
    X(11, "T3.K2^4.U12", Class11) \
    X(12, "T3.T3.K2^5.U3", Class12) \
    X(13, "T3.K2^5.U9", Class13) \
    X(14, "T3.T3.K2^5.U4", Class14) \
    X(15, "T3.T3.K2^5.U5", Class15) \
    X(16, "T3.T3.K2^4.U13", Class16) \
    X(17, "T3.T3.K2^5.U7", Class17) \
    X(18, "T3.T3.K2^5.U10", Class18) \
    X(19, "T3.T3.T3.K2^5.U4", Class19) \
    X(20, "T3.T3.T3.K2^5.U5", Class20) \
    X(21, "T3.K2^5.U7", Class21) \
    X(22, "T3.K2^5.U4", Class22) \
    X(23, "K2^5.U6", Class23) \
    X(24, "K2^5.U9", Class24) \
    X(25, "T4.K2^5.U9", Class25) \
    X(26, "T4.T3.K2^5.U5", Class26) \
    X(27, "T4.T3.K2^5.U4", Class27) \
    X(28, "K3.K2^5.U6", Class28) \
    X(29, "K3.K2^5.U9", Class29) \
    X(30, "K3.T3.K2^5.U5", Class30) \
    X(31, "K5.K2^5.U9", Class31) \
    X(32, "K5.K2^5.U6", Class32) \
    X(33, "T3m.K2^5.U6", Class33) \
    X(34, "T3m.K2^5.U5", Class34) \
    X(35, "T3m.K2^5.U9", Class35) \
    X(36, "T4m.K2^5.U9", Class36) \
    X(37, "T4m.T3.K2^5.U5", Class37) \
    X(38, "T4m.T3.K2^5.U4", Class38) \
    X(39, "T3m.T3.K2^5.U5", Class39) \
    X(40, "T3m.T3.K2^5.U4", Class40)

// Staged classes: the top Toom-3 (5 points) or Toom-4 (7 points) level of a
// class is spread over workgroups.  An evaluation kernel writes the point
// operands of every product to a workspace, the child class computes all of
// them as one batch of full products, and an interpolation kernel recombines
// and folds.
// X(id, name, top schedule type, child class id, child schedule type)
#define GF2X_STAGED_LIST(X) \
    X(41, "G.T3.T3.K2^5.U4", Class14, 22, Class22) \
    X(42, "G.T3.T3.K2^5.U5", Class15, 9, Class9) \
    X(43, "G.T3.T3.K2^5.U7", Class17, 21, Class21) \
    X(44, "G.T3.K2^5.U6", Class10, 23, Class23) \
    X(45, "G.T3.K2^5.U9", Class13, 24, Class24) \
    X(46, "G.T3.T3.T3.K2^5.U5", Class20, 15, Class15) \
    X(47, "G.T4.T3.K2^5.U5", Top4Class9, 9, Class9) \
    X(48, "G.T4.T3.K2^5.U4", Top4Class22, 22, Class22) \
    X(49, "G.T4.K2^5.U9", Top4Class24, 24, Class24) \
    X(50, "G.T5.T3.K2^5.U4", Top5Class22, 22, Class22) \
    X(51, "G.T5.K2^5.U9", Top5Class24, 24, Class24)

#define GF2X_COUNT_CLASS(id, name, T) +1
constexpr int NUM_CLASSES = 0 GF2X_CLASS_LIST(GF2X_COUNT_CLASS);
#define GF2X_COUNT_STAGED(id, name, T, c, C) +1
constexpr int NUM_STAGED = 0 GF2X_STAGED_LIST(GF2X_COUNT_STAGED);
static_assert(NUM_CLASSES == kNumDirect && NUM_CLASSES + NUM_STAGED == kNumClasses, "class count mismatch");

template <class Sch>
constexpr int lds_words() { return (Sch::FROM_MEM ? 0 : 2 * Sch::S) + Sch::SCRATCH; }

// Workgroups of a class that fit in one CU's 160 KB of LDS; with 4 waves per
// workgroup this is also the number of waves per SIMD the register
// allocation should leave room for (at most 8).
template <class Sch>
constexpr int waves_per_simd() {
    const int wg = (160 * 1024) / (lds_words<Sch>() * 4);
    return wg < 1 ? 1 : (wg > 8 ? 8 : wg);
}

#define GF2X_CHECK_LDS(id, name, T) \
    static_assert(lds_words<T>() * 4 <= 160 * 1024, "class " name " exceeds LDS");
GF2X_CLASS_LIST(GF2X_CHECK_LDS)

// --------------------------------------------------------- one product
__device__ __forceinline__ u32 load_word32(const uint64_t *src, int k) {
    return reinterpret_cast<const u32 *>(src)[k];
}

// Stage a and b (n bits each) into [A | B] as S zero-padded 32-bit words.
template <int S>
__device__ __forceinline__ void stage(const uint64_t *a, const uint64_t *b, u32 n, u32 *smem) {
    const int w32 = (int)((n + 31u) / 32u);
    const u32 s = n % 32u;
    const u32 top = s ? ((1u << s) - 1u) : 0xFFFFFFFFu;
    auto word = [&](const uint64_t *src, int k) -> u32 {
        if (k >= w32) return 0u;
        const u32 x = load_word32(src, k);
        return k == w32 - 1 ? (x & top) : x;
    };
    par_map<2 * S>(smem, [&](int idx) -> u32 { return idx < S ? word(a, idx) : word(b, idx - S); });
}

// Ring product epilogue: out32[k] = R[k] ^ (R >> n)[k] for k < ceil(n/32),
// zero for the remaining 32-bit halves of the W(n) output words.
template <int S>
__device__ __forceinline__ void store_cyclic(const u32 *R, u32 n, uint64_t *c) {
    const int w32 = (int)((n + 31u) / 32u);
    const int out32 = 2 * (int)((n + 63u) / 64u);
    const int q = (int)(n / 32u);
    const u32 s = n % 32u;
    const u32 top = s ? ((1u << s) - 1u) : 0xFFFFFFFFu;
    u32 *c32 = reinterpret_cast<u32 *>(c);
    for (int k = tid(); k < out32; k += NT) {
        u32 v = 0;
        if (k < w32) {
            const int i0 = k + q, i1 = k + q + 1;
            const u32 lo = i0 < 2 * S ? R[i0] : 0u;
            const u32 hi = i1 < 2 * S ? R[i1] : 0u;
            v = R[k] ^ funnel(hi, lo, s);
            if (k == w32 - 1) v &= top;
        }
        c32[k] = v;
    }
}

// Full product epilogue: 2*W(n) output words; R holds 2S words and every
// bit at or above 2n-1 is zero.
template <int S>
__device__ __forceinline__ void store_full(const u32 *R, u32 n, uint64_t *c) {
    const int out32 = 4 * (int)((n + 63u) / 64u);
    u32 *c32 = reinterpret_cast<u32 *>(c);
    for (int k = tid(); k < out32; k += NT) c32[k] = k < 2 * S ? R[k] : 0u;
}

// Staged top level (Toom-3 or Toom-4), evaluation of one item by one
// workgroup: both operands are staged in LDS (masked to n bits, zero padded
// to S words, smem holds 2S words), then the NP point operand pairs are
// written to dst as ((e * 2 + x) * S1 + w), coalesced.
template <class Top>
__device__ __forceinline__ void staged_eval_item(const DevItem &it, const uint64_t *a_base, const uint64_t *b_base,
                                                 u32 *dst, u32 *smem) {
    constexpr int S1 = Top::S1, m = Top::m, S = Top::S;
    stage<S>(a_base + it.a_off, b_base + it.b_off, it.n, smem);
    __syncthreads();
    auto part = [&](int x, int p, int j) -> u32 { return (j >= 0 && j < m) ? smem[x * S + p * m + j] : 0u; };
    // one point at a time, so that each point's combination of parts is fixed
    // at compile time; point e's pair occupies dst[2 e S1, 2 (e + 1) S1)
#pragma unroll
    for (int e = 0; e < Top::NP; ++e) {
        for (int r = tid(); r < 2 * S1; r += NT) {
            const int x = r >= S1 ? 1 : 0;
            dst[e * 2 * S1 + r] = Top::point_word(e, x, r - x * S1, part);
        }
    }
    __syncthreads();  // smem is reused by the next item
}

// Staged top level, interpolation of one item from its NP point products
// (2*S1 words each, consecutive), then the ring fold or the full store.
template <class Top>
__device__ __forceinline__ void staged_interp_item(const DevItem &it, uint64_t *c_base, const u32 *products,
                                                   u32 *smem) {
    if constexpr (Top::INTERP_STORES) {
        Top::interp_store(products, smem, it.n, it.kind, c_base + it.c_off);
    } else {
        const u32 *R = Top::interp_from(products, smem);
        if (it.kind == kKindCyclic) store_cyclic<Top::S>(R, it.n, c_base + it.c_off);
        else store_full<Top::S>(R, it.n, c_base + it.c_off);
        __syncthreads();
    }
}

template <class Sch>
__device__ __forceinline__ void one_product(const uint64_t *a, const uint64_t *b, uint64_t *c, u32 n,
                                            u32 kind, u32 *smem) {
    constexpr int S = Sch::S;
    const u32 *R;
    if constexpr (Sch::FROM_MEM) {
        R = Sch::run_mem(reinterpret_cast<const u32 *>(a), reinterpret_cast<const u32 *>(b), n, smem);
    } else {
        stage<S>(a, b, n, smem);
        __syncthreads();
        R = Sch::run_ab(smem, smem + 2 * S);
    }
    if (kind == kKindCyclic) store_cyclic<S>(R, n, c);
    else store_full<S>(R, n, c);
    __syncthreads();  // LDS is reused by the next product of a persistent loop
}

}  // namespace gf2x
