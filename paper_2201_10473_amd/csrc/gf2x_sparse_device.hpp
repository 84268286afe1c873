// gf2x_sparse_device.hpp -- ring product of a dense operand a and a sparse
// operand s = X^p_1 + ... + X^p_w in F2[X]/(X^n - 1), in constant time with
// respect to the positions p_t (one wavefront per product).
//
// Section 1 of the paper describes the HQC/BIKE products where one factor
// has a small fixed weight (the "sparse-dense convolution"), and explains
// that a product must not leak its operands through timing; here the
// positions are secret and only n and the weight w are public.
//
// a * s = sum over t of a * X^p_t, and a * X^p is a shifted copy of a.  Each
// shifted copy is built by a barrel whose stage i shifts by 2^i words or not,
// selected by bit i of the word offset: the data movement of every stage is
// the same for every position (a fixed register renaming plus a fixed lane
// rotation), and the secret bit only chooses, through a mask, which of the
// two values a register keeps.  No branch, loop bound, memory or LDS address
// depends on a position.
//
// Layout.  The shifted copy and the accumulator are 64*R 32-bit words held in
// registers across the wave: word j lives in lane j mod 64, register j / 64.
// With 64 R >= 2 ceil(n/32) + 2 every shifted copy fits.  A shift by D < 64
// words is a lane rotation by D (the words of lanes below D move up into the
// next register); a shift by 64 k words renames registers by k.  Only the
// registers that can hold a nonzero word at a stage (a bound that depends
// on the class only) are computed.  The accumulator is kept in the frame
// X^32 * (a * s), i.e. each copy is a * X^(p + 32): then the bit shift of a
// copy is a funnel shift by 32 q - p in [0, 31] with q = ceil(p / 32), and
// the word shift is q <= ceil(n / 32).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace gf2x {
namespace sparse {

typedef uint32_t u32;

constexpr int WAVE = 64;

__device__ __forceinline__ u32 lane_id() { return threadIdx.x & (WAVE - 1); }

// The value v of lane (l - K) mod 64, for every lane l (lanes hold words in
// increasing order, so this moves words K lanes up, cyclically).  K = 1 is
// one DPP move (wave_ror:1); other K a ds_bpermute with a lane address that
// depends on the lane index and K only.
template <int K>
__device__ __forceinline__ u32 lane_rot(u32 v) {
    constexpr int k = ((K % WAVE) + WAVE) % WAVE;
    if constexpr (k == 0) {
        return v;
    } else if constexpr (k == 1) {
        return (u32)__builtin_amdgcn_mov_dpp((int)v, 0x13C, 0xF, 0xF, true);
    } else {
        return (u32)__builtin_amdgcn_ds_bpermute((int)(((lane_id() - (u32)k) & (WAVE - 1)) << 2), (int)v);
    }
}

// m ? x1 : x0 for a mask m of all ones or all zeros (v_bitop3_b32, truth
// table 0xD8 over S0 = x0, S1 = x1, S2 = m).
__device__ __forceinline__ u32 select(u32 m, u32 x1, u32 x0) { return __builtin_amdgcn_bitop3_b32(x0, x1, m, 0xD8); }

// All ones when v >= lim (unsigned), else zero, without a branch.
__device__ __forceinline__ u32 ge_mask(u32 v, u32 lim) { return (u32)0 - (u32)(((uint64_t)v - lim) >> 63 ^ 1u); }

// p mod n for any 32-bit p, without a branch: q = floor(p M / 2^32) with
// M = floor((2^32 - 1) / n) is floor(p / n) or one less, so one masked
// subtraction finishes the reduction.
__device__ __forceinline__ u32 mod_n(u32 p, u32 n, u32 M) {
    const u32 q = (u32)(((uint64_t)p * M) >> 32);
    const u32 r = p - q * n;
    return r - (n & ge_mask(r, n));
}

// Barrel stages 2^i for i = I .. NST-1.  Registers >= LIVE hold zero words
// (a bound fixed by the class); each stage keeps X where its bit of q is zero
// and replaces it by X shifted up by D = 2^i words where the bit is one.
//   D < 64:  word (r, l) takes word (r, l - D) for lanes l >= D and word
//            (r - 1, l - D + 64) below: one lane rotation per register, then a
//            per-lane choice (mask lm[I], public) between a register and the
//            one below it.  The content grows by at most one register.
//   D >= 64: word (r, l) takes word (r - D/64, l): a register renaming.
template <int R, int I, int NST, int LIVE>
__device__ __forceinline__ void barrel(u32 (&X)[R], u32 q, const u32 (&lm)[6]) {
    if constexpr (I < NST) {
        constexpr int D = 1 << I;
        const u32 m = (u32)0 - ((q >> I) & 1u);
        if constexpr (D < WAVE) {
            constexpr int NL = LIVE + 1 < R ? LIVE + 1 : R;
            u32 Z[LIVE];
#pragma unroll
            for (int r = 0; r < LIVE; ++r) Z[r] = lane_rot<D>(X[r]);
#pragma unroll
            for (int r = NL - 1; r >= 0; --r) {
                const u32 zc = r < LIVE ? Z[r] : 0u;
                const u32 zp = r >= 1 ? Z[r - 1] : 0u;  // words wrapping in below lane 0 are zero
                const u32 src = select(lm[I], zc, zp);
                X[r] = r < LIVE ? select(m, src, X[r]) : (src & m);
            }
            barrel<R, I + 1, NST, NL>(X, q, lm);
        } else {
            constexpr int DR = D / WAVE;
            constexpr int NL = LIVE + DR < R ? LIVE + DR : R;
#pragma unroll
            for (int r = NL - 1; r >= 0; --r) {  // descending: X[r - DR] is still the old word
                const u32 src = (r >= DR && r - DR < LIVE) ? X[r - DR] : 0u;
                X[r] = r < LIVE ? select(m, src, X[r]) : (src & m);
            }
            barrel<R, I + 1, NST, NL>(X, q, lm);
        }
    }
}

constexpr int log2_ceil(int v) { return v <= 1 ? 0 : 1 + log2_ceil((v + 1) / 2); }

// Sparse size classes: X(index, R).  A product of n bits runs in the first
// class with 64 R >= 2 ceil(n/32) + 2 (the six ring sizes 12323 ... 57637
// take R = 13, 18, 25, 36, 41, 57); R = 64 holds n <= 65504.
#define GF2X_SPARSE_LIST(X) X(0, 8) X(1, 13) X(2, 18) X(3, 25) X(4, 36) X(5, 41) X(6, 57) X(7, 64)
constexpr int kSparseClasses = 8;
constexpr uint32_t kSparseMaxBits = 65504;

// Words per lane that n bits need: 64 R >= 2 ceil(n/32) + 2.
constexpr int words_per_lane_needed(uint32_t n) { return (int)((2 * ((n + 31) / 32) + 2 + WAVE - 1) / WAVE); }

// One product: c (W(n) uint64 words) = a (W(n) words, bits >= n ignored) *
// sum_t X^(pos[t] mod n) mod (X^n - 1), with w positions (uint32) at pos,
// by NW waves of one workgroup: wave k takes positions k, k + NW, ...; the
// waves' accumulators are XORed together in LDS.  buf: 64R words of LDS.
// Needs 64 R >= 2 ceil(n/32) + 2.
template <int R, int NW>
__device__ __forceinline__ void product(const uint64_t *a64, const u32 *pos, u32 w, uint64_t *c64, u32 n, u32 *buf) {
    constexpr int WORDS = WAVE * R;
    // q <= ceil(n/32) <= 32 R - 1 (since 64 R >= 2 ceil(n/32) + 2)
    constexpr int NST = log2_ceil(32 * R);
    // registers that hold words of a, and of a shifted by at most 32 bits
    // (words 0 .. ceil(n/32) <= 32 R - 1)
    constexpr int RA = (32 * R - 1) / WAVE + 1;
    const u32 l = lane_id();
    const u32 wave = NW > 1 ? (u32)threadIdx.x / WAVE : 0u;
    const int w32 = (int)((n + 31u) / 32u);
    const u32 sn = n % 32u;
    const u32 top = sn ? ((1u << sn) - 1u) : 0xFFFFFFFFu;
    const u32 M = 0xFFFFFFFFu / n;
    const u32 *a32 = reinterpret_cast<const u32 *>(a64);

    // a (masked to n bits, zero above) -> registers, coalesced
    u32 a[RA], ap[RA], acc[R], lm[6];
#pragma unroll
    for (int r = 0; r < RA; ++r) {
        const int j = r * WAVE + (int)l;
        u32 v = 0;
        if (j < w32) v = a32[j] & (j == w32 - 1 ? top : 0xFFFFFFFFu);
        a[r] = v;
    }
    // ap: word j - 1 of a at the place of word j
#pragma unroll
    for (int r = 0; r < RA; ++r) {
        const u32 own = lane_rot<1>(a[r]);
        const u32 below = r >= 1 ? lane_rot<1>(a[r - 1]) : 0u;
        ap[r] = l == 0 ? below : own;
    }
#pragma unroll
    for (int i = 0; i < 6; ++i) lm[i] = l >= (1u << i) ? 0xFFFFFFFFu : 0u;
#pragma unroll
    for (int r = 0; r < R; ++r) acc[r] = 0;

    for (u32 t = wave; t < w; t += NW) {
        const u32 p = mod_n(pos[t], n, M);
        const u32 q = (p + 31u) >> 5;
        const u32 sh = (q << 5) - p;  // a * X^(p + 32) = (a << (32 - sh)) shifted by q words
        u32 X[R];
#pragma unroll
        for (int r = 0; r < RA; ++r) X[r] = __builtin_amdgcn_alignbit(a[r], ap[r], sh);
#pragma unroll
        for (int r = RA; r < R; ++r) X[r] = 0;
        barrel<R, 0, NST, RA>(X, q, lm);
#pragma unroll
        for (int r = 0; r < R; ++r) acc[r] ^= X[r];
    }

    // the waves' accumulators into buf
    if constexpr (NW == 1) {
#pragma unroll
        for (int r = 0; r < R; ++r) buf[r * WAVE + (int)l] = acc[r];
    } else {
        for (int j = (int)threadIdx.x; j < WORDS; j += NW * WAVE) buf[j] = 0;
        __syncthreads();
#pragma unroll
        for (int r = 0; r < R; ++r)
            __hip_atomic_fetch_xor(&buf[r * WAVE + (int)l], acc[r], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    }
    __syncthreads();
    // fold: the product is acc >> 32 (word j of a * s is word j + 1 of acc);
    // bit k + n of it is added to bit k
    const int out32 = 2 * (int)((n + 63u) / 64u);
    const int qn = (int)(n / 32u);
    auto cw = [&](int x) -> u32 { return (x + 1 < WORDS) ? buf[x + 1] : 0u; };
    u32 *c32 = reinterpret_cast<u32 *>(c64);
    for (int k = (int)threadIdx.x; k < out32; k += NW * WAVE) {
        u32 v = 0;
        if (k < w32) {
            v = cw(k) ^ __builtin_amdgcn_alignbit(cw(k + qn + 1), cw(k + qn), sn);
            if (k == w32 - 1) v &= top;
        }
        c32[k] = v;
    }
    __syncthreads();  // buf is reused by the next product
}

}  // namespace sparse
}  // namespace gf2x
