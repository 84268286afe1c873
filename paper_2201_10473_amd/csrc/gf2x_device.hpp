// gf2x_device.hpp -- device-side building blocks of the bit-packed product
// in F2[X] on gfx950 (MI355X).
//
// Words are 32 bits on the device (the VALU word); a polynomial of S words
// holds coefficient i in bit (i mod 32) of word floor(i/32).  One workgroup
// of NT threads computes one product with every operand, partial product
// and accumulator resident in LDS.
//
// The recursion is a compile-time schedule built from three pieces:
//   * unit_mul<T>      -- T x T word schoolbook product held in one thread's
//                         registers (the base case).
//   * ParK2<D, T>      -- D levels of 2-way Karatsuba (Appendix A, KaratRec),
//                         executed breadth first: all 3^D base products of a
//                         level run at once, one per thread.
//   * SeqT3<Child>     -- word-aligned Toom-Cook 3 (Appendix D, Section 3.2)
//                         with w = 32, whose five point products are computed
//                         one after another by Child (saves LDS).
//
// Constant time: every loop bound, branch and LDS/global address depends
// only on the compile-time schedule, the thread index and the public n --
// never on operand bits.  Bits of an operand only ever reach the datapath
// as data (masks built by bit-field extraction, XOR/AND), never as control.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace gf2x {

typedef uint32_t u32;

constexpr int NT = 256;      // threads per workgroup
constexpr int NWAVE = NT / 64;

constexpr long long pow3(int d) { return d == 0 ? 1 : 3 * pow3(d - 1); }

// acc ^ (x & m) in one gfx950 v_bitop3_b32 (truth table 0x78 over
// S0 = acc -> 0xF0, S1 = x -> 0xCC, S2 = m -> 0xAA).
__device__ __forceinline__ u32 xor_and(u32 acc, u32 x, u32 m) {
    return __builtin_amdgcn_bitop3_b32(acc, x, m, 0x78);
}

// All ones when bit j of a is set, else zero (v_bfe_i32 a, j, 1).
__device__ __forceinline__ u32 bit_mask(u32 a, u32 j) {
    return (u32)__builtin_amdgcn_sbfe((int)a, (int)j, 1);
}

// Low word of the 64-bit value {hi, lo} shifted right by s (0 <= s < 32).
__device__ __forceinline__ u32 funnel(u32 hi, u32 lo, u32 s) {
    return __builtin_amdgcn_alignbit(hi, lo, s);
}

// dst[idx] = f(idx) for 0 <= idx < TOTAL, spread over the workgroup.  Each
// thread computes all of its values before it stores any, so its loads are
// issued back to back and the pass costs one memory round trip, not one per
// element.  f may read dst only at its own idx.
template <int TOTAL, class F>
__device__ __forceinline__ void par_map(u32 *dst, F f) {
    constexpr int IT = (TOTAL + NT - 1) / NT;
    u32 v[IT];
#pragma unroll
    for (int i = 0; i < IT; ++i) {
        const int idx = threadIdx.x + i * NT;
        if (IT * NT == TOTAL || idx < TOTAL) v[i] = f(idx);
    }
#pragma unroll
    for (int i = 0; i < IT; ++i) {
        const int idx = threadIdx.x + i * NT;
        if (IT * NT == TOTAL || idx < TOTAL) dst[idx] = v[i];
    }
}

// ------------------------------------------------------------------ base case
// c (2T words) = a (T words) * b (T words) in F2[X], all in registers.
//
// The carry-less product is sum over bits j of a_i of (b << j) placed at word
// i.  For each bit position j the whole T-word b is shifted left by j once
// ((T+1) funnel shifts, shared by every a_i), and then for every word a_i the
// shifted b is XORed into c at word offset i under the mask "bit j of a_i is
// set": (T+1) v_bitop3 per (i, j).  Each v_bitop3 therefore retires 32
// bit-pair products, and the low and high halves of the 32x32 products merge
// into one accumulator word instead of two.
template <int T>
struct Unit {
    // VALU lane-ops of one call: j = 0 uses T bfe + T*T bitop3; each of the
    // other 31 bit positions uses (T+1) shifts + T bfe + T*(T+1) bitop3.
    static constexpr long long OPS = (long long)T * T + T + 31LL * (T * T + 3 * T + 1);
};

template <int T>
__device__ __forceinline__ void unit_mul(const u32 (&a)[T], const u32 (&b)[T], u32 (&c)[2 * T]) {
#pragma unroll
    for (int k = 0; k < 2 * T; ++k) c[k] = 0;
#pragma unroll
    for (int i = 0; i < T; ++i) {
        const u32 m = bit_mask(a[i], 0);
#pragma unroll
        for (int u = 0; u < T; ++u) c[i + u] = xor_and(c[i + u], b[u], m);
    }
#pragma unroll 1
    for (u32 j = 1; j < 32; ++j) {
        const u32 r = 32u - j;
        u32 sh[T + 1];
        sh[0] = b[0] << j;
#pragma unroll
        for (int u = 1; u < T; ++u) sh[u] = funnel(b[u], b[u - 1], r);
        sh[T] = b[T - 1] >> r;
#pragma unroll
        for (int i = 0; i < T; ++i) {
            const u32 m = bit_mask(a[i], j);
#pragma unroll
            for (int u = 0; u <= T; ++u) c[i + u] = xor_and(c[i + u], sh[u], m);
        }
    }
}

// One thread per unit: unit u's operands [a_u | b_u] (2T words) sit at
// P + 2T*u; its 2T-word product overwrites them.
template <int T, int UNITS>
__device__ __forceinline__ void run_units(u32 *P) {
    for (int u = threadIdx.x; u < UNITS; u += NT) {
        u32 *p = P + 2 * T * u;
        u32 a[T], b[T], c[2 * T];
#pragma unroll
        for (int k = 0; k < T; ++k) {
            a[k] = p[k];
            b[k] = p[T + k];
        }
        unit_mul<T>(a, b, c);
#pragma unroll
        for (int k = 0; k < 2 * T; ++k) p[k] = c[k];
    }
}

// ----------------------------------------------------- 2-way Karatsuba levels
// Splitting (KaratRec, Appendix A): a node of SL words with operands [a | b]
// becomes three children of H = SL/2 words, in this order:
//   child 0: (a0, b0), child 1: (a1, b1), child 2: (a0 + a1, b0 + b1).
// Every level is stored densely: node v's operands at v*2*SL.
template <int NL, int SL>
__device__ __forceinline__ void k2_split(const u32 *src, u32 *dst) {
    constexpr int H = SL / 2;
    constexpr int TOTAL = NL * 2 * H;
    for (int idx = threadIdx.x; idx < TOTAL; idx += NT) {
        const int v = idx / (2 * H);
        const int r = idx - v * 2 * H;  // r = x*H + w, x = which operand
        const int x = r / H;
        const int w = r - x * H;
        const u32 lo = src[v * 2 * SL + x * SL + w];
        const u32 hi = src[v * 2 * SL + x * SL + H + w];
        u32 *d = dst + 3 * v * 2 * H + r;
        d[0] = lo;
        d[2 * H] = hi;
        d[4 * H] = lo ^ hi;
    }
}

// Reconstruction (KaratRec): R = R0 + (R0 + R1 + R2) X^{32H} + R1 X^{64H}
// with children products R_k of 2H words stored densely; since R0 and R1 are
// adjacent, [R0 | R1] already is R0 + R1 X^{64H}.  Parent products are 4H
// words, stored densely.
template <int NL, int H>
__device__ __forceinline__ void k2_merge(const u32 *src, u32 *dst) {
    constexpr int TOTAL = NL * 4 * H;
    for (int idx = threadIdx.x; idx < TOTAL; idx += NT) {
        const int v = idx / (4 * H);
        const int k = idx - v * 4 * H;
        const u32 *R = src + 3 * v * 2 * H;
        u32 val = R[k];
        if (k >= H && k < 3 * H) {
            const int j = k - H;
            val ^= R[j] ^ R[j + 2 * H] ^ R[j + 4 * H];
        }
        dst[idx] = val;
    }
}

// D levels of 2-way Karatsuba over T-word units, breadth first.
//   S       = T * 2^D operand words; the product has 2S words.
//   scratch = [P (units: 2T * 3^D words) | DA (4T * 3^(D-1) words)].
// Down pass: level D-1 lands in DA, level D-2 in P, alternating backwards,
// and the units in P.  Up pass: alternates P -> DA -> P ...  Every buffer
// a level is written to is dead at that point (see the alternation).
template <int D, int T>
struct ParK2 {
    static constexpr int S = T << D;
    static constexpr long long UNITS = pow3(D);
    static constexpr int P_WORDS = (int)(2 * T * UNITS);
    static constexpr int DA_WORDS = D > 0 ? (int)(4 * T * pow3(D - 1)) : 0;
    static constexpr int SCRATCH = P_WORDS + DA_WORDS;
    static constexpr long long BASE = UNITS * T * T;   // 32x32 word products
    // XOR lane-ops of one level of size SL over NL nodes: split SL, merge 3*SL.
    static constexpr long long xor_ops(int l) {
        return l >= D ? 0 : pow3(l) * 4LL * (T << (D - l)) + xor_ops(l + 1);
    }
    static constexpr long long OPS = UNITS * Unit<T>::OPS + xor_ops(0);

    template <int L>
    __device__ static u32 *down_dst(u32 *P, u32 *DA) {
        // destination of level L (1 <= L <= D)
        if constexpr (L == D) return P;
        else return ((D - 1 - L) % 2 == 0) ? DA : P;
    }

    template <int L>
    __device__ static void down(const u32 *src, u32 *P, u32 *DA) {
        constexpr int SL = T << (D - L);
        u32 *dst = down_dst<L + 1>(P, DA);
        k2_split<(int)pow3(L), SL>(src, dst);
        __syncthreads();
        if constexpr (L + 1 < D) down<L + 1>(dst, P, DA);
    }

    template <int L>
    __device__ static u32 *up(const u32 *src, u32 *P, u32 *DA) {
        constexpr int H = T << (D - L - 1);
        u32 *dst = ((D - L) % 2) ? DA : P;
        k2_merge<(int)pow3(L), H>(src, dst);
        __syncthreads();
        if constexpr (L > 0) return up<L - 1>(dst, P, DA);
        else return dst;
    }

    // in: [a (S) | b (S)]; returns the 2S-word product (inside scratch).
    __device__ static u32 *run(const u32 *in, u32 *scratch) {
        u32 *P = scratch;
        u32 *DA = scratch + P_WORDS;
        if constexpr (D == 0) {
            for (int k = threadIdx.x; k < 2 * T; k += NT) P[k] = in[k];
            __syncthreads();
            run_units<T, 1>(P);
            __syncthreads();
            return P;
        } else {
            down<0>(in, P, DA);
            run_units<T, (int)UNITS>(P);
            __syncthreads();
            return up<D - 1>(P, P, DA);
        }
    }
};

// --------------------------------------------------------- workgroup scans
// x[k] <- XOR of x[1..k+1] and y[k] <- XOR of y[1..k+1] for 0 <= k < L:
// division by x (drop the low word, which exact division leaves zero) then by
// x + 1 (multiplication by sum_i x^i, i.e. a prefix XOR over w-bit blocks,
// Section 3.2) in one pass.  tmp: 2*NWAVE words.  Ends with a barrier.
template <int L>
__device__ __forceinline__ void div_xx1_pair(u32 *x, u32 *y, u32 *tmp) {
    constexpr int C = (L + NT - 1) / NT;
    const int t = threadIdx.x;
    u32 vx[C], vy[C];
    u32 ax = 0, ay = 0;
#pragma unroll
    for (int i = 0; i < C; ++i) {
        const int k = t * C + i;
        ax ^= (k < L) ? x[k + 1] : 0u;
        ay ^= (k < L) ? y[k + 1] : 0u;
        vx[i] = ax;
        vy[i] = ay;
    }
    const u32 tx = ax, ty = ay;
    const int lane = t & 63;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const u32 ox = __shfl_up(ax, d, 64);
        const u32 oy = __shfl_up(ay, d, 64);
        if (lane >= d) {
            ax ^= ox;
            ay ^= oy;
        }
    }
    const int wave = t >> 6;
    if (lane == 63) {
        tmp[wave] = ax;
        tmp[NWAVE + wave] = ay;
    }
    __syncthreads();
    u32 px = ax ^ tx, py = ay ^ ty;  // exclusive prefix within the wave
    for (int w = 0; w < wave; ++w) {
        px ^= tmp[w];
        py ^= tmp[NWAVE + w];
    }
#pragma unroll
    for (int i = 0; i < C; ++i) {
        const int k = t * C + i;
        if (k < L) {
            x[k] = px ^ vx[i];
            y[k] = py ^ vy[i];
        }
    }
    __syncthreads();
}

// ------------------------------------------------------------- Toom-Cook 3
// Word-aligned Toom-Cook 3 (Appendix D) with x = X^32.  Operands of S = 3m
// words split as a = a0 + a1 Y + a2 Y^2, Y = X^{32m}.  The five point
// products C(0), C(1), C(x), C(x+1), C(inf) have operands of at most m + 2
// words, so the child size is S1 = m + 2 (the sizing rule of Section 3.2:
// the split is two words smaller than the elementary product).
//
// Interpolation, regrouped over the common denominator x(x+1) so that every
// intermediate is a polynomial (the individual terms of the paper's inverse
// matrix are not):
//   c0 = C(0), c4 = C(inf)
//   c3 = (C(0) + C(1) + C(x) + C(x+1)) / (x^2 + x)
//   c2 = (C(1) + x C(x) + (x+1) C(x+1) + (x^4 + x) c4) / (x^2 + x)
//   c1 = C(1) + c0 + c2 + c3 + c4
// and the result c0 + c1 Y + ... + c4 Y^4 is accumulated directly:
//   R = c0 (1 + Y) + C(1) Y + c2 (Y + Y^2) + c3 (Y + Y^3) + c4 (Y + Y^4).
// Each point product is folded into R and into the two numerators as soon as
// it is computed, so only one child product is alive at a time.
template <class Child>
struct SeqT3 {
    static constexpr int S1 = Child::S;
    static constexpr int m = S1 - 2;
    static constexpr int S = 3 * m;
    static constexpr int R_WORDS = 6 * m;
    static constexpr int SA_WORDS = 2 * S1 + 2;
    static constexpr int UA_WORDS = 2 * S1 + 2;
    static constexpr int CIN_WORDS = 2 * S1;
    static constexpr int TMP_WORDS = 2 * NWAVE;
    static constexpr int SCRATCH = R_WORDS + SA_WORDS + UA_WORDS + CIN_WORDS + TMP_WORDS + Child::SCRATCH;
    static constexpr long long BASE = 5 * Child::BASE;
    // evaluation 16*S1, absorption 30*S1, divisions 4m, recombination 8m
    static constexpr long long OPS = 5 * Child::OPS + 46LL * S1 + 12LL * m;

    // Operands of point e (0: 0, 1: 1, 2: x, 3: x+1, 4: inf) into cin.
    template <int E>
    __device__ static void eval(const u32 *A, u32 *cin) {
        par_map<2 * S1>(cin, [&](int idx) -> u32 {
            const int x = idx / S1;
            const int w = idx - x * S1;
            const u32 *p = A + x * S;  // [a | b] layout, each S words
            auto get = [&](int part, int j) -> u32 {
                return (j >= 0 && j < m) ? p[part * m + j] : 0u;
            };
            if constexpr (E == 0) return get(0, w);
            else if constexpr (E == 1) return get(0, w) ^ get(1, w) ^ get(2, w);
            else if constexpr (E == 2) return get(0, w) ^ get(1, w - 1) ^ get(2, w - 2);
            else if constexpr (E == 3)
                return get(0, w) ^ get(1, w) ^ get(2, w) ^ get(1, w - 1) ^ get(2, w - 2);
            else return get(2, w);
        });
    }

    // Fold point product p (2*S1 words) into R and the numerators Sa, Ua.
    template <int E>
    __device__ static void absorb(const u32 *p, u32 *R, u32 *Sa, u32 *Ua) {
        auto P = [&](int j) -> u32 { return (j >= 0 && j < 2 * S1) ? p[j] : 0u; };
        if constexpr (E == 0 || E == 1 || E == 4) {
            par_map<R_WORDS>(R, [&](int r) -> u32 {
                if constexpr (E == 0) return R[r] ^ P(r) ^ P(r - m);
                else if constexpr (E == 1) return R[r] ^ P(r - m);
                else return R[r] ^ P(r - m) ^ P(r - 4 * m);
            });
        }
        if constexpr (E != 4) par_map<2 * S1>(Sa, [&](int k) -> u32 { return Sa[k] ^ p[k]; });
        if constexpr (E != 0) {
            par_map<UA_WORDS>(Ua, [&](int k) -> u32 {
                if constexpr (E == 1) return Ua[k] ^ P(k);
                else if constexpr (E == 2) return Ua[k] ^ P(k - 1);
                else if constexpr (E == 3) return Ua[k] ^ P(k) ^ P(k - 1);
                else return Ua[k] ^ P(k - 1) ^ P(k - 4);
            });
        }
    }

    template <int E>
    __device__ static void point(const u32 *in, u32 *R, u32 *Sa, u32 *Ua, u32 *cin, u32 *cs) {
        eval<E>(in, cin);
        __syncthreads();
        const u32 *p = Child::run(cin, cs);
        absorb<E>(p, R, Sa, Ua);
        __syncthreads();
    }

    // in: [a (S) | b (S)]; returns the 2S-word product (inside scratch).
    __device__ static u32 *run(const u32 *in, u32 *scratch) {
        u32 *R = scratch;
        u32 *Sa = R + R_WORDS;
        u32 *Ua = Sa + SA_WORDS;
        u32 *cin = Ua + UA_WORDS;
        u32 *tmp = cin + CIN_WORDS;
        u32 *cs = tmp + TMP_WORDS;
        for (int k = threadIdx.x; k < R_WORDS + SA_WORDS + UA_WORDS; k += NT) R[k] = 0;
        // (the barrier inside point<0> orders these stores before any absorb)
        point<0>(in, R, Sa, Ua, cin, cs);
        point<1>(in, R, Sa, Ua, cin, cs);
        point<2>(in, R, Sa, Ua, cin, cs);
        point<3>(in, R, Sa, Ua, cin, cs);
        point<4>(in, R, Sa, Ua, cin, cs);
        div_xx1_pair<2 * m>(Sa, Ua, tmp);  // Sa <- c3, Ua <- c2 (first 2m words)
        auto c3 = [&](int j) -> u32 { return (j >= 0 && j < 2 * m) ? Sa[j] : 0u; };
        auto c2 = [&](int j) -> u32 { return (j >= 0 && j < 2 * m) ? Ua[j] : 0u; };
        par_map<R_WORDS>(R, [&](int r) -> u32 { return R[r] ^ c2(r - m) ^ c2(r - 2 * m) ^ c3(r - m) ^ c3(r - 3 * m); });
        __syncthreads();
        return R;
    }
};

}  // namespace gf2x
