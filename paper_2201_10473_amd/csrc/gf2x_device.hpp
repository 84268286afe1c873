// gf2x_device.hpp -- device-side building blocks of the bit-packed product
// in F2[X] on gfx950 (MI355X).
//
// Words are 32 bits on the device (the VALU word); a polynomial of S words
// holds coefficient i in bit (i mod 32) of word floor(i/32).  One workgroup
// of NT threads computes one product with its partial products and
// accumulators in LDS and registers.
//
// The recursion is a compile-time schedule built from these pieces:
//   * unit_mul<T>      -- T x T word schoolbook product held in one thread's
//                         registers (the base case).
//   * ParK2<D, T>      -- D levels of 2-way Karatsuba (Appendix A, KaratRec),
//                         executed breadth first: all 3^D base products of a
//                         level run at once, one per thread.
//   * SeqT3<Child,MEM> -- word-aligned Toom-Cook 3 (Appendix D, Section 3.2)
//                         with w = 32, whose five point products are computed
//                         one after another by Child (saves LDS).
//   * SeqT4<Child,MEM> -- Toom-Cook 4 (Section 3, seven products), the same
//                         way; TopT4<Child> is its form spread over workgroups.
//   * SeqKN<N, Child>  -- 3- and 5-way Karatsuba (Appendix A, karat3/karat5).
// With MEM, a Toom level reads the parent's operands from global memory
// whenever it forms a point operand, so no LDS holds them.
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

// The thread index, re-read at each use: index arithmetic derived from it is
// then recomputed in each pass instead of being hoisted out of the item and
// point loops and kept live (and spilled) across the whole product.  Host-side
// builds of these headers use the plain index.
__device__ __forceinline__ int tid() {
#if defined(__HIP_DEVICE_COMPILE__)
    int t;
    asm volatile("v_mov_b32 %0, %1" : "=v"(t) : "v"((int)threadIdx.x));
    __builtin_assume(t >= 0 && t < NT);
    return t;
#else
    return (int)threadIdx.x;
#endif
}

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
        const int idx = tid() + i * NT;
        if (IT * NT == TOTAL || idx < TOTAL) v[i] = f(idx);
    }
#pragma unroll
    for (int i = 0; i < IT; ++i) {
        const int idx = tid() + i * NT;
        if (IT * NT == TOTAL || idx < TOTAL) dst[idx] = v[i];
    }
}

// ------------------------------------------------------------------ base case
// c (2T words) = a (T words) * b (T words) in F2[X], all in registers.
//
// The carry-less product is sum over bits j of a_i of (b << j) placed at word
// i.  The shifted copy sh = b << j is kept as T+1 words and advanced from
// j - 1 to j by one add-with-carry chain (v_add_co / v_addc: sh + sh with the
// carry of the word below, full-rate ops), shared by every a_i; then for
// every word a_i, sh is XORed into c at word offset i under the mask "bit j
// of a_i is set" (one v_bfe_i32): (T+1) v_bitop3 per (i, j).  Each v_bitop3
// retires 32 bit-pair products, and the low and high halves of the 32x32
// products merge into one accumulator word instead of two.
template <int T>
struct Unit {
    // VALU lane-ops of one call: j = 0 uses T bfe + T*T bitop3; each of the
    // other 31 bit positions uses (T+1) carry-chain adds + T bfe + T*(T+1) bitop3.
    static constexpr long long OPS = (long long)T * T + T + 31LL * (T * T + 3 * T + 1);
};

template <int T>
__device__ __forceinline__ void unit_mul(const u32 (&a)[T], const u32 (&b)[T], u32 (&c)[2 * T]) {
#pragma unroll
    for (int k = 0; k < 2 * T; ++k) c[k] = 0;
    u32 sh[T + 1];
#pragma unroll
    for (int u = 0; u < T; ++u) sh[u] = b[u];
    sh[T] = 0;
#pragma unroll
    for (int i = 0; i < T; ++i) {
        const u32 m = bit_mask(a[i], 0);
#pragma unroll
        for (int u = 0; u < T; ++u) c[i + u] = xor_and(c[i + u], sh[u], m);
    }
#pragma unroll 1
    for (u32 j = 1; j < 32; ++j) {
        // sh <<= 1 over T+1 words: each word doubled plus the top bit of the word below
        u32 cy = 0, co;
#pragma unroll
        for (int u = 0; u <= T; ++u) {
            sh[u] = __builtin_addc(sh[u], sh[u], cy, &co);
            cy = co;
        }
#pragma unroll
        for (int i = 0; i < T; ++i) {
            const u32 m = bit_mask(a[i], j);
#pragma unroll
            for (int u = 0; u <= T; ++u) c[i + u] = xor_and(c[i + u], sh[u], m);
        }
    }
}

// XOR a value into an LDS word: ds_xor_b32.  The order of the XORs into
// one word does not change the result, so results are deterministic.
__device__ __forceinline__ void lds_xor(u32 *p, u32 v) {
    __hip_atomic_fetch_xor(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// ------------------------------------------------------- operand sources
// The first split of a Karatsuba subtree reads its root operands through a
// source: word w of operand x (0 = a, 1 = b).
struct LdsSource {
    const u32 *ab;  // [a (S) | b (S)]
    int S;
    __device__ __forceinline__ u32 get(int x, int w) const { return ab[x * S + w]; }
};

// ----------------------------------------------------- 2-way Karatsuba levels
// f(row, col) for 0 <= row < ROWS and 0 <= col < COLS, spread over the
// workgroup.  A thread keeps one column and steps through the rows, so the
// per-element index arithmetic of a level pass reduces to constant offsets
// from one address, and the condition on the column is fixed per thread.
template <int ROWS, int COLS, class F>
__device__ __forceinline__ void grid_map(F f) {
    if constexpr (COLS <= NT) {
        constexpr int RPP = NT / COLS;  // rows per pass
        constexpr int PASSES = (ROWS + RPP - 1) / RPP;
        const int t = tid();
        const int row0 = t / COLS;
        const int col = t - row0 * COLS;
        if (row0 < RPP) {
#pragma unroll
            for (int q = 0; q < PASSES; ++q) {
                const int row = row0 + q * RPP;
                if ((ROWS % RPP) == 0 || row < ROWS) f(row, col);
            }
        }
    } else {
#pragma unroll 1
        for (int row = 0; row < ROWS; ++row)
            for (int col = tid(); col < COLS; col += NT) f(row, col);
    }
}

// As grid_map, in two phases: load(row, col, v) for every element of the
// thread, then store(row, col, v) for every element, so that a pass over a
// level costs one LDS round trip instead of one per row.  load must not read
// what store writes.
template <int ROWS, int COLS, int NV, class L, class S>
__device__ __forceinline__ void grid_map2(L load, S store) {
    if constexpr (COLS <= NT) {
        constexpr int RPP = NT / COLS;
        constexpr int PASSES = (ROWS + RPP - 1) / RPP;
        const int t = tid();
        const int row0 = t / COLS;
        const int col = t - row0 * COLS;
        if (row0 < RPP) {
            u32 v[PASSES][NV];
#pragma unroll
            for (int q = 0; q < PASSES; ++q) {
                const int row = row0 + q * RPP;
                if ((ROWS % RPP) == 0 || row < ROWS) load(row, col, v[q]);
            }
#pragma unroll
            for (int q = 0; q < PASSES; ++q) {
                const int row = row0 + q * RPP;
                if ((ROWS % RPP) == 0 || row < ROWS) store(row, col, v[q]);
            }
        }
    } else {
#pragma unroll 1
        for (int row = 0; row < ROWS; ++row)
            for (int col = tid(); col < COLS; col += NT) {
                u32 v[NV];
                load(row, col, v);
                store(row, col, v);
            }
    }
}

// 3-input XOR in one v_bitop3_b32 (truth table 0x96).
__device__ __forceinline__ u32 xor3(u32 a, u32 b, u32 c) { return __builtin_amdgcn_bitop3_b32(a, b, c, 0x96); }

// Splitting (KaratRec, Appendix A): a node of SL words with operands [a | b]
// becomes three children of H = SL/2 words, in this order:
//   child 0: (a0, b0), child 1: (a1, b1), child 2: (a0 + a1, b0 + b1).
// Node v's operands are at v*2*SL; the children are written at a stride of
// CS >= 2H words (CS > 2H pads a level).  Column r = x*H + w of node v is
// word w of operand x of each child.
template <int NL, int SL, int CS = SL>
__device__ __forceinline__ void k2_split(const u32 *src, u32 *dst) {
    constexpr int H = SL / 2;
    static_assert(CS >= 2 * H, "child stride holds a child");
    grid_map2<NL, 2 * H, 2>(
        [&](int v, int r, u32 (&x)[2]) {
            const u32 *s = src + v * 2 * SL + r + (r >= H ? H : 0);  // word w of operand x: x*SL + w
            x[0] = s[0];
            x[1] = s[H];
        },
        [&](int v, int r, const u32 (&x)[2]) {
            u32 *d = dst + 3 * v * CS + r;
            d[0] = x[0];
            d[CS] = x[1];
            d[2 * CS] = x[0] ^ x[1];
        });
}

// The root split, reading the root operands from a source.
template <int SL, class Src, int CS = SL>
__device__ __forceinline__ void k2_split_src(const Src &src, u32 *dst) {
    constexpr int H = SL / 2;
    grid_map<1, 2 * H>([&](int, int r) {
        const int x = r >= H ? 1 : 0;
        const int w = r - x * H;
        const u32 lo = src.get(x, w);
        const u32 hi = src.get(x, H + w);
        dst[r] = lo;
        dst[CS + r] = hi;
        dst[2 * CS + r] = lo ^ hi;
    });
}

// Reconstruction (KaratRec): R = R0 + (R0 + R1 + R2) X^{32H} + R1 X^{64H}
// with children products R_k of 2H words at a stride of CS words.  Parent
// products are 4H words, stored densely.  Column j < 2H of node v writes the
// middle word H + j (R0[H + j] or R1[j - H], plus R0[j] + R1[j] + R2[j]) and
// one outer word: word j (= R0[j]) when j < H, else word 2H + j (= R1[j]).
template <int NL, int H, int CS = 2 * H>
__device__ __forceinline__ void k2_merge(const u32 *src, u32 *dst) {
    static_assert(CS >= 2 * H, "child stride holds a child");
    grid_map2<NL, 2 * H, 2>(
        [&](int v, int j, u32 (&x)[2]) {
            const u32 *R = src + 3 * v * CS + j;
            const u32 r0 = R[0], r1 = R[CS];
            const u32 rm = j < H ? R[H] : R[CS - H];  // word H + j of [R0 | R1]
            x[0] = xor3(rm, r0, r1) ^ R[2 * CS];
            x[1] = j < H ? r0 : r1;
        },
        [&](int v, int j, const u32 (&x)[2]) {
            u32 *O = dst + v * 4 * H;
            O[H + j] = x[0];
            O[j < H ? j : 2 * H + j] = x[1];
        });
}

// D levels of 2-way Karatsuba over T-word units, breadth first, 3^D <= NT
// units (one per thread, one round).
//   S       = T * 2^D operand words; the product has 2S words.
//   scratch = [DA (level D-1: 3^(D-1) nodes x 4T words) | DB (3^(D-2) x 8T)].
// Down pass: the root split reads the source; level L is stored in DA when
// D-1-L is even, else in DB (so level D-1 lands in DA).  The units read
// their operands from level D-1, i.e. they perform the last split while
// loading (child 0 reads the low halves of its parent's operands, child 1
// the high halves, child 2 both).  The last merge is fused too: after every
// unit has loaded its operands, each unit writes its product into its
// parent's product in place, at offset T*k for child k:
//   child 0 and 1 add [c_lo, c_lo + c_hi, c_hi], child 2 adds [c_lo, c_hi]
// (the KaratRec reconstruction, distributed over the three children).  The
// words that one child alone covers, and child 2's middle words, are plain
// stores; after a barrier children 0 and 1 add into the middle (LDS atomics),
// so level D-1 needs no clearing.  The
// up pass then alternates DA -> DB -> DA ... with the same parity rule, and
// every buffer written is dead at that point.
template <int D, int T>
struct ParK2 {
    static_assert(D >= 0 && pow3(D) <= NT, "one unit per thread");
    static constexpr bool IS_SEQ = false;
    static constexpr bool FROM_MEM = false;  // operands staged in LDS by the caller
    static constexpr int S = T << D;
    static constexpr long long UNITS = pow3(D);
    // Level D-1 (the units' parents) is stored at a node stride of 4T + 1
    // words: an odd stride spreads the nodes read and XORed by the lanes of a
    // wave over distinct LDS banks.
    static constexpr int NS = D >= 2 ? 4 * T + 1 : 4 * T;
    static constexpr int DA_WORDS = D >= 1 ? (int)(NS * pow3(D - 1)) : 2 * T;
    static constexpr int DB_WORDS = D >= 2 ? (int)(8 * T * pow3(D - 2)) : 0;
    static constexpr int SCRATCH = DA_WORDS + DB_WORDS;
    static constexpr long long BASE = UNITS * T * T;   // 32x32 word products
    // XOR lane-ops of one level of size SL over NL nodes: split SL, merge 3*SL.
    static constexpr long long xor_ops(int l) {
        return l >= D ? 0 : pow3(l) * 4LL * (T << (D - l)) + xor_ops(l + 1);
    }
    static constexpr long long OPS = UNITS * Unit<T>::OPS + xor_ops(0);

    template <int L>
    __device__ __forceinline__ static u32 *level_buf(u32 *DA, u32 *DB) {
        if constexpr (((D - 1 - L) % 2) == 0) return DA;
        else return DB;
    }

    // levels L -> L+1 for 1 <= L < D-1
    template <int L>
    __device__ __forceinline__ static void down(u32 *DA, u32 *DB) {
        if constexpr (L + 1 <= D - 1) {
            constexpr int CS = (L + 1 == D - 1) ? NS : (T << (D - L));
            k2_split<(int)pow3(L), (T << (D - L)), CS>(level_buf<L>(DA, DB), level_buf<L + 1>(DA, DB));
            __syncthreads();
            down<L + 1>(DA, DB);
        }
    }

    // merges from level L+1 (products) to level L, down to the root
    template <int L>
    __device__ __forceinline__ static u32 *up(u32 *DA, u32 *DB) {
        if constexpr (L < 0) {
            return level_buf<0>(DA, DB);
        } else {
            constexpr int CS = (L + 1 == D - 1) ? NS : (T << (D - L));
            k2_merge<(int)pow3(L), (T << (D - L - 1)), CS>(level_buf<L + 1>(DA, DB), level_buf<L>(DA, DB));
            __syncthreads();
            return up<L - 1>(DA, DB);
        }
    }

    // The unit phase: load (last split), multiply, write the product into
    // the parent (last merge).  Source Src is only used for D == 1.
    template <class Src>
    __device__ __forceinline__ static void units(const Src &src, u32 *DA) {
        const int u = tid();
        const bool active = u < (int)UNITS;
        const int v = u / 3, k = u - 3 * (u / 3);
        u32 a[T], b[T], c[2 * T];
        if (active) {
            if constexpr (D == 1) {
#pragma unroll
                for (int w = 0; w < T; ++w) {
                    const u32 alo = src.get(0, w), ahi = src.get(0, T + w);
                    const u32 blo = src.get(1, w), bhi = src.get(1, T + w);
                    a[w] = (k != 1 ? alo : 0u) ^ (k != 0 ? ahi : 0u);
                    b[w] = (k != 1 ? blo : 0u) ^ (k != 0 ? bhi : 0u);
                }
            } else {
                // [a_v (2T) | b_v (2T)]: unit 0 takes the low halves, unit 1
                // the high halves, unit 2 their sums
                const u32 *node = DA + v * NS;
                const u32 *half = node + (k == 1 ? T : 0);
#pragma unroll
                for (int w = 0; w < T; ++w) {
                    a[w] = half[w];
                    b[w] = half[2 * T + w];
                }
                if (k == 2) {
#pragma unroll
                    for (int w = 0; w < T; ++w) {
                        a[w] ^= node[T + w];
                        b[w] ^= node[3 * T + w];
                    }
                }
            }
        }
        __syncthreads();
        // Node v's product (4T words) replaces its operands.  Child 0 alone
        // writes words [0, T), child 1 alone [3T, 4T); child 2 first stores
        // its [c_lo, c_hi] over the middle [T, 3T), then children 0 and 1 add
        // theirs there.
        u32 *node = DA + v * NS;
        if (active) {
            unit_mul<T>(a, b, c);
            u32 *own = node + (k == 0 ? 0 : k == 1 ? 3 * T : T);
#pragma unroll
            for (int w = 0; w < T; ++w) own[w] = k == 1 ? c[T + w] : c[w];
            if (k == 2) {
#pragma unroll
                for (int w = 0; w < T; ++w) node[2 * T + w] = c[T + w];
            }
        }
        __syncthreads();
        if (active && k < 2) {
#pragma unroll
            for (int w = 0; w < T; ++w) {
                const u32 mid = c[w] ^ c[T + w];
                lds_xor(node + T + w, k == 0 ? mid : c[w]);
                lds_xor(node + 2 * T + w, k == 0 ? c[T + w] : mid);
            }
        }
        __syncthreads();
    }

    // Product of the root operands given by src; returns its 2S words.
    template <class Src>
    __device__ __forceinline__ static u32 *run_src(const Src &src, u32 *scratch) {
        u32 *DA = scratch;
        u32 *DB = scratch + DA_WORDS;
        if constexpr (D == 0) {
            u32 a[T], b[T], c[2 * T];
            if (tid() == 0) {
#pragma unroll
                for (int w = 0; w < T; ++w) {
                    a[w] = src.get(0, w);
                    b[w] = src.get(1, w);
                }
                unit_mul<T>(a, b, c);
#pragma unroll
                for (int w = 0; w < 2 * T; ++w) DA[w] = c[w];
            }
            __syncthreads();
            return DA;
        } else {
            if constexpr (D >= 2) {
                k2_split_src<S, Src, (D == 2 ? NS : S)>(src, level_buf<1>(DA, DB));
                __syncthreads();
                down<1>(DA, DB);
            }
            units(src, DA);
            return up<D - 2>(DA, DB);
        }
    }

    __device__ __forceinline__ static u32 *run_ab(u32 *ab, u32 *scratch) { return run_src(LdsSource{ab, S}, scratch); }
};

// --------------------------------------------------------- workgroup scans
// x[k] <- XOR of x[1..k+1] and y[k] <- XOR of y[1..k+1] for 0 <= k < L:
// division by x (drop the low word, which exact division leaves zero) then by
// x + 1 (multiplication by sum_i x^i, i.e. a prefix XOR over w-bit blocks,
// Section 3.2) in one pass.  tmp: 2*NWAVE words.  Ends with a barrier.
template <int L>
__device__ __forceinline__ void div_xx1_pair(u32 *x, u32 *y, u32 *tmp) {
    constexpr int C = (L + NT - 1) / NT;
    const int t = tid();
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
// Operands of Toom-3 point E (0: 0, 1: 1, 2: x, 3: x+1, 4: inf) computed
// on the fly from the parent's [a | b] (S = 3m words each):
//   e0 = a0, e1 = a0+a1+a2, ex = a0 + x a1 + x^2 a2, ex1 = e1 + x a1 + x^2 a2,
//   einf = a2, with x a word shift.
template <int E>
struct EvalSource {
    const u32 *ab;
    int S, m;
    __device__ __forceinline__ u32 part(int x, int p, int j) const {
        return (j >= 0 && j < m) ? ab[x * S + p * m + j] : 0u;
    }
    __device__ __forceinline__ u32 get(int x, int w) const {
        if constexpr (E == 0) return part(x, 0, w);
        else if constexpr (E == 1) return part(x, 0, w) ^ part(x, 1, w) ^ part(x, 2, w);
        else if constexpr (E == 2) return part(x, 0, w) ^ part(x, 1, w - 1) ^ part(x, 2, w - 2);
        else if constexpr (E == 3)
            return part(x, 0, w) ^ part(x, 1, w) ^ part(x, 2, w) ^ part(x, 1, w - 1) ^ part(x, 2, w - 2);
        else return part(x, 2, w);
    }
};

// With FROM_MEM, the level reads the parent's operands straight from memory
// (global, masked to n bits) whenever a point operand is formed, instead of
// from a copy staged in LDS: the workgroup then needs no LDS for [a | b]
// (2S words), and the product is assembled in the child's scratch.
template <class Child, bool MEM = false>
struct SeqT3 {
    static constexpr bool IS_SEQ = true;
    static constexpr bool FROM_MEM = MEM;
    static constexpr int NP = 5;  // point products
    static constexpr int S1 = Child::S;
    static constexpr int m = S1 - 2;
    static constexpr int S = 3 * m;
    static constexpr int R_WORDS = 6 * m;
    // R lives in registers: word r of R is held by thread r mod NT.
    static constexpr int IRW = (R_WORDS + NT - 1) / NT;
    static constexpr int SA_WORDS = 2 * S1 + 2;
    static constexpr int UA_WORDS = 2 * S1 + 2;
    // a Toom-3 child needs its operands materialised (it reads them five
    // times); a Karatsuba child reads them through its root split
    static constexpr int CIN_WORDS = Child::IS_SEQ ? 2 * S1 : 0;
    static constexpr int TMP_WORDS = 2 * NWAVE;
    // The scan scratch of the final division is taken from the child's
    // scratch, which is dead by then; the product is written over the
    // operands [a | b] (2S words = R_WORDS), which are dead too.
    static_assert(Child::SCRATCH >= TMP_WORDS, "child scratch holds the scan scratch");
    static_assert(!MEM || Child::SCRATCH >= R_WORDS + TMP_WORDS, "child scratch holds the product and scan scratch");
    static constexpr int SCRATCH = SA_WORDS + UA_WORDS + CIN_WORDS + Child::SCRATCH;
    static constexpr long long BASE = 5 * Child::BASE;
    // evaluation 16*S1, absorption 30*S1, divisions 4m, recombination 8m
    static constexpr long long OPS = 5 * Child::OPS + 46LL * S1 + 12LL * m;

    // Fold point product p (2*S1 words) into R (registers) and the numerators
    // Sa, Ua.  Only the words of R that receive a nonzero term are touched,
    // and every new numerator word is computed before any is stored.
    template <int E>
    __device__ __forceinline__ static void absorb(const u32 *p, u32 (&R)[IRW], u32 *Sa, u32 *Ua) {
        auto P = [&](int j) -> u32 { return (j >= 0 && j < 2 * S1) ? p[j] : 0u; };
        // R gets P(r) + P(r-m) (point 0), P(r-m) (point 1), P(r-m) + P(r-4m) (point inf)
        constexpr int R_LO = (E == 0 || E == 2 || E == 3) ? 0 : m;
        constexpr int R_HI = (E == 0) ? m + 2 * S1 : (E == 1) ? m + 2 * S1 : (E == 4) ? R_WORDS : 0;
        constexpr int NS = (E != 4) ? 2 * S1 : 0, IS = (NS + NT - 1) / NT;
        constexpr int NU = (E != 0) ? UA_WORDS : 0, IU = (NU + NT - 1) / NT;
        static_assert(R_HI <= R_WORDS, "point 0 and 1 terms fit in R");
        const int t = tid();
        u32 vs[IS > 0 ? IS : 1], vu[IU > 0 ? IU : 1];
        if constexpr (R_HI > R_LO) {
#pragma unroll
            for (int i = 0; i < IRW; ++i) {
                const int r = t + i * NT;
                if (r >= R_LO && r < R_HI) {
                    if constexpr (E == 0) R[i] ^= P(r) ^ P(r - m);
                    else if constexpr (E == 1) R[i] ^= P(r - m);
                    else R[i] ^= P(r - m) ^ P(r - 4 * m);
                }
            }
        }
#pragma unroll
        for (int i = 0; i < IS; ++i) {
            const int k = t + i * NT;
            if (k < NS) vs[i] = Sa[k] ^ p[k];
        }
#pragma unroll
        for (int i = 0; i < IU; ++i) {
            const int k = t + i * NT;
            if (k < NU) {
                u32 v;
                if constexpr (E == 1) v = P(k);
                else if constexpr (E == 2) v = P(k - 1);
                else if constexpr (E == 3) v = P(k) ^ P(k - 1);
                else v = P(k - 1) ^ P(k - 4);
                vu[i] = Ua[k] ^ v;
            }
        }
#pragma unroll
        for (int i = 0; i < IS; ++i) {
            const int k = t + i * NT;
            if (k < NS) Sa[k] = vs[i];
        }
#pragma unroll
        for (int i = 0; i < IU; ++i) {
            const int k = t + i * NT;
            if (k < NU) Ua[k] = vu[i];
        }
    }

    template <int E>
    __device__ __forceinline__ static void point(u32 *ab, u32 (&R)[IRW], u32 *Sa, u32 *Ua, u32 *cin, u32 *cs) {
        point_from<E>(EvalSource<E>{ab, S, m}, R, Sa, Ua, cin, cs);
    }

    // Word w of operand x of point E from the parent's operands in memory:
    // part j of operand x is words p m + j of a or b (u32 words), masked to n.
    template <int E>
    struct MemSource {
        const u32 *a, *b;
        int w32;
        u32 top;
        __device__ __forceinline__ u32 part(int x, int p, int j) const {
            const int k = p * m + j;
            if (j < 0 || j >= m || k >= w32) return 0u;
            const u32 v = (x ? b : a)[k];
            return k == w32 - 1 ? (v & top) : v;
        }
        __device__ __forceinline__ u32 get(int x, int w) const {
            if constexpr (E == 0) return part(x, 0, w);
            else if constexpr (E == 1) return part(x, 0, w) ^ part(x, 1, w) ^ part(x, 2, w);
            else if constexpr (E == 2) return part(x, 0, w) ^ part(x, 1, w - 1) ^ part(x, 2, w - 2);
            else if constexpr (E == 3)
                return part(x, 0, w) ^ part(x, 1, w) ^ part(x, 2, w) ^ part(x, 1, w - 1) ^ part(x, 2, w - 2);
            else return part(x, 2, w);
        }
    };

    template <int E, class Src>
    __device__ __forceinline__ static void point_from(const Src &src, u32 (&R)[IRW], u32 *Sa, u32 *Ua, u32 *cin,
                                                      u32 *cs) {
        const u32 *p;
        if constexpr (Child::IS_SEQ) {
            par_map<2 * S1>(cin, [&](int idx) -> u32 {
                const int x = idx / S1;
                return src.get(x, idx - x * S1);
            });
            __syncthreads();
            p = Child::run_ab(cin, cs);
        } else {
            p = Child::run_src(src, cs);
        }
        absorb<E>(p, R, Sa, Ua);
        __syncthreads();
    }

    // Final division and recombination: Sa <- c3, Ua <- c2 (first 2m words),
    // then out[r] = R[r] + c2 (Y + Y^2) + c3 (Y + Y^3) at word r.
    __device__ __forceinline__ static void finish(const u32 (&R)[IRW], u32 *Sa, u32 *Ua, u32 *tmp, u32 *out) {
        div_xx1_pair<2 * m>(Sa, Ua, tmp);
        auto c3 = [&](int j) -> u32 { return (j >= 0 && j < 2 * m) ? Sa[j] : 0u; };
        auto c2 = [&](int j) -> u32 { return (j >= 0 && j < 2 * m) ? Ua[j] : 0u; };
        const int t = tid();
#pragma unroll
        for (int i = 0; i < IRW; ++i) {
            const int r = t + i * NT;
            if (r < R_WORDS) out[r] = R[i] ^ c2(r - m) ^ c2(r - 2 * m) ^ c3(r - m) ^ c3(r - 3 * m);
        }
        __syncthreads();
    }

    // Interpolation only: the five point products (2*S1 words each, in order
    // 0, 1, x, x+1, inf) were computed elsewhere and sit at products (any
    // address space).  scratch needs INTERP_SCRATCH words; returns the 2S-word
    // product inside scratch.
    static constexpr int INTERP_SCRATCH = R_WORDS + SA_WORDS + UA_WORDS + TMP_WORDS;
    static constexpr bool INTERP_STORES = false;  // interp_from returns the product
    __device__ __forceinline__ static u32 *interp_from(const u32 *products, u32 *scratch) {
        u32 *out = scratch;
        u32 *Sa = out + R_WORDS;
        u32 *Ua = Sa + SA_WORDS;
        u32 *tmp = Ua + UA_WORDS;
        u32 R[IRW];
#pragma unroll
        for (int i = 0; i < IRW; ++i) R[i] = 0;
        for (int k = tid(); k < SA_WORDS + UA_WORDS; k += NT) Sa[k] = 0;
        __syncthreads();
        absorb<0>(products + 0 * 2 * S1, R, Sa, Ua);
        __syncthreads();
        absorb<1>(products + 1 * 2 * S1, R, Sa, Ua);
        __syncthreads();
        absorb<2>(products + 2 * 2 * S1, R, Sa, Ua);
        __syncthreads();
        absorb<3>(products + 3 * 2 * S1, R, Sa, Ua);
        __syncthreads();
        absorb<4>(products + 4 * 2 * S1, R, Sa, Ua);
        __syncthreads();
        finish(R, Sa, Ua, tmp, out);
        return out;
    }

    // Word w of operand x of point e, from a source of the parent's words.
    template <class Part>
    __device__ __forceinline__ static u32 point_word(int e, int x, int w, const Part &part) {
        switch (e) {
            case 0: return part(x, 0, w);
            case 1: return part(x, 0, w) ^ part(x, 1, w) ^ part(x, 2, w);
            case 2: return part(x, 0, w) ^ part(x, 1, w - 1) ^ part(x, 2, w - 2);
            case 3: return part(x, 0, w) ^ part(x, 1, w) ^ part(x, 2, w) ^ part(x, 1, w - 1) ^ part(x, 2, w - 2);
            default: return part(x, 2, w);
        }
    }

    // The parent's operands a, b (n bits each, u32 words) read from memory;
    // returns the 2S-word product, assembled in the child's scratch.
    __device__ __forceinline__ static u32 *run_mem(const u32 *a, const u32 *b, u32 n, u32 *scratch) {
        u32 *Sa = scratch;
        u32 *Ua = Sa + SA_WORDS;
        u32 *cin = Ua + UA_WORDS;
        u32 *cs = cin + CIN_WORDS;
        const int w32 = (int)((n + 31u) / 32u);
        const u32 sn = n % 32u;
        const u32 top = sn ? ((1u << sn) - 1u) : 0xFFFFFFFFu;
        u32 R[IRW];
#pragma unroll
        for (int i = 0; i < IRW; ++i) R[i] = 0;
        for (int k = tid(); k < SA_WORDS + UA_WORDS; k += NT) Sa[k] = 0;
        point_from<0>(MemSource<0>{a, b, w32, top}, R, Sa, Ua, cin, cs);
        point_from<1>(MemSource<1>{a, b, w32, top}, R, Sa, Ua, cin, cs);
        point_from<2>(MemSource<2>{a, b, w32, top}, R, Sa, Ua, cin, cs);
        point_from<3>(MemSource<3>{a, b, w32, top}, R, Sa, Ua, cin, cs);
        point_from<4>(MemSource<4>{a, b, w32, top}, R, Sa, Ua, cin, cs);
        finish(R, Sa, Ua, cs + R_WORDS, cs);
        return cs;
    }

    // ab: [a (S) | b (S)] in LDS.  Returns the 2S-word product, written over
    // ab (whose words are dead once the last point has been evaluated).
    __device__ __forceinline__ static u32 *run_ab(u32 *ab, u32 *scratch) {
        u32 *Sa = scratch;
        u32 *Ua = Sa + SA_WORDS;
        u32 *cin = Ua + UA_WORDS;
        u32 *cs = cin + CIN_WORDS;
        u32 R[IRW];
#pragma unroll
        for (int i = 0; i < IRW; ++i) R[i] = 0;
        for (int k = tid(); k < SA_WORDS + UA_WORDS; k += NT) Sa[k] = 0;
        // (the barriers inside the first child run order these stores before any absorb)
        point<0>(ab, R, Sa, Ua, cin, cs);
        point<1>(ab, R, Sa, Ua, cin, cs);
        point<2>(ab, R, Sa, Ua, cin, cs);
        point<3>(ab, R, Sa, Ua, cin, cs);
        point<4>(ab, R, Sa, Ua, cin, cs);
        finish(R, Sa, Ua, cs, ab);
        return ab;
    }
};

// ------------------------------------------------------ strided prefix XOR
// x[k] <- x[k] + x[k-s] + x[k-2s] + ... for 0 <= k < L (s = STRIDE): exact
// division by 1 + x^s of a polynomial in x = X^32 given by its words, from
// the low end (the division by x + 1 of Section 3.2, generalised to x^s + 1).
// Each thread scans a block of C consecutive words (C a multiple of s, so
// the chain k mod s of a word is its offset mod s), then the block totals of
// the s chains are scanned across the workgroup.  tmp: NWAVE*STRIDE words.
// Ends with a barrier.
template <int L, int STRIDE>
struct XorScan {
    static constexpr int C = STRIDE * ((L + NT * STRIDE - 1) / (NT * STRIDE));
    u32 v[C], acc[STRIDE], tot[STRIDE];

    // This thread's C words: local prefixes, then the wave's inclusive
    // prefix of the per-thread totals; lane 63 leaves the wave total in
    // tmp[wave * STRIDE + c].
    __device__ __forceinline__ void up(const u32 *x, u32 *tmp) {
        const int t = tid();
#pragma unroll
        for (int c = 0; c < STRIDE; ++c) acc[c] = 0;
#pragma unroll
        for (int i = 0; i < C; ++i) {
            const int k = t * C + i;
            acc[i % STRIDE] ^= (k < L) ? x[k] : 0u;
            v[i] = acc[i % STRIDE];
        }
#pragma unroll
        for (int c = 0; c < STRIDE; ++c) tot[c] = acc[c];
        const int lane = t & 63;
#pragma unroll
        for (int d = 1; d < 64; d <<= 1) {
#pragma unroll
            for (int c = 0; c < STRIDE; ++c) {
                const u32 o = __shfl_up(acc[c], d, 64);
                if (lane >= d) acc[c] ^= o;
            }
        }
        if (lane == 63) {
#pragma unroll
            for (int c = 0; c < STRIDE; ++c) tmp[(t >> 6) * STRIDE + c] = acc[c];
        }
    }

    // After a barrier: adds the exclusive prefix of this thread's block.
    __device__ __forceinline__ void down(u32 *x, const u32 *tmp) {
        const int t = tid();
        const int wave = t >> 6;
        u32 pre[STRIDE];
#pragma unroll
        for (int c = 0; c < STRIDE; ++c) {
            pre[c] = acc[c] ^ tot[c];
            for (int w = 0; w < wave; ++w) pre[c] ^= tmp[w * STRIDE + c];
        }
#pragma unroll
        for (int i = 0; i < C; ++i) {
            const int k = t * C + i;
            if (k < L) x[k] = v[i] ^ pre[i % STRIDE];
        }
    }
};

template <int L, int STRIDE>
__device__ __forceinline__ void scan_xor_stride(u32 *x, u32 *tmp) {
    XorScan<L, STRIDE> sc;
    sc.up(x, tmp);
    __syncthreads();
    sc.down(x, tmp);
    __syncthreads();
}

// Three independent strided scans (as scan_xor_stride) under one pair of
// barriers.  tmp: NWAVE*(SA+SB+SC) words.
template <int L, int SA, int SB, int SC>
__device__ __forceinline__ void scan_xor_stride3(u32 *a, u32 *b, u32 *c, u32 *tmp) {
    XorScan<L, SA> sa;
    XorScan<L, SB> sb;
    XorScan<L, SC> sc;
    sa.up(a, tmp);
    sb.up(b, tmp + NWAVE * SA);
    sc.up(c, tmp + NWAVE * (SA + SB));
    __syncthreads();
    sa.down(a, tmp);
    sb.down(b, tmp + NWAVE * SA);
    sc.down(c, tmp + NWAVE * (SA + SB));
    __syncthreads();
}

// ------------------------------------------------------------- Toom-Cook 4
// Word-aligned Toom-Cook 4 with x = X^32 (the four-way split that the
// Toom-Cook complexity table of Section 3 lists for operands above 346
// 64-bit words), used as the staged top level only.  Operands of S = 4m words
// split as a = a0 + a1 Y + a2 Y^2 + a3 Y^3, Y = X^{32m}.  Seven points, in
// this order:
//   0, 1, x, z = x+1, 1/x, 1/z, inf,
// the two reciprocal points homogenised (x^3 a(1/x), z^3 a(1/z)) so that
// every point operand is a polynomial of at most m + 3 words: S1 = m + 3.
//
// Interpolation.  With c(Y) = c0 + Y P(Y) + c6 Y^6, P(t) = c1 + c2 t + ... +
// c5 t^4, the symmetric sums E(t) = P(t) + t^4 P(1/t) only involve
// u = c1 + c5 and v = c2 + c4:  E(t) = u (1+t)^4 + v t (1+t)^2, so that
// E(x) and E(z) (note 1 + z = x) give
//   u = (x E(x) + z E(z)) / (x (x^3 + 1)),   v = (x E(x) + (x + x^5) u) / (x^2 (x^2 + 1)),
// then c3 = C(1) + c0 + c6 + u + v.  The same two-point system in G(t) =
// P(t) + c3 t^2 + v t^3 + u t^4 = c1 (1+t)^4 + c2 t (1+t)^2 gives c1 and c2,
// and c5 = u + c1, c4 = v + c2.  Every division is exact; division by x^s is
// a word shift and by x^s + 1 a strided prefix XOR (scan_xor_stride), with
// s = 3 (x^3 + 1 = (x + 1)(x^2 + x + 1)) and s = 2 ((x + 1)^2 = x^2 + 1).
template <class Child>
struct TopT4 {
    static constexpr bool IS_SEQ = true;
    static constexpr bool FROM_MEM = false;
    static constexpr int NP = 7;
    static constexpr int S1 = Child::S;
    static constexpr int m = S1 - 3;
    static constexpr int S = 4 * m;
    static constexpr int L = 2 * m;  // words of each coefficient c_i
    static constexpr int TMP_WORDS = 3 * NWAVE;
    // u, v, c3, c1, c2 (L words each), the words of the product that the
    // fold shifts down (S + 2), scan scratch
    static constexpr int INTERP_SCRATCH = 5 * L + (S + 2) + TMP_WORDS;
    static constexpr bool INTERP_STORES = true;  // interp_store writes the result
    static constexpr long long BASE = 7 * Child::BASE;
    // evaluation 50*S1 (25 XORs per word of each operand), interpolation
    // about 39 XORs per coefficient word and 6 per product word
    static constexpr long long OPS = 7 * Child::OPS + 50LL * S1 + 126LL * m;

    // Word w of operand x of point e, from a source of the parent's words.
    template <class Part>
    __device__ __forceinline__ static u32 point_word(int e, int x, int w, const Part &part) {
        auto p = [&](int q, int j) -> u32 { return part(x, q, j); };
        switch (e) {
            case 0: return p(0, w);
            case 1: return p(0, w) ^ p(1, w) ^ p(2, w) ^ p(3, w);
            case 2: return p(0, w) ^ p(1, w - 1) ^ p(2, w - 2) ^ p(3, w - 3);
            case 3:  // a0 + a1 (x+1) + a2 (x^2+1) + a3 (x^3+x^2+x+1)
                return p(0, w) ^ p(1, w) ^ p(1, w - 1) ^ p(2, w) ^ p(2, w - 2) ^ p(3, w) ^ p(3, w - 1) ^ p(3, w - 2) ^
                       p(3, w - 3);
            case 4: return p(0, w - 3) ^ p(1, w - 2) ^ p(2, w - 1) ^ p(3, w);
            case 5:  // a0 z^3 + a1 z^2 + a2 z + a3
                return p(0, w) ^ p(0, w - 1) ^ p(0, w - 2) ^ p(0, w - 3) ^ p(1, w) ^ p(1, w - 2) ^ p(2, w) ^ p(2, w - 1) ^
                       p(3, w);
            default: return p(3, w);
        }
    }

    // The seven point products (2*S1 words each, in point order) sit at
    // products (any address space).  Interpolates, recombines and stores
    // the product of n-bit operands at c64: the ring product (kind 0: W(n)
    // words, the fold r = c + (c >> n)) or the full product (2 W(n) words).
    // The 2S-word product is never stored whole: its words are formed where
    // they are used, and only the S + 2 words that the fold shifts down are
    // staged.  scratch needs INTERP_SCRATCH words.
    __device__ __forceinline__ static void interp_store(const u32 *products, u32 *scratch, u32 n, u32 kind,
                                                        uint64_t *c64) {
        u32 *U = scratch;
        u32 *V = U + L;
        u32 *C3 = V + L;
        u32 *C1 = C3 + L;
        u32 *C2 = C1 + L;
        u32 *H = C2 + L;
        u32 *tmp = H + S + 2;
        // word j of point product e, and of a coefficient array, zero outside
        auto P = [&](int e, int j) -> u32 { return (j >= 0 && j < 2 * S1) ? products[e * 2 * S1 + j] : 0u; };
        auto A = [&](const u32 *c, int j) -> u32 { return (j >= 0 && j < L) ? c[j] : 0u; };
        auto s06 = [&](int j) -> u32 { return P(0, j) ^ P(6, j); };
        const int t = tid();
        // One pass over the point products: every term of the five
        // numerators that depends on them alone (the terms in u, v, c1, c3
        // are added once those are known).
        for (int k = t; k < L; k += NT) {
            const int j1 = k + 1, j2 = k + 2;
            // (x E(x) + z E(z)) / x
            U[k] = P(2, j1) ^ P(4, j1) ^ P(3, j1) ^ P(5, j1) ^ s06(j1) ^ s06(j1 - 2) ^ s06(j1 - 4);
            // x E(x) / x^2, without the (x + x^5) u term
            V[k] = P(2, j2) ^ P(4, j2) ^ s06(j2) ^ s06(j2 - 6);
            // C(1) + c0 + c6, without u + v
            C3[k] = P(1, k) ^ s06(k);
            // (x G(x) + z G(z)) / x, without the c3, v, u terms
            C1[k] = P(2, j1) ^ P(3, j1) ^ P(6, j1) ^ P(6, j1 - 2) ^ P(6, j1 - 4);
            // x G(x) / x^2, without the c3, v, u, c1 terms
            C2[k] = P(2, j2) ^ P(0, j2) ^ P(6, j2 - 6);
        }
        __syncthreads();
        // u = ... / (x^3 + 1)
        scan_xor_stride<L, 3>(U, tmp);
        // v = (x E(x) + (x + x^5) u) / x^2, then / (x^2 + 1)
        for (int k = t; k < L; k += NT) V[k] ^= A(U, k + 1) ^ A(U, k - 3);
        __syncthreads();
        scan_xor_stride<L, 2>(V, tmp);
        // c3 = C(1) + c0 + c6 + u + v
        for (int k = t; k < L; k += NT) C3[k] ^= U[k] ^ V[k];
        __syncthreads();
        // c1 = (x G(x) + z G(z)) / x, then / (x^3 + 1):
        // the terms (1 + x + x^2) c3 + v + (1 + x + x^4) u at word k + 1
        for (int k = t; k < L; k += NT)
            C1[k] ^= A(C3, k + 1) ^ A(C3, k) ^ A(C3, k - 1) ^ A(V, k + 1) ^ A(U, k + 1) ^ A(U, k) ^ A(U, k - 3);
        __syncthreads();
        scan_xor_stride<L, 3>(C1, tmp);
        // c2 = (x G(x) + (x + x^5) c1) / x^2, then / (x^2 + 1):
        // the terms x^3 c3 + x^4 v + x^5 u + (x + x^5) c1 at word k + 2
        for (int k = t; k < L; k += NT)
            C2[k] ^= A(C3, k - 1) ^ A(V, k - 2) ^ A(U, k - 3) ^ A(C1, k + 1) ^ A(C1, k - 3);
        __syncthreads();
        scan_xor_stride<L, 2>(C2, tmp);
        // recomposition: word r of c0 + c1 Y + ... + c6 Y^6 (c4 = v + c2,
        // c5 = u + c1), zero outside [0, 2S)
        auto word = [&](int r) -> u32 {
            if (r < 0 || r >= 2 * S) return 0u;
            u32 w = (r < L) ? P(0, r) : 0u;
            w ^= A(C1, r - m);
            w ^= A(C2, r - 2 * m);
            w ^= A(C3, r - 3 * m);
            w ^= A(V, r - 4 * m) ^ A(C2, r - 4 * m);
            w ^= A(U, r - 5 * m) ^ A(C1, r - 5 * m);
            w ^= (r - 6 * m >= 0 && r - 6 * m < L) ? P(6, r - 6 * m) : 0u;
            return w;
        };
        u32 *c32 = reinterpret_cast<u32 *>(c64);
        const int W64 = (int)((n + 63u) / 64u);
        if (kind == 0u) {
            // ring: out[k] = c[k] + (c >> n)[k], the shifted words staged in H
            const int w32 = (int)((n + 31u) / 32u);
            const int q = (int)(n / 32u);
            const u32 sn = n % 32u;
            const u32 top = sn ? ((1u << sn) - 1u) : 0xFFFFFFFFu;
            for (int k = t; k <= w32; k += NT) H[k] = word(k + q);  // w32 <= S
            __syncthreads();
            for (int k = t; k < 2 * W64; k += NT) {
                u32 v = 0;
                if (k < w32) {
                    v = word(k) ^ __builtin_amdgcn_alignbit(H[k + 1], H[k], sn);
                    if (k == w32 - 1) v &= top;
                }
                c32[k] = v;
            }
        } else {
            for (int k = t; k < 4 * W64; k += NT) c32[k] = word(k);
        }
        __syncthreads();
    }
};

// --------------------------------------------- Toom-Cook 4 in one workgroup
// The Toom-Cook 4 level of TopT4 computed inside one workgroup: the seven
// point products one after another (each by Child, its operands read
// through TopT4::point_word from the parent's [a | b] in LDS), and the
// interpolation of TopT4 streamed: the first pass of that interpolation is
// linear in the point products, so each product is folded into the five
// numerator arrays U, V, C3, C1, C2 (2m words each) as soon as it exists, and
// C(0) and C(inf) go straight into the result accumulator R (8m words, in
// registers: word r is held by thread r mod NT).  Then the four exact
// divisions and the recomposition of TopT4 run in LDS.  With MEM, the point
// operands are formed from the parent's operands in memory (masked to n
// bits), as in SeqT3: no LDS holds [a | b].
template <int E, class Top>
struct T4Source {
    const u32 *ab;
    __device__ __forceinline__ u32 get(int x, int w) const {
        auto part = [&](int xx, int q, int j) -> u32 {
            return (j >= 0 && j < Top::m) ? ab[xx * Top::S + q * Top::m + j] : 0u;
        };
        return Top::point_word(E, x, w, part);
    }
};

// Part q (m words) of operand x read from memory: words q m + j of a or b.
template <int E, class Top>
struct T4MemSource {
    const u32 *a, *b;
    int w32;
    u32 top;
    __device__ __forceinline__ u32 get(int x, int w) const {
        auto part = [&](int xx, int q, int j) -> u32 {
            const int k = q * Top::m + j;
            if (j < 0 || j >= Top::m || k >= w32) return 0u;
            const u32 v = (xx ? b : a)[k];
            return k == w32 - 1 ? (v & top) : v;
        };
        return Top::point_word(E, x, w, part);
    }
};

template <class Child, bool MEM = false>
struct SeqT4 {
    using Top = TopT4<Child>;
    static constexpr bool IS_SEQ = true;
    static constexpr bool FROM_MEM = MEM;
    static constexpr int NP = 7;
    static constexpr int S1 = Child::S;
    static constexpr int m = S1 - 3;
    static constexpr int S = 4 * m;
    static constexpr int L = 2 * m;
    static constexpr int R_WORDS = 8 * m;
    static constexpr int IRW = (R_WORDS + NT - 1) / NT;
    static constexpr int CIN_WORDS = Child::IS_SEQ ? 2 * S1 : 0;
    static constexpr int TMP_WORDS = 3 * NWAVE;
    static_assert(Child::SCRATCH >= TMP_WORDS, "child scratch holds the scan scratch");
    // with MEM the product is written over the child's operands and scratch
    static_assert(!MEM || CIN_WORDS + Child::SCRATCH >= R_WORDS, "child operands and scratch hold the product");
    static constexpr int SCRATCH = 5 * L + CIN_WORDS + Child::SCRATCH;
    static constexpr long long BASE = 7 * Child::BASE;
    static constexpr long long OPS = Top::OPS;

    // Fold point product e (2*S1 words) into the numerators and R.
    template <int E>
    __device__ __forceinline__ static void absorb(const u32 *p, u32 (&R)[IRW], u32 *U, u32 *V, u32 *C3, u32 *C1,
                                                  u32 *C2) {
        auto P = [&](int j) -> u32 { return (j >= 0 && j < 2 * S1) ? p[j] : 0u; };
        const int t = tid();
        if constexpr (E == 0 || E == 6) {
            constexpr int at = E == 0 ? 0 : 6 * m;  // c0 at word 0, c6 at word 6m of the product
#pragma unroll
            for (int i = 0; i < IRW; ++i) {
                const int r = t + i * NT;
                if (r >= at && r < at + L) R[i] ^= P(r - at);
            }
        }
        for (int k = t; k < L; k += NT) {
            if constexpr (E == 0) {
                U[k] ^= P(k + 1) ^ P(k - 1) ^ P(k - 3);
                V[k] ^= P(k + 2) ^ P(k - 4);
                C3[k] ^= P(k);
                C2[k] ^= P(k + 2);
            } else if constexpr (E == 1) {
                C3[k] ^= P(k);
            } else if constexpr (E == 2) {
                U[k] ^= P(k + 1);
                V[k] ^= P(k + 2);
                C1[k] ^= P(k + 1);
                C2[k] ^= P(k + 2);
            } else if constexpr (E == 3) {
                U[k] ^= P(k + 1);
                C1[k] ^= P(k + 1);
            } else if constexpr (E == 4) {
                U[k] ^= P(k + 1);
                V[k] ^= P(k + 2);
            } else if constexpr (E == 5) {
                U[k] ^= P(k + 1);
            } else {
                const u32 q = P(k + 1) ^ P(k - 1) ^ P(k - 3);
                U[k] ^= q;
                V[k] ^= P(k + 2) ^ P(k - 4);
                C3[k] ^= P(k);
                C1[k] ^= q;
                C2[k] ^= P(k - 4);
            }
        }
    }

    template <int E, class Src>
    __device__ __forceinline__ static void point(const Src &src, u32 (&R)[IRW], u32 *U, u32 *V, u32 *C3, u32 *C1,
                                                 u32 *C2, u32 *cin, u32 *cs) {
        const u32 *p;
        if constexpr (Child::IS_SEQ) {
            par_map<2 * S1>(cin, [&](int idx) -> u32 {
                const int x = idx / S1;
                return src.get(x, idx - x * S1);
            });
            __syncthreads();
            p = Child::run_ab(cin, cs);
        } else {
            p = Child::run_src(src, cs);
        }
        absorb<E>(p, R, U, V, C3, C1, C2);
        __syncthreads();
    }

    // Divisions and recombination, as in TopT4::interp_store; tmp is the
    // child's scratch (dead now), the 2S-word product goes to out.
    __device__ __forceinline__ static void finish(const u32 (&R)[IRW], u32 *U, u32 *V, u32 *C3, u32 *C1, u32 *C2,
                                                  u32 *tmp, u32 *out) {
        auto A = [&](const u32 *c, int j) -> u32 { return (j >= 0 && j < L) ? c[j] : 0u; };
        const int t = tid();
        scan_xor_stride<L, 3>(U, tmp);
        for (int k = t; k < L; k += NT) V[k] ^= A(U, k + 1) ^ A(U, k - 3);
        __syncthreads();
        scan_xor_stride<L, 2>(V, tmp);
        for (int k = t; k < L; k += NT) C3[k] ^= U[k] ^ V[k];
        __syncthreads();
        for (int k = t; k < L; k += NT)
            C1[k] ^= A(C3, k + 1) ^ A(C3, k) ^ A(C3, k - 1) ^ A(V, k + 1) ^ A(U, k + 1) ^ A(U, k) ^ A(U, k - 3);
        __syncthreads();
        scan_xor_stride<L, 3>(C1, tmp);
        for (int k = t; k < L; k += NT)
            C2[k] ^= A(C3, k - 1) ^ A(V, k - 2) ^ A(U, k - 3) ^ A(C1, k + 1) ^ A(C1, k - 3);
        __syncthreads();
        scan_xor_stride<L, 2>(C2, tmp);  // ends with a barrier: tmp is dead before out is written
#pragma unroll
        for (int i = 0; i < IRW; ++i) {
            const int r = t + i * NT;
            if (r < R_WORDS)
                out[r] = R[i] ^ A(C1, r - m) ^ A(C2, r - 2 * m) ^ A(C3, r - 3 * m) ^ A(V, r - 4 * m) ^
                         A(C2, r - 4 * m) ^ A(U, r - 5 * m) ^ A(C1, r - 5 * m);
        }
        __syncthreads();
    }

    // ab: [a (S) | b (S)] in LDS.  Returns the 2S-word product, written over
    // ab (whose words are dead once the last point has been evaluated).
    __device__ __forceinline__ static u32 *run_ab(u32 *ab, u32 *scratch) {
        u32 *U = scratch;
        u32 *V = U + L;
        u32 *C3 = V + L;
        u32 *C1 = C3 + L;
        u32 *C2 = C1 + L;
        u32 *cin = C2 + L;
        u32 *cs = cin + CIN_WORDS;
        u32 R[IRW];
#pragma unroll
        for (int i = 0; i < IRW; ++i) R[i] = 0;
        for (int k = tid(); k < 5 * L; k += NT) U[k] = 0;
        // (the barriers inside the first child run order these stores before any absorb)
        point<0>(T4Source<0, Top>{ab}, R, U, V, C3, C1, C2, cin, cs);
        point<1>(T4Source<1, Top>{ab}, R, U, V, C3, C1, C2, cin, cs);
        point<2>(T4Source<2, Top>{ab}, R, U, V, C3, C1, C2, cin, cs);
        point<3>(T4Source<3, Top>{ab}, R, U, V, C3, C1, C2, cin, cs);
        point<4>(T4Source<4, Top>{ab}, R, U, V, C3, C1, C2, cin, cs);
        point<5>(T4Source<5, Top>{ab}, R, U, V, C3, C1, C2, cin, cs);
        point<6>(T4Source<6, Top>{ab}, R, U, V, C3, C1, C2, cin, cs);
        finish(R, U, V, C3, C1, C2, cs, ab);
        return ab;
    }

    // The parent's operands a, b (n bits each, u32 words) read from memory;
    // returns the 2S-word product, assembled over the child's operands and
    // scratch.
    __device__ __forceinline__ static u32 *run_mem(const u32 *a, const u32 *b, u32 n, u32 *scratch) {
        u32 *U = scratch;
        u32 *V = U + L;
        u32 *C3 = V + L;
        u32 *C1 = C3 + L;
        u32 *C2 = C1 + L;
        u32 *cin = C2 + L;
        u32 *cs = cin + CIN_WORDS;
        const int w32 = (int)((n + 31u) / 32u);
        const u32 sn = n % 32u;
        const u32 top = sn ? ((1u << sn) - 1u) : 0xFFFFFFFFu;
        u32 R[IRW];
#pragma unroll
        for (int i = 0; i < IRW; ++i) R[i] = 0;
        for (int k = tid(); k < 5 * L; k += NT) U[k] = 0;
        point<0>(T4MemSource<0, Top>{a, b, w32, top}, R, U, V, C3, C1, C2, cin, cs);
        point<1>(T4MemSource<1, Top>{a, b, w32, top}, R, U, V, C3, C1, C2, cin, cs);
        point<2>(T4MemSource<2, Top>{a, b, w32, top}, R, U, V, C3, C1, C2, cin, cs);
        point<3>(T4MemSource<3, Top>{a, b, w32, top}, R, U, V, C3, C1, C2, cin, cs);
        point<4>(T4MemSource<4, Top>{a, b, w32, top}, R, U, V, C3, C1, C2, cin, cs);
        point<5>(T4MemSource<5, Top>{a, b, w32, top}, R, U, V, C3, C1, C2, cin, cs);
        point<6>(T4MemSource<6, Top>{a, b, w32, top}, R, U, V, C3, C1, C2, cin, cs);
        finish(R, U, V, C3, C1, C2, cs, cin);
        return cin;
    }
};

// ------------------------------------------------------------- Toom-Cook 5
// Word-aligned Toom-Cook 5 with x = X^32 (the five-way split with nine
// products of Section 3, Table compToom), spread over workgroups like TopT4.
// The paper gives neither points nor interpolation; the construction used:
//   points 0, 1, x, 1/x, x+1, 1/(x+1), x^2, 1/x^2, inf (the reciprocal points
//   homogenised: x^4 a(1/x), (x+1)^4 a(1/(x+1)), x^8 a(1/x^2)), so a point
//   operand has at most m + 8 words;
//   with c(Y) = c0 + ... + c8 Y^8, the sums E(t) = C(t) + t^8 C(1/t) depend
//   only on s_k = c_k + c_{8-k}: with s0 = c0 + c8 known,
//     G(t) = (E(t) + s0 (1+t)^8) / (t (1+t)^2)
//          = s1 (1 + t^2 + t^4) + s2 (t + t^3) + s3 t^2;
//   at t = x, x+1, x^2 this 3x3 system is solved by exact divisions only:
//     K = G(x) + G(x+1) = s3 + s2 x (1+x),
//     R1 = G(x) + x^2 K,  R3 = G(x^2) + x^4 K,
//     R3 + x R1 = s1 (1+x+x^2)^2 (1+x) (1+x^2+x^3),
//     s2 = (R1 + s1 (1+x^2+x^4)) / (x (1+x^3)),  s3 = K + s2 (x + x^2),
//   where 1/(1+x+x^2)^2 = (1+x^2)/(1+x^6) and 1/(1+x^2+x^3) =
//   (1+x^2+x^3+x^4)/(1+x^7) (x^3+x^2+1 divides x^7+1), so every division is
//   a word shift or a strided prefix XOR (scan_xor_stride, s = 1 ... 7);
//   then c4 = C(1) + s0 + s1 + s2 + s3, and
//     D(t) = C(t) + c0 + c8 t^8 + s1 t^7 + s2 t^6 + s3 t^5 + c4 t^4
//   has the form of E(t) + s0 (1+t)^8 with (c1, c2, c3) in place of
//   (s1, s2, s3): the same solve gives them, and c_{8-k} = s_k + c_k.
// Every intermediate fits in 2 S1 words (S1 = m + 8).
template <class Child>
struct TopT5 {
    static constexpr bool IS_SEQ = true;
    static constexpr bool FROM_MEM = false;
    static constexpr int NP = 9;
    static constexpr int S1 = Child::S;
    static constexpr int m = S1 - 8;
    static constexpr int S = 5 * m;
    static constexpr int LW = 2 * S1;  // words of every intermediate polynomial
    static constexpr int TMP_WORDS = 7 * NWAVE;
    // eight LW-word arrays, the words of the product that the fold shifts
    // down (S + 2), scan scratch
    static constexpr int INTERP_SCRATCH = 8 * LW + (S + 2) + TMP_WORDS;
    static constexpr bool INTERP_STORES = true;  // interp_store writes the result
    // its interpolation kernel keeps to 80 VGPRs, so that six workgroups fit
    // a CU where the LDS allows it (the Toom-5 classes use about 86 otherwise)
    static constexpr int INTERP_WAVES = 6;
    static constexpr long long BASE = 9 * Child::BASE;
    // evaluation about 44 XORs per word of each operand; interpolation about
    // 40 XORs per word of each of its LW-word arrays (24 synchronised passes)
    // and 9 XORs per product word
    static constexpr long long OPS = 9 * Child::OPS + 88LL * S1 + 40LL * LW + 18LL * S;

    // Word w of operand x of point e, from a source of the parent's words.
    template <class Part>
    __device__ __forceinline__ static u32 point_word(int e, int x, int w, const Part &part) {
        auto p = [&](int q, int j) -> u32 { return part(x, q, j); };
        // part q times (x+1)^k at word w
        auto px1 = [&](int q, int k) -> u32 {
            switch (k) {
                case 0: return p(q, w);
                case 1: return p(q, w) ^ p(q, w - 1);
                case 2: return p(q, w) ^ p(q, w - 2);
                case 3: return p(q, w) ^ p(q, w - 1) ^ p(q, w - 2) ^ p(q, w - 3);
                default: return p(q, w) ^ p(q, w - 4);
            }
        };
        switch (e) {
            case 0: return p(0, w);
            case 1: return p(0, w) ^ p(1, w) ^ p(2, w) ^ p(3, w) ^ p(4, w);
            case 2: return p(0, w) ^ p(1, w - 1) ^ p(2, w - 2) ^ p(3, w - 3) ^ p(4, w - 4);
            case 3: return p(0, w - 4) ^ p(1, w - 3) ^ p(2, w - 2) ^ p(3, w - 1) ^ p(4, w);
            case 4: return px1(0, 0) ^ px1(1, 1) ^ px1(2, 2) ^ px1(3, 3) ^ px1(4, 4);
            case 5: return px1(0, 4) ^ px1(1, 3) ^ px1(2, 2) ^ px1(3, 1) ^ px1(4, 0);
            case 6: return p(0, w) ^ p(1, w - 2) ^ p(2, w - 4) ^ p(3, w - 6) ^ p(4, w - 8);
            case 7: return p(0, w - 8) ^ p(1, w - 6) ^ p(2, w - 4) ^ p(3, w - 2) ^ p(4, w);
            default: return p(4, w);
        }
    }

    // For 0 <= j < LW: f(j, v) computes NO values, then dst[o][j] = v[o];
    // every value is computed before any is stored, so f may read the
    // destination arrays at any index.  Ends with a barrier.
    template <int NO, class F>
    __device__ __forceinline__ static void xpass(u32 *const (&dst)[NO], F f) {
        constexpr int IT = (LW + NT - 1) / NT;
        u32 v[IT][NO];
        const int t = tid();
#pragma unroll
        for (int i = 0; i < IT; ++i) {
            const int j = t + i * NT;
#pragma unroll
            for (int o = 0; o < NO; ++o) v[i][o] = 0u;
            if (j < LW) f(j, v[i]);
        }
        __syncthreads();
#pragma unroll
        for (int i = 0; i < IT; ++i) {
            const int j = t + i * NT;
            if (j < LW) {
#pragma unroll
                for (int o = 0; o < NO; ++o) dst[o][j] = v[i][o];
            }
        }
        __syncthreads();
    }

    __device__ __forceinline__ static u32 A(const u32 *c, int j) { return (j >= 0 && j < LW) ? c[j] : 0u; }

    // Given G(x), G(x+1), G(x^2) of the form s1 (1+t^2+t^4) + s2 (t+t^3) +
    // s3 t^2 in gx, gx1, gx2, leaves s1 in gx2, s2 in gx and s3 in k.  K, R1
    // and (R3 + x R1)(1 + x^2) are formed in one pass from the G arrays.
    template <bool ADD>
    __device__ __forceinline__ static void solve3(u32 *gx, u32 *gx1, u32 *gx2, u32 *k, u32 *tmp,
                                                  u32 *const (&add)[3]) {
        auto K = [&](int i) -> u32 { return A(gx, i) ^ A(gx1, i); };
        auto R1 = [&](int i) -> u32 { return A(gx, i) ^ K(i - 2); };
        auto N = [&](int i) -> u32 { return A(gx2, i) ^ K(i - 4) ^ R1(i - 1); };
        {
            u32 *const out[3] = {k, gx, gx2};
            xpass(out, [&](int j, u32 (&v)[3]) {
                v[0] = K(j);
                v[1] = R1(j);
                v[2] = N(j) ^ N(j - 2);  // (R3 + x R1) (1 + x^2)
            });
        }
        scan_xor_stride<LW, 6>(gx2, tmp);
        scan_xor_stride<LW, 1>(gx2, tmp);
        {
            u32 *const out[1] = {gx2};
            xpass(out, [&](int j, u32 (&v)[1]) { v[0] = gx2[j] ^ A(gx2, j - 2) ^ A(gx2, j - 3) ^ A(gx2, j - 4); });
        }
        scan_xor_stride<LW, 7>(gx2, tmp);  // s1
        {
            // s2 = (R1 + s1 (1 + x^2 + x^4)) / x / (1 + x^3)
            u32 *const out[1] = {gx};
            xpass(out, [&](int j, u32 (&v)[1]) {
                const int i = j + 1;
                v[0] = A(gx, i) ^ A(gx2, i) ^ A(gx2, i - 2) ^ A(gx2, i - 4);
            });
        }
        scan_xor_stride<LW, 3>(gx, tmp);  // s2
        if constexpr (ADD) {
            // also add s1, s2, s3 into the arrays at add (in that order)
            u32 *const out[4] = {k, add[0], add[1], add[2]};
            xpass(out, [&](int j, u32 (&v)[4]) {
                v[0] = k[j] ^ A(gx, j - 1) ^ A(gx, j - 2);
                v[1] = add[0][j] ^ gx2[j];
                v[2] = add[1][j] ^ gx[j];
                v[3] = add[2][j] ^ v[0];
            });
        } else {
            u32 *const out[1] = {k};
            xpass(out, [&](int j, u32 (&v)[1]) { v[0] = k[j] ^ A(gx, j - 1) ^ A(gx, j - 2); });  // s3
        }
    }

    // The nine point products (2*S1 words each, in point order) sit at
    // products (any address space).  Interpolates, recombines and stores the
    // product of n-bit operands at c64: the ring product (kind 0: W(n)
    // words) or the full product (2 W(n) words), as TopT4::interp_store.
    __device__ __forceinline__ static void interp_store(const u32 *products, u32 *scratch, u32 n, u32 kind,
                                                        uint64_t *c64) {
        u32 *a0 = scratch;
        u32 *a1 = a0 + LW;
        u32 *a2 = a1 + LW;
        u32 *a3 = a2 + LW;
        u32 *a4 = a3 + LW;
        u32 *a5 = a4 + LW;
        u32 *a6 = a5 + LW;
        u32 *a7 = a6 + LW;
        u32 *H = a7 + LW;
        u32 *tmp = H + S + 2;
        auto P = [&](int e, int j) -> u32 { return (j >= 0 && j < 2 * S1) ? products[e * 2 * S1 + j] : 0u; };
        auto s0 = [&](int j) -> u32 { return P(0, j) ^ P(8, j); };
        // Every read of the products, in one pass: E(t) + s0 (1+t)^8 at t = x,
        // x+1, x^2 divided at once by x, x^2, x^2 (word shifts) into a0..a2,
        // and the parts of c4 and of D(t) that the products give: C(1) + s0
        // into a4, D(t) less its c4..c7 terms at t = x, x+1, x^2 into a5..a7.
        {
            auto E0 = [&](int i) -> u32 { return P(2, i) ^ P(3, i) ^ s0(i) ^ s0(i - 8); };
            auto E1 = [&](int i) -> u32 { return P(4, i) ^ P(5, i) ^ s0(i - 8); };
            auto E2 = [&](int i) -> u32 { return P(6, i) ^ P(7, i) ^ s0(i) ^ s0(i - 16); };
            u32 *const out[7] = {a0, a1, a2, a4, a5, a6, a7};
            xpass(out, [&](int j, u32 (&v)[7]) {
                v[0] = E0(j + 1);
                v[1] = E1(j + 2);
                v[2] = E2(j + 2);
                v[3] = P(1, j) ^ s0(j);
                v[4] = P(2, j) ^ P(0, j) ^ P(8, j - 8);
                v[5] = P(4, j) ^ s0(j) ^ P(8, j - 8);
                v[6] = P(6, j) ^ P(0, j) ^ P(8, j - 16);
            });
        }
        // then by 1 + x^2, 1 + x and 1 + x^4: G(t)
        scan_xor_stride3<LW, 2, 1, 4>(a0, a1, a2, tmp);
        u32 *const none[3] = {nullptr, nullptr, nullptr};
        solve3<false>(a0, a1, a2, a3, tmp, none);  // s1 = a2, s2 = a0, s3 = a3
        const u32 *s1 = a2, *s2 = a0, *s3 = a3;
        // c4 = C(1) + s0 + s1 + s2 + s3 into a4, and q = (1 + x^2) s1 +
        // (1 + x) s2 + s3 into a1, so that s1 (x+1)^7 + s2 (x+1)^6 + s3 (x+1)^5
        // = (1 + x)(1 + x^4) q
        {
            u32 *const out[2] = {a4, a1};
            xpass(out, [&](int j, u32 (&v)[2]) {
                const u32 t3 = s1[j] ^ s2[j] ^ s3[j];
                v[0] = a4[j] ^ t3;
                v[1] = t3 ^ A(s1, j - 2) ^ A(s2, j - 1);
            });
        }
        // D(t) at x, x+1, x^2, divided by the same word shifts, into a5, a1, a7
        {
            const u32 *c4 = a4, *q = a1;
            u32 *const out[3] = {a5, a1, a7};
            xpass(out, [&](int j, u32 (&v)[3]) {
                int i = j + 1;
                v[0] = A(a5, i) ^ A(s1, i - 7) ^ A(s2, i - 6) ^ A(s3, i - 5) ^ A(c4, i - 4);
                i = j + 2;
                v[1] = A(a6, i) ^ A(c4, i) ^ A(c4, i - 4) ^ A(q, i) ^ A(q, i - 1) ^ A(q, i - 4) ^ A(q, i - 5);
                v[2] = A(a7, i) ^ A(s1, i - 14) ^ A(s2, i - 12) ^ A(s3, i - 10) ^ A(c4, i - 8);
            });
        }
        scan_xor_stride3<LW, 2, 1, 4>(a5, a1, a7, tmp);
        // c1 = a7, c2 = a5, c3 = a6; c7 = s1 + c1, c6 = s2 + c2 and
        // c5 = s3 + c3 replace s1, s2, s3 in a2, a0, a3
        u32 *const sums[3] = {a2, a0, a3};
        solve3<true>(a5, a1, a7, a6, tmp, sums);
        const int t = tid();
        // recomposition: word r of c0 + c1 Y + ... + c8 Y^8 (Y = x^m); zero
        // outside [0, 2S)
        auto word = [&](int r) -> u32 {
            if (r < 0 || r >= 2 * S) return 0u;
            u32 w = P(0, r);
            w ^= A(a7, r - m);
            w ^= A(a5, r - 2 * m);
            w ^= A(a6, r - 3 * m);
            w ^= A(a4, r - 4 * m);
            w ^= A(a3, r - 5 * m);
            w ^= A(a0, r - 6 * m);
            w ^= A(a2, r - 7 * m);
            w ^= P(8, r - 8 * m);
            return w;
        };
        u32 *c32 = reinterpret_cast<u32 *>(c64);
        const int W64 = (int)((n + 63u) / 64u);
        if (kind == 0u) {
            const int w32 = (int)((n + 31u) / 32u);
            const int q = (int)(n / 32u);
            const u32 sn = n % 32u;
            const u32 top = sn ? ((1u << sn) - 1u) : 0xFFFFFFFFu;
            for (int k = t; k <= w32; k += NT) H[k] = word(k + q);  // w32 <= S
            __syncthreads();
            for (int k = t; k < 2 * W64; k += NT) {
                u32 v = 0;
                if (k < w32) {
                    v = word(k) ^ __builtin_amdgcn_alignbit(H[k + 1], H[k], sn);
                    if (k == w32 - 1) v &= top;
                }
                c32[k] = v;
            }
        } else {
            for (int k = t; k < 4 * W64; k += NT) c32[k] = word(k);
        }
        __syncthreads();
    }
};

// ------------------------------------- N-way Karatsuba (Appendix A, karat3/5)
// Operands of S = N S1 words split as a = sum a_i Y^i, Y = X^{32 S1}.  The
// N(N+1)/2 products P_ii = a_i b_i and P_ij = (a_i + a_j)(b_i + b_j), i < j,
// give every coefficient: c_k = [k even] P_{k/2,k/2} + sum over i < j with
// i + j = k of (P_ij + P_ii + P_jj).  So P_ij (i < j) is added at Y^{i+j},
// and P_ii at Y^{2i} and at Y^{i+j} for every j != i.  The products are
// computed one after another by Child and added into the result
// accumulator R (2S words, in registers) as soon as they exist.
template <int N, class Child>
struct SeqKN {
    static constexpr bool IS_SEQ = true;
    static constexpr bool FROM_MEM = false;
    static constexpr int NP = N * (N + 1) / 2;
    static constexpr int S1 = Child::S;
    static constexpr int S = N * S1;
    static constexpr int R_WORDS = 2 * S;
    static constexpr int IRW = (R_WORDS + NT - 1) / NT;
    static constexpr int CIN_WORDS = Child::IS_SEQ ? 2 * S1 : 0;
    static constexpr int SCRATCH = CIN_WORDS + Child::SCRATCH;
    static constexpr long long BASE = NP * Child::BASE;
    // evaluation: one XOR per word of the N(N-1)/2 sum operands (2 S1 each);
    // absorption: N offsets for each P_ii, one for each P_ij, 2 S1 words each
    static constexpr long long OPS =
        NP * Child::OPS + (long long)N * (N - 1) * S1 + 2LL * S1 * ((long long)N * N + N * (N - 1) / 2);

    template <int I, int J>
    struct Src {
        const u32 *ab;
        __device__ __forceinline__ u32 get(int x, int w) const {
            const u32 *o = ab + x * S;
            if constexpr (I == J) return o[I * S1 + w];
            else return o[I * S1 + w] ^ o[J * S1 + w];
        }
    };

    // P (2 S1 words) added to R at word offset Y^k, for each k with bit k of MASK set
    template <unsigned MASK>
    __device__ __forceinline__ static void absorb(const u32 *p, u32 (&R)[IRW]) {
        const int t = tid();
#pragma unroll
        for (int i = 0; i < IRW; ++i) {
            const int r = t + i * NT;
            u32 v = 0;
#pragma unroll
            for (int k = 0; k < 2 * N - 1; ++k) {
                if ((MASK >> k) & 1u) {
                    const int j = r - k * S1;
                    if (j >= 0 && j < 2 * S1) v ^= p[j];
                }
            }
            if (r < R_WORDS) R[i] ^= v;
        }
    }

    template <int I, int J>
    static constexpr unsigned offsets() {
        if constexpr (I != J) {
            return 1u << (I + J);
        } else {
            unsigned mk = 1u << (2 * I);
            for (int j = 0; j < N; ++j)
                if (j != I) mk |= 1u << (I + j);
            return mk;
        }
    }

    template <int I, int J>
    __device__ __forceinline__ static void product(u32 *ab, u32 (&R)[IRW], u32 *cin, u32 *cs) {
        const Src<I, J> src{ab};
        const u32 *p;
        if constexpr (Child::IS_SEQ) {
            par_map<2 * S1>(cin, [&](int idx) -> u32 {
                const int x = idx / S1;
                return src.get(x, idx - x * S1);
            });
            __syncthreads();
            p = Child::run_ab(cin, cs);
        } else {
            p = Child::run_src(src, cs);
        }
        absorb<offsets<I, J>()>(p, R);
        __syncthreads();
    }

    template <int I, int J>
    __device__ __forceinline__ static void products(u32 *ab, u32 (&R)[IRW], u32 *cin, u32 *cs) {
        if constexpr (I < N) {
            product<I, J>(ab, R, cin, cs);
            if constexpr (J + 1 < N) products<I, J + 1>(ab, R, cin, cs);
            else products<I + 1, I + 1>(ab, R, cin, cs);
        }
    }

    // ab: [a (S) | b (S)] in LDS.  Returns the 2S-word product, written over
    // ab (whose words are dead once the last product has been computed).
    __device__ __forceinline__ static u32 *run_ab(u32 *ab, u32 *scratch) {
        u32 *cin = scratch;
        u32 *cs = cin + CIN_WORDS;
        u32 R[IRW];
#pragma unroll
        for (int i = 0; i < IRW; ++i) R[i] = 0;
        products<0, 0>(ab, R, cin, cs);
        const int t = tid();
#pragma unroll
        for (int i = 0; i < IRW; ++i) {
            const int r = t + i * NT;
            if (r < R_WORDS) ab[r] = R[i];
        }
        __syncthreads();
        return ab;
    }
};

}  // namespace gf2x
