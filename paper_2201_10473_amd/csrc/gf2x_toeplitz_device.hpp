// gf2x_toeplitz_device.hpp -- a batch h * r_i mod (X^n - 1) with one shared operand h,
// computed as one matrix product on the int8 matrix cores.
//
// By the circulant / ring isomorphism (Section 1), h * r mod (X^n - 1) is the
// matrix-vector product T r over F2 with T[k][j] = h_{(k - j) mod n} (the
// circulant whose first column is h).  For a batch, C = T [r_1 ... r_B] is a
// matrix product.  Bits become 0/1 int8 values, the matrix cores sum the
// n products of each output in int32 (exact: a count is at most n < 2^31),
// and the output bit is the count's parity.
//
// Kernel layout (gfx950, v_mfma_i32_16x16x64_i8):
//   * workgroup = 4 waves; tile = 256 output bits (rows k) x 64 batch items;
//     each wave owns 64 rows (4 row tiles of 16) x 64 items (4 column tiles).
//   * K steps of 128 bits: each lane group g = lane/16 covers 32 consecutive
//     j; a 32-bit word of bits is spread to 8 dwords of 0/1 bytes by
//     (x >> q) & 0x01010101, q = 0..7 (byte b of dword q = bit 8b + q); the
//     first MFMA takes dwords 0-3, the second 4-7.  A and B use the same
//     spreading, so every j meets its partner in exactly one MFMA.
//   * T fragments are built in registers from a reversed, extended bit image
//     of h staged in LDS (32-bit window + funnel shift per row).
//   * batch bits are spread once per K step into an LDS tile shared by the
//     four waves (double buffered, rows padded to avoid bank conflicts).
// Constant time: addresses depend on n, the tile indices and the lane only.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "gf2x_toeplitz.hpp"

namespace gf2x {
namespace toeplitz {

typedef uint32_t u32;
typedef int v4i __attribute__((ext_vector_type(4)));


// Dword d of the bit image of h read by the tiles: bit q = 32 d + m is
// h_{(P - q) mod n}, so that row k of T, read left to right from column j,
// is the increasing window starting at bit P - k + j.
__device__ __forceinline__ u32 hr_dword(const uint64_t *h, u32 n, u32 P, u32 d) {
    u32 v = 0;
    for (u32 m = 0; m < 32; ++m) {
        const long long q = (long long)d * 32 + m;
        long long pos = ((long long)P - q) % (long long)n;
        if (pos < 0) pos += n;
        v |= (u32)((h[pos >> 6] >> (pos & 63)) & 1u) << m;
    }
    return v;
}

__device__ __forceinline__ void spread8(u32 x, u32 (&out)[8]) {
#pragma unroll
    for (int q = 0; q < 8; ++q) out[q] = (x >> q) & 0x01010101u;
}

// One K step of one batch item column: 32 bits of r_i at bit j, masked to n.
__device__ __forceinline__ u32 load_r_bits(const u32 *r32, u32 words32, u32 n, u32 j) {
    const u32 d = j >> 5;
    if (d >= words32 || j >= n) return 0u;
    u32 y = r32[d];
    if (n - j < 32u) y &= (1u << (n - j)) - 1u;
    return y;
}

// One workgroup tile (bx: block of 256 output bits, by: block of 64 items).
__device__ __forceinline__ void toeplitz_tile(const u32 *hr, u32 hr_dwords, u32 n, u32 P, const uint64_t *r_base,
                                              const uint64_t *b_off, uint64_t *c_base, const uint64_t *c_off,
                                              u32 count, u32 bx, u32 by, u32 *lds) {
    const u32 W = (n + 63u) / 64u;
    const u32 words32 = 2u * W;
    const u32 steps = (n + kStepBits - 1) / kStepBits;
    const u32 t = threadIdx.x;
    const u32 lane = t & 63u, wave = t >> 6;
    const u32 g = lane >> 4, lr = lane & 15u;
    const u32 k_wg = bx * kRowsWG;
    const u32 col0 = by * kColsWG;

    // -- stage the window of hr this workgroup reads
    // q ranges over [P - (k_wg + 255), P - k_wg + 128*(steps-1) + 96 + 31]
    const u32 q_lo = P - (k_wg + kRowsWG - 1);
    const u32 d_lo = q_lo >> 5;
    const u32 d_hi = (P - k_wg + kStepBits * (steps - 1) + 96u + 31u) / 32u + 1u;
    const u32 hr_len = d_hi - d_lo + 1u;
    u32 *hrL = lds;
    u32 *tile0 = lds + ((hr_len + 3u) & ~3u);
    u32 *tile1 = tile0 + kTileDwords;
    for (u32 i = t; i < hr_len; i += 256u) hrL[i] = (d_lo + i < hr_dwords) ? hr[d_lo + i] : 0u;

    // -- this thread's batch column for the spread step
    const u32 scol = t >> 2, sg = t & 3u;
    const u32 item = col0 + scol;
    const u32 *r32 = (item < count) ? reinterpret_cast<const u32 *>(r_base + b_off[item]) : nullptr;
    auto spread_step = [&](u32 s, u32 *tile) {
        const u32 y = r32 ? load_r_bits(r32, words32, n, s * kStepBits + 32u * sg) : 0u;
        u32 e[8];
        spread8(y, e);
        v4i *dst = reinterpret_cast<v4i *>(tile + scol * kColStride + sg * 8u);
        dst[0] = v4i{(int)e[0], (int)e[1], (int)e[2], (int)e[3]};
        dst[1] = v4i{(int)e[4], (int)e[5], (int)e[6], (int)e[7]};
    };
    spread_step(0, tile0);
    __syncthreads();

    v4i acc[4][4];
#pragma unroll
    for (int mt = 0; mt < 4; ++mt)
#pragma unroll
        for (int nt = 0; nt < 4; ++nt) acc[mt][nt] = v4i{0, 0, 0, 0};

    const u32 k_wave = k_wg + 64u * wave;
    for (u32 s = 0; s < steps; ++s) {
        u32 *cur = (s & 1u) ? tile1 : tile0;
        u32 *nxt = (s & 1u) ? tile0 : tile1;
        // T fragments: row k, bits j = 128 s + 32 g + m  ->  window of hr at
        // q0 = P - k + 128 s + 32 g
        u32 a[4][8];
#pragma unroll
        for (int mt = 0; mt < 4; ++mt) {
            const u32 k = k_wave + 16u * mt + lr;
            const u32 q0 = P - k + kStepBits * s + 32u * g;
            const u32 i0 = (q0 >> 5) - d_lo;
            const u32 x = __builtin_amdgcn_alignbit(hrL[i0 + 1], hrL[i0], q0 & 31u);
            spread8(x, a[mt]);
        }
        v4i b[4][2];
#pragma unroll
        for (int nt = 0; nt < 4; ++nt) {
            const v4i *src = reinterpret_cast<const v4i *>(cur + (16u * nt + lr) * kColStride + g * 8u);
            b[nt][0] = src[0];
            b[nt][1] = src[1];
        }
#pragma unroll
        for (int mt = 0; mt < 4; ++mt) {
            const v4i a0 = v4i{(int)a[mt][0], (int)a[mt][1], (int)a[mt][2], (int)a[mt][3]};
            const v4i a1 = v4i{(int)a[mt][4], (int)a[mt][5], (int)a[mt][6], (int)a[mt][7]};
#pragma unroll
            for (int nt = 0; nt < 4; ++nt) {
                acc[mt][nt] = __builtin_amdgcn_mfma_i32_16x16x64_i8(a0, b[nt][0], acc[mt][nt], 0, 0, 0);
                acc[mt][nt] = __builtin_amdgcn_mfma_i32_16x16x64_i8(a1, b[nt][1], acc[mt][nt], 0, 0, 0);
            }
        }
        if (s + 1 < steps) spread_step(s + 1, nxt);
        __syncthreads();
    }

    // -- parity of the counts, packed: lane (g, lr) of column tile nt holds rows
    // 16 mt + 4 g + r of item 16 nt + lr
    const u32 word = k_wave / 64u;
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) {
        u32 lo = 0, hi = 0;
#pragma unroll
        for (int mt = 0; mt < 4; ++mt)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const u32 bit = (u32)acc[mt][nt][r] & 1u;
                const u32 pos = 16u * mt + 4u * g + r;
                if (pos < 32u) lo |= bit << pos;
                else hi |= bit << (pos - 32u);
            }
        lo |= __shfl_xor(lo, 16, 64);
        hi |= __shfl_xor(hi, 16, 64);
        lo |= __shfl_xor(lo, 32, 64);
        hi |= __shfl_xor(hi, 32, 64);
        const u32 it = col0 + 16u * nt + lr;
        if (g == 0 && it < count && word < W) {
            uint64_t v = ((uint64_t)hi << 32) | lo;
            const u32 rem = n - 64u * word;
            if (rem < 64u) v &= (((uint64_t)1) << rem) - 1u;
            c_base[c_off[it] + word] = v;
        }
    }
}

}  // namespace toeplitz
}  // namespace gf2x
