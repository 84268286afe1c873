// Stand-in for <hip/hip_runtime.h> used only by the CPU emulation harness:
// it lets the library's device headers compile with g++ so that one
// workgroup's algorithm can be run by NT host threads.  Each workgroup
// thread is an OS thread; __syncthreads is a pthread barrier; __shfl_up
// exchanges through a shared array between two barriers (every call site in
// the library is reached by all threads of the workgroup).  The gfx950
// builtins are given their documented bitwise meaning.
#pragma once
#include <stdint.h>

#define __device__
#define __host__
#define __global__
#define __forceinline__ inline
#define __launch_bounds__(x)

typedef int hipError_t;
typedef struct ihipStream_t *hipStream_t;
typedef struct ihipEvent_t *hipEvent_t;

struct EmuIdx {
    unsigned x, y, z;
};
extern thread_local EmuIdx threadIdx;

void __syncthreads();
unsigned __shfl_up(unsigned v, int delta, int width);
unsigned __shfl_xor(unsigned v, int mask, int width);
// Cross-lane moves within a wave of 64 emulated lanes (every lane of the
// workgroup reaches every call): ds_bpermute returns the value of lane
// (addr / 4) mod 64; the DPP wave rotations move values one lane up
// (wave_ror:1, lane l receives lane l - 1) or down (wave_rol:1).
int emu_ds_bpermute(int addr, int v);
int emu_update_dpp(int old, int v, int ctrl);
#define __builtin_amdgcn_ds_bpermute(addr, v) emu_ds_bpermute((addr), (v))
#define __builtin_amdgcn_update_dpp(old, v, ctrl, rm, bm, bc) emu_update_dpp((old), (v), (ctrl))
#define __builtin_amdgcn_mov_dpp(v, ctrl, rm, bm, bc) emu_update_dpp(0, (v), (ctrl))

// v_mfma_i32_16x16x64_i8 for one wave of 64 emulated lanes (all lanes of the
// workgroup reach every call): lane l supplies A[l%16][16*(l/16) + byte],
// B[16*(l/16) + byte][l%16] and receives C[4*(l/16) + r][l%16] -- the layout
// measured on gfx950.
typedef int emu_v4i __attribute__((ext_vector_type(4)));
emu_v4i emu_mfma_i32_16x16x64_i8(emu_v4i a, emu_v4i b, emu_v4i c);
#define __builtin_amdgcn_mfma_i32_16x16x64_i8(a, b, c, x, y, z) emu_mfma_i32_16x16x64_i8((a), (b), (c))

// v_bitop3_b32: bit k of the result is bit (4*S0_k + 2*S1_k + S2_k) of imm.
static inline uint32_t emu_bitop3(uint32_t s0, uint32_t s1, uint32_t s2, unsigned imm) {
    uint32_t r = 0;
    for (unsigned idx = 0; idx < 8; ++idx)
        if ((imm >> idx) & 1u)
            r |= ((idx & 4) ? s0 : ~s0) & ((idx & 2) ? s1 : ~s1) & ((idx & 1) ? s2 : ~s2);
    return r;
}
// v_bfe_i32: sign-extended field of `width` bits at `offset`.
static inline int emu_sbfe(int a, int offset, int width) {
    const uint32_t u = ((uint32_t)a >> (offset & 31)) & ((width >= 32) ? 0xFFFFFFFFu : ((1u << width) - 1u));
    return (width < 32 && ((u >> (width - 1)) & 1u)) ? (int)(u | ~((1u << width) - 1u)) : (int)u;
}
// v_alignbit_b32: low 32 bits of {hi, lo} >> (s mod 32).
static inline uint32_t emu_alignbit(uint32_t hi, uint32_t lo, uint32_t s) {
    return (uint32_t)(((((uint64_t)hi) << 32) | lo) >> (s & 31u));
}
#ifndef __HIP_MEMORY_SCOPE_WORKGROUP
#define __HIP_MEMORY_SCOPE_WORKGROUP 3
#endif
static inline uint32_t emu_atomic_xor(uint32_t *p, uint32_t v) { return __atomic_fetch_xor(p, v, __ATOMIC_RELAXED); }
#define __hip_atomic_fetch_xor(p, v, order, scope) emu_atomic_xor((p), (v))
#define __builtin_amdgcn_bitop3_b32(a, b, c, imm) emu_bitop3((a), (b), (c), (imm))
#define __builtin_amdgcn_sbfe(a, o, w) emu_sbfe((a), (o), (w))
#define __builtin_amdgcn_alignbit(h, l, s) emu_alignbit((h), (l), (s))
