"""The device algorithm of every schedule class, run on the CPU.

The library's device headers are compiled with g++ behind a stand-in
hip/hip_runtime.h (tests/emu): one workgroup is NT host threads with a
pthread barrier for __syncthreads.  Products are compared bit for bit with
the oracle.  This checks the Karatsuba / Toom-3 bookkeeping, the fold and
the staging logic without a GPU (it does not check gfx950 code generation,
which the GPU tests do)."""
import ctypes
import os
import subprocess

import numpy as np
import pytest

import oracle
from paper_2201_10473_amd import inputs

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def emu(tmp_path_factory):
    so = str(tmp_path_factory.mktemp("emu") / "libemu.so")
    subprocess.check_call(
        ["/opt/rocm/llvm/bin/clang++", "-O2", "-std=c++17", "-fPIC", "-shared", "-pthread", "-Wno-unknown-pragmas",
         "-I", os.path.join(ROOT, "tests", "emu"), "-I", os.path.join(ROOT, "include"),
         "-I", os.path.join(ROOT, "paper_2201_10473_amd", "csrc"),
         os.path.join(ROOT, "tests", "emu", "emu.cpp"), "-o", so]
    )
    lib = ctypes.CDLL(so)
    u64p = ctypes.POINTER(ctypes.c_uint64)
    lib.emu_mul.argtypes = [ctypes.c_int, u64p, u64p, u64p, ctypes.c_uint32, ctypes.c_uint32]
    lib.emu_class_words.argtypes = [ctypes.c_int]
    lib.emu_toeplitz.argtypes = [u64p, ctypes.c_uint32, u64p, u64p, ctypes.c_uint32]
    lib.emu_staged.argtypes = [ctypes.c_int, u64p, u64p, u64p, ctypes.c_uint32, ctypes.c_uint32]
    lib.emu_staged_words.argtypes = [ctypes.c_int]
    lib.emu_sparse.argtypes = [ctypes.c_int, ctypes.c_int, u64p, ctypes.POINTER(ctypes.c_uint32), ctypes.c_uint32,
                               u64p, ctypes.c_uint32]
    lib.emu_sparse_words_per_lane.argtypes = [ctypes.c_int]
    return lib


def _run(lib, cls, n, seed):
    u64p = ctypes.POINTER(ctypes.c_uint64)
    a = inputs.dense(n, seed, cls, 0)
    b = inputs.dense(n, seed, cls, 1)
    W = oracle.words(n)
    c = np.zeros(W, dtype=np.uint64)
    f = np.zeros(2 * W, dtype=np.uint64)
    lib.emu_mul(cls, a.ctypes.data_as(u64p), b.ctypes.data_as(u64p), c.ctypes.data_as(u64p), n, 0)
    lib.emu_mul(cls, a.ctypes.data_as(u64p), b.ctypes.data_as(u64p), f.ctypes.data_as(u64p), n, 1)
    assert np.array_equal(c, oracle.mul_cyclic(a, b, n)), (cls, n)
    assert np.array_equal(f, oracle.mul(a, b, n)), (cls, n)


# classes 19 and 20 (three Toom-3 levels) take ~15 s each on the CPU and are
# covered on the GPU by test_every_schedule_class
@pytest.mark.parametrize("cls", list(range(19)) + list(range(21, 41)))
def test_class_full_and_ragged(emu, cls):
    S = emu.emu_class_words(cls)
    for n in sorted({S * 32, max(1, S * 32 - 37)}):
        _run(emu, cls, n, 12)


@pytest.mark.parametrize("n,count", [(1, 3), (37, 5), (127, 70), (300, 9), (700, 3)])
def test_toeplitz_tile(emu, n, count):
    """The shared-operand MFMA tile with an emulated 16x16x64 int8 matrix
    instruction (layout as measured on gfx950); bits above n are ignored."""
    u64p = ctypes.POINTER(ctypes.c_uint64)
    W = oracle.words(n)
    h = inputs.dense(n, 3, n, 0)
    R = inputs.dense_batch(n, count, 3, 1)
    R[:, -1] |= ~inputs.top_mask(n)
    C = np.full((count, W), 0x5A5A5A5A5A5A5A5A, dtype=np.uint64)
    emu.emu_toeplitz(h.ctypes.data_as(u64p), n, R.ctypes.data_as(u64p), C.ctypes.data_as(u64p), count)
    R[:, -1] &= inputs.top_mask(n)
    for i in range(count):
        assert np.array_equal(C[i], oracle.mul_cyclic(h, R[i], n)), i


@pytest.mark.parametrize("which", [0, 3, 4, 6, 7, 8, 9, 10])
def test_staged_top_level(emu, which):
    """Top Toom-3 (which < 6), Toom-4 (6 <= which < 9) or Toom-5 (which >= 9)
    level spread over workgroups: evaluation words, the five, seven or nine
    point products by the child class, interpolation and fold."""
    u64p = ctypes.POINTER(ctypes.c_uint64)
    S = emu.emu_staged_words(which)
    for n in (S * 32, S * 32 - 37):
        a = inputs.dense(n, 21, which, 0)
        b = inputs.dense(n, 21, which, 1)
        a[-1] |= ~inputs.top_mask(n)
        W = oracle.words(n)
        c = np.zeros(W, dtype=np.uint64)
        f = np.zeros(2 * W, dtype=np.uint64)
        emu.emu_staged(which, a.ctypes.data_as(u64p), b.ctypes.data_as(u64p), c.ctypes.data_as(u64p), n, 0)
        emu.emu_staged(which, a.ctypes.data_as(u64p), b.ctypes.data_as(u64p), f.ctypes.data_as(u64p), n, 1)
        a[-1] &= inputs.top_mask(n)
        assert np.array_equal(c, oracle.mul_cyclic(a, b, n))
        assert np.array_equal(f, oracle.mul(a, b, n))


def _sparse_dense(pos, n):
    s = np.zeros(oracle.words(n), dtype=np.uint64)
    for p in pos:
        p = int(p) % n
        s[p // 64] ^= np.uint64(1) << np.uint64(p % 64)
    return s


@pytest.mark.parametrize("which,nw", [(i, 1) for i in range(8)] + [(1, 4), (6, 4)])
def test_sparse_barrel(emu, which, nw):
    """Dense x sparse ring product by the rotation barrel, one emulated wave
    (or four sharing the positions) with emulated DPP and ds_bpermute lane
    moves: the largest and a smaller n of each sparse class, positions that
    repeat or exceed n, weight 0."""
    u64p = ctypes.POINTER(ctypes.c_uint64)
    u32p = ctypes.POINTER(ctypes.c_uint32)
    R = emu.emu_sparse_words_per_lane(which)
    nmax = 32 * ((64 * R - 2) // 2)
    rng = np.random.default_rng(which)
    for n in sorted({nmax, max(1, nmax // 2 - 37), 33 if which == 0 else nmax - 1}):
        a = inputs.dense(n, 31, which, 0)
        a[-1] |= ~inputs.top_mask(n)
        for pos in (list(rng.integers(0, n, 5)) + [0, n - 1, n, 0xFFFFFFFF, 7 % n, 7 % n], []):
            p32 = np.asarray(pos, dtype=np.uint32)
            c = np.full(oracle.words(n), 0x5A5A5A5A5A5A5A5A, dtype=np.uint64)
            rc = emu.emu_sparse(which, nw, a.ctypes.data_as(u64p), p32.ctypes.data_as(u32p), len(p32),
                                c.ctypes.data_as(u64p), n)
            assert rc == 0
            ref = oracle.mul_cyclic(a & np.append(np.full(len(a) - 1, ~np.uint64(0)), inputs.top_mask(n)),
                                    _sparse_dense(pos, n), n)
            assert np.array_equal(c, ref), (which, nw, n, len(pos))
