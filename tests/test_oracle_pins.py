"""Pins of the CPU oracle against facts that do not come from the oracle itself:
bit-level brute force, the paper's worked example, closed forms and ring
invariants.  CPU only."""
import os
import random

import numpy as np
import pytest

import oracle
from paper_2201_10473_amd import inputs
from tests import brute

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
RING_SIZES = inputs.RING_SIZES


def _rand_words(rng, n):
    x = rng.getrandbits(n) if n else 0
    return x, brute.int_to_words(x, oracle.words(n))


# ---------------------------------------------------------------- clmul64
def test_clmul64_exhaustive_8bit():
    for x in range(256):
        for y in range(256):
            lo, hi = oracle.clmul64(x, y)
            assert hi == 0
            assert lo == brute.clmul_bitloop(x, y), (x, y)


def test_clmul64_random_64bit():
    rng = random.Random(1)
    for _ in range(3000):
        x, y = rng.getrandbits(64), rng.getrandbits(64)
        lo, hi = oracle.clmul64(x, y)
        assert lo | (hi << 64) == brute.clmul_bitloop(x, y)


def test_clmul64_identities():
    rng = random.Random(2)
    for _ in range(200):
        x, y = rng.getrandbits(64), rng.getrandbits(64)
        assert oracle.clmul64(x, 1) == (x, 0)
        assert oracle.clmul64(x, y) == oracle.clmul64(y, x)
        for k in (0, 1, 31, 32, 63):
            lo, hi = oracle.clmul64(x, 1 << k)
            assert lo | (hi << 64) == x << k
    # top bits meet: X^63 * X^63 = X^126
    assert oracle.clmul64(1 << 63, 1 << 63) == (0, 1 << 62)


# ---------------------------------------------------------------- full product
@pytest.mark.parametrize("n", list(range(1, 131)) + [191, 192, 193, 255, 256, 257])
def test_full_product_matches_bitloop(n):
    rng = random.Random(1000 + n)
    for _ in range(3):
        x, a = _rand_words(rng, n)
        y, b = _rand_words(rng, n)
        c = oracle.mul(a, b, n)
        assert c.shape == (2 * oracle.words(n),)
        assert brute.words_to_int(c) == brute.clmul_bitloop(x, y)


@pytest.mark.parametrize("n", range(1, 9))
def test_full_product_exhaustive_tiny(n):
    for x in range(1 << n):
        a = brute.int_to_words(x, 1)
        for y in range(1 << n):
            c = oracle.mul(a, brute.int_to_words(y, 1), n)
            assert int(c[0]) == brute.clmul_bitloop(x, y) and int(c[1]) == 0


def test_input_bits_above_n_are_ignored():
    rng = random.Random(7)
    for n in (1, 5, 63, 64, 65, 100, 12323):
        x, a = _rand_words(rng, n)
        y, b = _rand_words(rng, n)
        W = oracle.words(n)
        junk_a, junk_b = a.copy(), b.copy()
        if n % 64:
            junk_a[-1] |= np.uint64(~((1 << (n % 64)) - 1) & 0xFFFFFFFFFFFFFFFF)
            junk_b[-1] |= np.uint64(0xFFFFFFFFFFFFFFFF << (n % 64) & 0xFFFFFFFFFFFFFFFF)
        assert np.array_equal(oracle.mul(junk_a, junk_b, n), oracle.mul(a, b, n))
        assert np.array_equal(oracle.mul_cyclic(junk_a, junk_b, n), oracle.mul_cyclic(a, b, n))
        c = oracle.mul(a, b, n)
        assert brute.words_to_int(c) >> max(2 * n - 1, 0) == 0
        assert c.shape == (2 * W,)


def test_paper_exact_division_example():
    """Section 3.2 toy example: P = Q * (X+1) and (X+1) * (X+1)^{-1} = 1 mod X^8."""
    vals = {}
    with open(os.path.join(GOLDEN, "paper_exact_division_example.txt")) as f:
        for line in f:
            line = line.strip()
            if line and not line.startswith("#"):
                k, v = line.split()
                vals[k] = int(v, 0)
    P, Q, INV, D = vals["P"], vals["Q"], vals["INV"], vals["D"]
    w = lambda v: brute.int_to_words(v, 1)
    c = oracle.mul(w(Q), w(0x3), D)
    assert int(c[0]) == P
    c = oracle.mul(w(P), w(INV), D)
    assert int(c[0]) & ((1 << D) - 1) == Q
    c = oracle.mul(w(0x3), w(INV), D)
    assert int(c[0]) & ((1 << D) - 1) == 1


# ---------------------------------------------------------------- ring product
@pytest.mark.parametrize("n", list(range(1, 70)) + [127, 128, 129, 191, 193])
def test_cyclic_matches_bitloop(n):
    rng = random.Random(5000 + n)
    for _ in range(3):
        x, a = _rand_words(rng, n)
        y, b = _rand_words(rng, n)
        r = oracle.mul_cyclic(a, b, n)
        assert r.shape == (oracle.words(n),)
        assert brute.words_to_int(r) == brute.cyclic_bitloop(x, y, n)


@pytest.mark.parametrize("n", [1, 2, 63, 64, 65, 640, 641, 1000, 12323])
def test_fold_matches_repeated_reduction(n):
    rng = random.Random(9000 + n)
    c_int = rng.getrandbits(2 * n - 1) if n > 1 else rng.getrandbits(1)
    c = brute.int_to_words(c_int, 2 * oracle.words(n))
    assert brute.words_to_int(oracle.fold(c, n)) == brute.reduce_cyclic(c_int, n)


@pytest.mark.parametrize("n", RING_SIZES)
def test_ring_product_against_shift_xor(n):
    seed = inputs.SEED_BASE + 99
    a, b = inputs.dense(n, seed, 0, 0), inputs.dense(n, seed, 0, 1)
    x, y = brute.words_to_int(a), brute.words_to_int(b)
    r = oracle.mul_cyclic(a, b, n)
    assert brute.words_to_int(r) == brute.reduce_cyclic(brute.clmul_shiftxor(x, y), n)


@pytest.mark.parametrize("n", RING_SIZES)
def test_ring_invariants(n):
    seed = inputs.SEED_BASE + 98
    a, b, c = (inputs.dense(n, seed, 0, r) for r in range(3))
    W = oracle.words(n)
    one = np.zeros(W, dtype=np.uint64)
    one[0] = 1
    zero = np.zeros(W, dtype=np.uint64)
    ab = oracle.mul_cyclic(a, b, n)
    # commutativity, identity, zero
    assert np.array_equal(ab, oracle.mul_cyclic(b, a, n))
    assert np.array_equal(oracle.mul_cyclic(a, one, n), a)
    assert np.array_equal(oracle.mul_cyclic(a, zero, n), zero)
    # distributivity
    assert np.array_equal(oracle.mul_cyclic(a, b ^ c, n), ab ^ oracle.mul_cyclic(a, c, n))
    # associativity
    assert np.array_equal(oracle.mul_cyclic(ab, c, n), oracle.mul_cyclic(a, oracle.mul_cyclic(b, c, n), n))
    # evaluation at X = 1: parity(a*b) = parity(a) * parity(b)
    xa, xb, xr = (brute.words_to_int(v) for v in (a, b, ab))
    assert brute.parity(xr) == brute.parity(xa) & brute.parity(xb)
    # multiplication by the all-ones polynomial J gives parity(a) * J
    J = brute.int_to_words((1 << n) - 1, W)
    aJ = brute.words_to_int(oracle.mul_cyclic(a, J, n))
    assert aJ == ((1 << n) - 1 if brute.parity(xa) else 0)


@pytest.mark.parametrize("n", RING_SIZES)
def test_monomial_is_rotation(n):
    seed = inputs.SEED_BASE + 97
    a = inputs.dense(n, seed, 0, 0)
    xa = brute.words_to_int(a)
    for k in (1, 63, 64, 65, n // 2, n - 1):
        mono = brute.int_to_words(1 << k, oracle.words(n))
        r = oracle.mul_cyclic(a, mono, n)
        assert brute.words_to_int(r) == brute.rotate(xa, k, n)


@pytest.mark.parametrize("n", RING_SIZES)
def test_squaring_is_the_doubling_permutation(n):
    # n is prime and 2 is a primitive root mod n (the ring condition stated in
    # the introduction), so i -> 2i mod n is a permutation of order n - 1.
    assert pow(2, n - 1, n) == 1
    for p in _prime_factors(n - 1):
        assert pow(2, (n - 1) // p, n) != 1
    a = inputs.dense(n, inputs.SEED_BASE + 96, 0, 0)
    xa = brute.words_to_int(a)
    assert brute.words_to_int(oracle.mul_cyclic(a, a, n)) == brute.square_by_permutation(xa, n)


def _prime_factors(m):
    out, p = set(), 2
    while p * p <= m:
        while m % p == 0:
            out.add(p)
            m //= p
        p += 1
    if m > 1:
        out.add(m)
    return out


@pytest.mark.parametrize("n", RING_SIZES)
def test_sparse_operand_closed_form(n):
    """a * s = XOR over the support of s of the rotations of a (the convolution view)."""
    w = inputs.sparse_weight_for(n)
    seed = inputs.SEED_BASE + 95
    pos = inputs.sparse_positions(n, w, seed, 0)
    assert len(set(pos)) == w and all(0 <= p < n for p in pos)
    s = inputs.from_positions(n, pos)
    a = inputs.dense(n, seed, 0, 0)
    xa = brute.words_to_int(a)
    expect = 0
    for p in pos:
        expect ^= brute.rotate(xa, p, n)
    assert brute.words_to_int(oracle.mul_cyclic(a, s, n)) == expect


@pytest.mark.parametrize("n", [1, 5, 13, 64, 67, 101, 130])
def test_circulant_orientation(n):
    """The ring product h*r equals T r over F2 with T[k][j] = h_{(k - j) mod n}."""
    rng = random.Random(77 + n)
    xh, h = _rand_words(rng, n)
    xr, r = _rand_words(rng, n)
    hb = np.array([(xh >> i) & 1 for i in range(n)], dtype=np.int64)
    rb = np.array([(xr >> i) & 1 for i in range(n)], dtype=np.int64)
    k = np.arange(n)
    T = hb[(k[:, None] - k[None, :]) % n]
    counts = T @ rb
    assert counts.max(initial=0) <= n
    expect = sum(int(v & 1) << i for i, v in enumerate(counts))
    assert brute.words_to_int(oracle.mul_cyclic(h, r, n)) == expect


def test_mul_cyclic_many_matches_single():
    n = 1000
    A = inputs.dense_batch(n, 5, inputs.SEED_BASE + 94, 0)
    B = inputs.dense_batch(n, 5, inputs.SEED_BASE + 94, 1)
    R = oracle.mul_cyclic_many(A, B, n)
    for i in range(5):
        assert np.array_equal(R[i], oracle.mul_cyclic(A[i], B[i], n))


@pytest.mark.parametrize("n", [1, 63, 64, 65, 1000, 12323])
def test_pclmul_fast_mode_equals_portable_mode(n):
    """The timing-only fast mode (PCLMULQDQ) gives the portable oracle's ring
    products (skipped on a CPU without the instruction)."""
    A = inputs.dense_batch(n, 4, inputs.SEED_BASE + 97, 0)
    B = inputs.dense_batch(n, 4, inputs.SEED_BASE + 97, 1)
    A[:, -1] |= ~inputs.top_mask(n)  # junk above n is ignored by both
    fast = oracle.mul_cyclic_many_pclmul(A, B, n)
    if fast is None:
        pytest.skip("no PCLMULQDQ on this CPU")
    assert np.array_equal(fast, oracle.mul_cyclic_many(A, B, n))


def test_mul_batched_matches_bit_loops():
    """The batched entry point on host arrays: ring, full and sparse items of
    tiny mixed sizes against the bit-by-bit definitions (the sparse operand
    as the sum of the rotations of a over its positions, equal positions
    cancelling), with shared operands and outputs in arbitrary order."""
    rng = random.Random(2201)
    sizes = [1, 5, 63, 64, 65, 127, 130, 200]
    A = np.zeros(512, dtype=np.uint64)
    B = np.zeros(512, dtype=np.uint64)
    for i in range(A.size):
        A[i] = rng.getrandbits(64)
        B[i] = rng.getrandbits(64)
    items, expect, c_off = [], [], 0
    for k in range(24):
        n = sizes[k % len(sizes)]
        W = oracle.words(n)
        kind = k % 3
        a_off, b_off = rng.randrange(0, 32), rng.randrange(0, 32)
        xa = brute.words_to_int(A[a_off:a_off + W]) & ((1 << n) - 1)
        if kind == 2:
            pos = [rng.randrange(0, 3 * n) for _ in range(rng.randrange(0, 9))]
            if k % 2:
                q = rng.randrange(0, n)
                pos += [q, q + n]  # equal modulo n: they cancel
            w = len(pos)
            b_off = 128 + 8 * k
            B[b_off:b_off + (w + 1) // 2] = 0
            B[b_off:b_off + (w + 1) // 2].view(np.uint32)[:w] = pos
            r = 0
            for p in pos:
                r ^= brute.rotate(xa, p % n, n)
            items.append((n, 2 | (w << 8), a_off, b_off, c_off))
            expect.append((c_off, brute.int_to_words(r, W)))
            c_off += W
        else:
            xb = brute.words_to_int(B[b_off:b_off + W]) & ((1 << n) - 1)
            if kind == 0:
                r, cw = brute.cyclic_bitloop(xa, xb, n), W
            else:
                r, cw = brute.clmul_bitloop(xa, xb), 2 * W
            items.append((n, kind, a_off, b_off, c_off))
            expect.append((c_off, brute.int_to_words(r, cw)))
            c_off += cw
    arr = np.array(items[::-1], dtype=oracle.REF_ITEM_DTYPE)
    C = np.full(c_off, 0xA5A5A5A5A5A5A5A5, dtype=np.uint64)
    oracle.mul_batched(arr, C, A, B)
    for off, e in expect:
        assert np.array_equal(C[off:off + e.size], e), off
    with pytest.raises(ValueError):
        oracle.mul_batched(np.array([(100, 0, 0, 0, C.size)], dtype=oracle.REF_ITEM_DTYPE), C, A, B)
    with pytest.raises(ValueError):
        oracle.mul_batched(np.array([(100, 3, 0, 0, 0)], dtype=oracle.REF_ITEM_DTYPE), C, A, B)


# ---------------------------------------------------------------- mutation check
# Each mutant plants one plausible mistake in a private copy of the oracle
# source; the pins above must reject every one of them.
MUTANTS = {
    "drop_high_half": ("c[i + j + 1] ^= hi;", "(void)hi;"),
    "clmul_short_loop": ("for (unsigned k = 0; k < 64; ++k)", "for (unsigned k = 0; k < 63; ++k)"),
    "fold_wrong_word": ("uint64_t w1 = (k + q + 1 < 2 * W) ? c[k + q + 1] : 0;",
                        "uint64_t w1 = (k + q + 1 < 2 * W) ? c[k + q] : 0;"),
    "fold_wrong_direction": ("((w0 >> s) | (w1 << (64u - s)))", "((w0 << s) | (w1 >> (64u - s)))"),
    "mask_one_bit_short": ("(((uint64_t)1 << s) - 1u)", "((((uint64_t)1 << s) - 1u) >> 1)"),
    "no_input_mask": ("y[W - 1] &= top_mask(n);", ""),
    "transposed_index": ("c[i + j] ^= lo;", "c[i + i] ^= lo;"),
}


def _build_mutant(tmp_path, name, old, new):
    import ctypes
    import subprocess
    src = open(oracle.oracle._SRC).read()
    assert old in src, name
    path = tmp_path / ("mut_%s.c" % name)
    path.write_text(src.replace(old, new))
    so = tmp_path / ("mut_%s.so" % name)
    subprocess.check_call(["gcc", "-O1", "-std=c99", "-fPIC", "-shared", str(path), "-o", str(so)])
    lib = ctypes.CDLL(str(so))
    u64p = ctypes.POINTER(ctypes.c_uint64)
    for fn in (lib.gf2x_ref_mul, lib.gf2x_ref_mul_cyclic):
        fn.restype = ctypes.c_int
        fn.argtypes = [u64p, u64p, u64p, ctypes.c_uint32]
    return lib, u64p


def _mutant_passes_pins(lib, u64p):
    rng = random.Random(11)
    for n in list(range(1, 70, 3)) + [128, 129, 193]:
        W = oracle.words(n)
        for _ in range(2):
            x, y = rng.getrandbits(n), rng.getrandbits(n)
            junk = (rng.getrandbits(64 * W) >> n) << n  # bits >= n must be ignored
            a = brute.int_to_words(x | junk, W)
            b = brute.int_to_words(y | junk, W)
            c = np.zeros(2 * W, dtype=np.uint64)
            r = np.zeros(W, dtype=np.uint64)
            lib.gf2x_ref_mul(c.ctypes.data_as(u64p), a.ctypes.data_as(u64p), b.ctypes.data_as(u64p), n)
            lib.gf2x_ref_mul_cyclic(r.ctypes.data_as(u64p), a.ctypes.data_as(u64p), b.ctypes.data_as(u64p), n)
            if brute.words_to_int(c) != brute.clmul_bitloop(x, y):
                return False
            if brute.words_to_int(r) != brute.cyclic_bitloop(x, y, n):
                return False
    return True


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_planted_oracle_mistakes_are_caught(tmp_path, name):
    old, new = MUTANTS[name]
    lib, u64p = _build_mutant(tmp_path, name, old, new)
    assert not _mutant_passes_pins(lib, u64p), "pins failed to reject mutant %s" % name


def test_unmutated_copy_passes_pins(tmp_path):
    lib, u64p = _build_mutant(tmp_path, "identity", "#include <stdint.h>", "#include <stdint.h>")
    assert _mutant_passes_pins(lib, u64p)
