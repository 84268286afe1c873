"""ctypes wrapper around the C oracle (``gf2x_oracle.c``).

TEST INFRASTRUCTURE ONLY (see the package docstring).  Operands are numpy
``uint64`` arrays of ``words(n)`` little-endian words; bit i of a polynomial
is bit i % 64 of word i // 64.
"""
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "gf2x_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None

_u64p = ctypes.POINTER(ctypes.c_uint64)


def words(n):
    """Number of 64-bit words holding a polynomial of n coefficients."""
    return (int(n) + 63) // 64


def build():
    """Compile the oracle with gcc -O2 into ``liboracle.so`` (always rebuilds)."""
    tmp = _LIB + ".tmp"
    subprocess.check_call(
        ["gcc", "-O2", "-std=c99", "-Wall", "-Wextra", "-fPIC", "-shared", _SRC, "-o", tmp]
    )
    os.replace(tmp, _LIB)
    return _LIB


def load():
    """Load the built oracle, building it first only if it is absent."""
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        lib = ctypes.CDLL(_LIB)
        for name in ("gf2x_ref_mul", "gf2x_ref_mul_cyclic"):
            fn = getattr(lib, name)
            fn.restype = ctypes.c_int
            fn.argtypes = [_u64p, _u64p, _u64p, ctypes.c_uint32]
        lib.gf2x_ref_fold.restype = ctypes.c_int
        lib.gf2x_ref_fold.argtypes = [_u64p, _u64p, ctypes.c_uint32]
        lib.gf2x_ref_mul_cyclic_many.restype = ctypes.c_int
        lib.gf2x_ref_mul_cyclic_many.argtypes = [_u64p, _u64p, _u64p, ctypes.c_uint32, ctypes.c_uint32]
        lib.gf2x_ref_mul_cyclic_many_pclmul.restype = ctypes.c_int
        lib.gf2x_ref_mul_cyclic_many_pclmul.argtypes = [_u64p, _u64p, _u64p, ctypes.c_uint32, ctypes.c_uint32]
        lib.gf2x_ref_mul_batched.restype = ctypes.c_int
        lib.gf2x_ref_mul_batched.argtypes = [_u64p, _u64p, _u64p, ctypes.c_void_p, ctypes.c_uint32]
        lib.gf2x_ref_clmul64.restype = None
        lib.gf2x_ref_clmul64.argtypes = [ctypes.c_uint64, ctypes.c_uint64, _u64p, _u64p]
        _lib = lib
    return _lib


def _ptr(arr):
    return arr.ctypes.data_as(_u64p)


def _as_words(x, n):
    x = np.ascontiguousarray(x, dtype=np.uint64)
    if x.shape != (words(n),):
        raise ValueError("operand must hold exactly words(n) = %d words" % words(n))
    return x


def clmul64(x, y):
    """Carry-less 64x64 -> 128 product; returns (lo, hi) as Python ints."""
    lo = ctypes.c_uint64()
    hi = ctypes.c_uint64()
    load().gf2x_ref_clmul64(int(x), int(y), ctypes.byref(lo), ctypes.byref(hi))
    return lo.value, hi.value


def mul(a, b, n):
    """Full product in F2[X]: returns 2*words(n) words."""
    a = _as_words(a, n)
    b = _as_words(b, n)
    c = np.zeros(2 * words(n), dtype=np.uint64)
    rc = load().gf2x_ref_mul(_ptr(c), _ptr(a), _ptr(b), int(n))
    if rc:
        raise RuntimeError("gf2x_ref_mul failed (%d)" % rc)
    return c


def fold(c, n):
    """Reduce a full product (2*words(n) words) modulo X^n - 1."""
    c = np.ascontiguousarray(c, dtype=np.uint64)
    if c.shape != (2 * words(n),):
        raise ValueError("full product must hold 2*words(n) words")
    r = np.zeros(words(n), dtype=np.uint64)
    rc = load().gf2x_ref_fold(_ptr(r), _ptr(c), int(n))
    if rc:
        raise RuntimeError("gf2x_ref_fold failed (%d)" % rc)
    return r


def mul_cyclic(a, b, n):
    """Ring product a*b mod (X^n - 1): returns words(n) words."""
    a = _as_words(a, n)
    b = _as_words(b, n)
    r = np.zeros(words(n), dtype=np.uint64)
    rc = load().gf2x_ref_mul_cyclic(_ptr(r), _ptr(a), _ptr(b), int(n))
    if rc:
        raise RuntimeError("gf2x_ref_mul_cyclic failed (%d)" % rc)
    return r


def mul_cyclic_many(a, b, n):
    """Ring products of row pairs: a, b are (count, words(n)) arrays."""
    a = np.ascontiguousarray(a, dtype=np.uint64)
    b = np.ascontiguousarray(b, dtype=np.uint64)
    if a.ndim != 2 or a.shape != b.shape or a.shape[1] != words(n):
        raise ValueError("operands must be (count, words(n)) arrays of equal shape")
    r = np.zeros_like(a)
    rc = load().gf2x_ref_mul_cyclic_many(_ptr(r), _ptr(a), _ptr(b), int(n), a.shape[0])
    if rc:
        raise RuntimeError("gf2x_ref_mul_cyclic_many failed (%d)" % rc)
    return r


def mul_cyclic_many_pclmul(a, b, n):
    """mul_cyclic_many with the CPU's carry-less multiply instruction (for
    timing the CPU side); None when the CPU lacks it."""
    a = np.ascontiguousarray(a, dtype=np.uint64)
    b = np.ascontiguousarray(b, dtype=np.uint64)
    if a.ndim != 2 or a.shape != b.shape or a.shape[1] != words(n):
        raise ValueError("operands must be (count, words(n)) arrays of equal shape")
    r = np.zeros_like(a)
    rc = load().gf2x_ref_mul_cyclic_many_pclmul(_ptr(r), _ptr(a), _ptr(b), int(n), a.shape[0])
    if rc == -3:
        return None
    if rc:
        raise RuntimeError("gf2x_ref_mul_cyclic_many_pclmul failed (%d)" % rc)
    return r


# One product of a batch: the C oracle's gf2x_ref_item (offsets in uint64
# words from the base arrays; kind 0 ring, 1 full, 2 + (w << 8) sparse).
REF_ITEM_DTYPE = np.dtype(
    [("n_bits", "<u4"), ("kind", "<u4"), ("a_off", "<u8"), ("b_off", "<u8"), ("c_off", "<u8")], align=True
)


def mul_batched(items, c_base, a_base, b_base):
    """Every product of a batch on host arrays, written into ``c_base`` in
    place (the items' ranges are checked against the arrays first)."""
    items = np.ascontiguousarray(items).view(REF_ITEM_DTYPE) if len(items) else np.zeros(0, REF_ITEM_DTYPE)
    for base in (c_base, a_base, b_base):
        if not (isinstance(base, np.ndarray) and base.dtype == np.uint64 and base.flags.c_contiguous):
            raise ValueError("bases must be contiguous uint64 arrays")
    for it in items:
        n, kind = int(it["n_bits"]), int(it["kind"])
        W = words(n)
        if n == 0 or (kind & 0xFF) > 2 or (kind & 0xFF) != 2 and kind > 1:
            raise ValueError("bad item %r" % (it,))
        b_len = ((kind >> 8) + 1) // 2 if kind & 0xFF == 2 else W
        c_len = 2 * W if kind == 1 else W
        if (int(it["a_off"]) + W > a_base.size or int(it["b_off"]) + b_len > b_base.size
                or int(it["c_off"]) + c_len > c_base.size):
            raise ValueError("item range outside its array: %r" % (it,))
    rc = load().gf2x_ref_mul_batched(_ptr(c_base), _ptr(a_base), _ptr(b_base), items.ctypes.data, len(items))
    if rc:
        raise RuntimeError("gf2x_ref_mul_batched failed (%d)" % rc)
    return c_base


# ------------------------------------------------------------------ inverses
# The inverse in F2[X]/(X^n - 1) by its definition: c with a*c = 1 modulo
# X^n - 1, found by the extended Euclidean algorithm on polynomials over F2
# held as Python integers (bit i = coefficient of X^i).  This is independent
# of the library's method (an exponentiation by repeated squarings and
# products); it exists when gcd(a, X^n - 1) = 1.


def _to_int(a, n):
    a = _as_words(a, n)
    x = 0
    for i, w in enumerate(a.tolist()):
        x |= int(w) << (64 * i)
    return x & ((1 << n) - 1)


def _from_int(x, n):
    return np.array([(x >> (64 * i)) & 0xFFFFFFFFFFFFFFFF for i in range(words(n))], dtype=np.uint64)


def _pmul(x, y):
    """Carry-less product of two integers (polynomials over F2)."""
    if x.bit_length() < y.bit_length():
        x, y = y, x
    r = 0
    while y:
        low = y & -y
        r ^= x << (low.bit_length() - 1)
        y ^= low
    return r


def _pdivmod(x, y):
    """Quotient and remainder of polynomial division over F2 (y != 0)."""
    q = 0
    dy = y.bit_length()
    while x.bit_length() >= dy:
        s = x.bit_length() - dy
        q |= 1 << s
        x ^= y << s
    return q, x


def inv_cyclic(a, n):
    """Inverse of a in F2[X]/(X^n - 1) as words(n) words, or None if a shares
    a factor with X^n - 1 (for instance when a has even weight)."""
    m = (1 << n) | 1  # X^n - 1 = X^n + 1 over F2
    r0, r1 = m, _to_int(a, n)
    s0, s1 = 0, 1  # invariant: r_i = s_i * a (mod m)
    while r1:
        q, r = _pdivmod(r0, r1)
        r0, r1 = r1, r
        s0, s1 = s1, s0 ^ _pmul(q, s1)
    if r0 != 1:
        return None
    return _from_int(_pdivmod(s0, m)[1], n)
