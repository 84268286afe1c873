"""Brute-force references used to pin the oracle.

They work bit by bit on Python integers (bit i of the integer is the
coefficient of X^i) and share nothing with the oracle's word-level loops.
"""
import numpy as np


def words_to_int(w):
    x = 0
    for i, v in enumerate(np.asarray(w, dtype=np.uint64).tolist()):
        x |= int(v) << (64 * i)
    return x


def int_to_words(x, count):
    mask = (1 << 64) - 1
    return np.array([(x >> (64 * i)) & mask for i in range(count)], dtype=np.uint64)


def bits(x):
    i = 0
    while x:
        if x & 1:
            yield i
        x >>= 1
        i += 1


def clmul_bitloop(x, y):
    """c_k = XOR over i + j = k of x_i AND y_j, as a double loop over bits."""
    c = 0
    for i in bits(x):
        for j in bits(y):
            c ^= 1 << (i + j)
    return c


def clmul_shiftxor(x, y):
    """Sum of x * X^j over the set bits j of y (one big-integer XOR per bit)."""
    c = 0
    for j in bits(y):
        c ^= x << j
    return c


def reduce_cyclic(c, n):
    """Reduce c modulo X^n - 1 by repeatedly adding the part above X^n back at 0."""
    mask = (1 << n) - 1
    while c >> n:
        c = (c & mask) ^ (c >> n)
    return c


def cyclic_bitloop(x, y, n):
    """r_{(i + j) mod n} ^= x_i AND y_j for all i, j < n (tiny n only)."""
    r = 0
    for i in bits(x):
        for j in bits(y):
            r ^= 1 << ((i + j) % n)
    return r


def rotate(x, k, n):
    """Cyclic rotation of an n-bit integer left by k (multiplication by X^k in the ring)."""
    k %= n
    mask = (1 << n) - 1
    return ((x << k) | (x >> (n - k))) & mask if k else x


def parity(x):
    return bin(x).count("1") & 1


def square_by_permutation(x, n):
    """In F2[X]/(X^n - 1) with n odd, a^2 moves bit i to bit 2i mod n."""
    r = 0
    for i in bits(x):
        r |= 1 << ((2 * i) % n)
    return r
