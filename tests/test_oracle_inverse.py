"""Pins of the oracle's inverse in F2[X]/(X^n - 1) (CPU): the defining
property a * inv(a) = 1 checked with the oracle's C multiplication, the
non-invertible cases, exhaustive search on tiny rings, and the exponent
identity the library's inversion relies on (for an odd prime n, a^(2^(n-1) - 2)
= a^-1 for every invertible a)."""
import numpy as np
import pytest

import oracle
from oracle import oracle as om
from paper_2201_10473_amd import inputs


def one(n):
    e = np.zeros(oracle.words(n), dtype=np.uint64)
    e[0] = 1
    return e


def odd_weight(n, seed):
    a = inputs.dense(n, 7000 + seed, n, 0)
    if bin(om._to_int(a, n)).count("1") % 2 == 0:
        a[0] ^= np.uint64(1)
    return a


@pytest.mark.parametrize("n", [5, 11, 13, 19, 29, 37, 53, 59, 61, 67, 83, 101, 12323])
def test_inverse_times_operand_is_one(n):
    for seed in range(4):
        a = odd_weight(n, seed)
        c = oracle.inv_cyclic(a, n)
        assert c is not None
        assert np.array_equal(oracle.mul_cyclic(a, c, n), one(n))
        assert np.array_equal(oracle.mul_cyclic(c, a, n), one(n))


@pytest.mark.parametrize("n", [5, 11, 64, 65, 12323])
def test_even_weight_has_no_inverse(n):
    a = inputs.dense(n, 11, n, 0)
    if bin(om._to_int(a, n)).count("1") % 2:
        a[0] ^= np.uint64(1)
    assert oracle.inv_cyclic(a, n) is None  # X + 1 divides both a and X^n - 1


@pytest.mark.parametrize("n", [3, 5, 7])
def test_exhaustive_tiny_rings(n):
    """Every a: the oracle returns the unique c with a*c = 1, or None when no
    such c exists."""
    for av in range(1 << n):
        a = np.array([av], dtype=np.uint64)
        sols = [cv for cv in range(1 << n)
                if int(oracle.mul_cyclic(a, np.array([cv], dtype=np.uint64), n)[0]) == 1]
        got = oracle.inv_cyclic(a, n)
        if sols:
            assert len(sols) == 1 and got is not None and int(got[0]) == sols[0], (n, av)
        else:
            assert got is None, (n, av)


def power(a, e, n):
    """a^e in the ring by square-and-multiply with the oracle's product."""
    r = one(n)
    b = a.copy()
    while e:
        if e & 1:
            r = oracle.mul_cyclic(r, b, n)
        b = oracle.mul_cyclic(b, b, n)
        e >>= 1
    return r


@pytest.mark.parametrize("n", [5, 7, 11, 13, 17, 19, 23, 29, 31])
def test_exponent_identity_for_odd_primes(n):
    """X^n - 1 = (X + 1) times irreducibles of degree d = ord_n(2), and d
    divides n - 1, so every unit u has u^(2^(n-1) - 1) = 1 (whether or not 2
    is primitive, as it is for 5, 11, 13, 19, 29 but not 7, 17, 23, 31)."""
    for seed in range(3):
        a = odd_weight(n, seed)
        c = oracle.inv_cyclic(a, n)
        if c is None:
            continue
        assert np.array_equal(power(a, 2 ** (n - 1) - 2, n), c)


@pytest.mark.parametrize("n", [9, 15])
def test_exponent_identity_fails_for_these_composites(n):
    """For n = 9 or 15 some factor of X^n - 1 has a degree d that does not
    divide n - 1 (ord_9(2) = 6, ord_15(2) = 4), and the identity fails for some
    invertible a: the library accepts odd primes only."""
    bad = 0
    for av in range(1, 1 << n):
        a = np.array([av], dtype=np.uint64)
        c = oracle.inv_cyclic(a, n)
        if c is not None and not np.array_equal(power(a, 2 ** (n - 1) - 2, n), c):
            bad += 1
    assert bad > 0
