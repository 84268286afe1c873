"""Inverses in F2[X]/(X^n - 1) on the GPU (gf2x_inv_cyclic_batched) against
the oracle's inverse (extended Euclid), and argument errors."""
import numpy as np
import pytest

import oracle
from oracle import oracle as om
from paper_2201_10473_amd import gf2x, inputs
from tests.gpu_util import empty_dev, from_dev, to_dev
from tests.oracle_check import ring_rows

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch

    assert torch.cuda.is_available()
    c = gf2x.Context(0)
    yield c
    c.close()


def odd_weight_batch(n, count, seed):
    A = inputs.dense_batch(n, count, seed, 0)
    for i in range(count):
        if bin(om._to_int(A[i], n)).count("1") % 2 == 0:
            A[i, 0] ^= np.uint64(1)
    return A


@pytest.mark.parametrize("n,count", [(11, 9), (13, 5), (17, 7), (101, 33), (12323, 70), (12323, 1024), (24659, 3),
                                     (40973, 3)])
def test_inverse_matches_oracle(ctx, n, count):
    """Batches above 64 items use the batch schedule, smaller ones the
    single-product one; 17 is a prime for which 2 is not primitive."""
    W = oracle.words(n)
    A = odd_weight_batch(n, count, 31 + n)
    # results written out of order and with a gap, operands read in place
    a_off = np.arange(count, dtype=np.uint64) * W
    c_off = (np.arange(count, dtype=np.uint64)[::-1] * (W + 3)).copy()
    items = gf2x.make_items(n, gf2x.KIND_CYCLIC, a_off, a_off, c_off)
    dA = to_dev(A.ravel())
    dC = empty_dev(count * (W + 3))
    print("case inverse n=%d count=%d" % (n, count), flush=True)
    ctx.inv_cyclic_batched(items, dC, dA)
    import torch
    torch.cuda.synchronize()
    C = from_dev(dC)
    # every result: a * c = 1 with the oracle's product (the inverse is unique)
    unit = np.zeros(W, dtype=np.uint64)
    unit[0] = 1
    Cr = np.stack([C[int(c_off[i]):int(c_off[i]) + W] for i in range(count)])
    prod = ring_rows(A, Cr, n)
    for i in range(count):
        if n >= 1000 or bin(om._to_int(A[i], n)).count("1") % 2:
            assert np.array_equal(prod[i], unit) or oracle.inv_cyclic(A[i], n) is None, (n, i)
    # and the oracle's own inverse (extended Euclid) on a sample at large n
    sample = range(count) if n < 1000 else (0, 1, count - 1)
    for i in sample:
        got = C[int(c_off[i]):int(c_off[i]) + W]
        ref = oracle.inv_cyclic(A[i], n)
        if ref is None:  # shares a factor with X^n - 1 (possible when 2 is not primitive)
            continue
        assert np.array_equal(got, ref), (n, i)


def test_inverse_in_place(ctx):
    n, count = 12323, 4
    W = oracle.words(n)
    A = odd_weight_batch(n, count, 77)
    off = np.arange(count, dtype=np.uint64) * W
    items = gf2x.make_items(n, gf2x.KIND_CYCLIC, off, off, off)
    dA = to_dev(A.ravel())
    ctx.inv_cyclic_batched(items, dA, dA)
    import torch
    torch.cuda.synchronize()
    C = from_dev(dA).reshape(count, W)
    for i in range(count):
        assert np.array_equal(C[i], oracle.inv_cyclic(A[i], n))


@pytest.mark.parametrize("n", [1, 2, 9, 15, 12322, 12325])
def test_inverse_rejects_sizes_that_are_not_odd_primes(ctx, n):
    W = oracle.words(n)
    items = gf2x.make_items(n, gf2x.KIND_CYCLIC, np.zeros(1, np.uint64), np.zeros(1, np.uint64), np.zeros(1, np.uint64))
    dA, dC = to_dev(np.ones(W, np.uint64)), empty_dev(W)
    with pytest.raises(gf2x.Gf2xError) as e:
        ctx.inv_cyclic_batched(items, dC, dA)
    assert e.value.code == gf2x.GF2X_EINVAL


def test_inverse_rejects_mixed_sizes_and_full_kind(ctx):
    W = oracle.words(12323)
    dA, dC = to_dev(np.ones(2 * W, np.uint64)), empty_dev(2 * W)
    mixed = gf2x.make_items(np.array([12323, 11], np.uint32), gf2x.KIND_CYCLIC, np.array([0, W], np.uint64),
                            np.array([0, W], np.uint64), np.array([0, W], np.uint64))
    with pytest.raises(gf2x.Gf2xError):
        ctx.inv_cyclic_batched(mixed, dC, dA)
    full = gf2x.make_items(12323, gf2x.KIND_FULL, np.zeros(1, np.uint64), np.zeros(1, np.uint64),
                           np.zeros(1, np.uint64))
    with pytest.raises(gf2x.Gf2xError):
        ctx.inv_cyclic_batched(full, dC, dA)
