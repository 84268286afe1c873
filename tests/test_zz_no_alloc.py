"""The allocation-free batched entry point (gf2x_mul_batched_noalloc): its
results equal gf2x_mul_batched's on the same items, over two calls in a row
(the second with a smaller batch, on the scratch the first one left), a
batch whose staged workspace exceeds the scratch, and the size limit."""
import numpy as np
import pytest

import oracle
from paper_2201_10473_amd import gf2x, inputs, serve
from tests.gpu_util import empty_dev, from_dev, to_dev
from tests.oracle_check import ring_mismatches

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    c = gf2x.Context(0)
    yield c
    c.close()


def _mixed(count, seed, full_every=0):
    """Items of the six ring sizes (and full products every `full_every`-th)."""
    ns, off, A, B = serve.make_requests(count, seed)
    kinds = np.zeros(count, dtype=np.uint32)
    if full_every:
        kinds[::full_every] = gf2x.KIND_FULL
    cw = np.where(kinds == gf2x.KIND_FULL, 2, 1) * ((ns.astype(np.uint64) + 63) // 64)
    c_off = np.concatenate([[0], np.cumsum(cw)[:-1]]).astype(np.uint64)
    items = gf2x.make_items(ns, kinds, off, off, c_off)
    return ns, kinds, off, c_off, int(cw.sum()), A, B, items


def _both(ctx, items, A, B, c_words):
    """(no-alloc result, gf2x_mul_batched result) as host words."""
    import torch
    dA, dB = to_dev(A), to_dev(B)
    d1, d2 = empty_dev(c_words, 0x1111111111111111), empty_dev(c_words, 0x2222222222222222)
    ctx.mul_batched_noalloc(items, d1, dA, dB)
    ctx.mul_batched(items, d2, dA, dB)
    torch.cuda.synchronize()
    return from_dev(d1), from_dev(d2)


def test_two_calls_in_a_row_equal_the_batched_entry_point(ctx):
    ns, kinds, off, c_off, cw, A, B, items = _mixed(700, inputs.SEED_BASE + 31, full_every=9)
    print("case noalloc first call: %d items, six sizes" % len(ns), flush=True)
    got, ref = _both(ctx, items, A, B, cw)
    assert np.array_equal(got, ref)
    ring = kinds == gf2x.KIND_CYCLIC
    assert ring_mismatches(ns[ring], off[ring], off[ring], c_off[ring], A, B, got) == []
    # second call, smaller: the scratch still holds the first call's descriptors
    ns2, kinds2, off2, c_off2, cw2, A2, B2, items2 = _mixed(45, inputs.SEED_BASE + 32)
    print("case noalloc second call: %d items" % len(ns2), flush=True)
    got2, ref2 = _both(ctx, items2, A2, B2, cw2)
    assert np.array_equal(got2, ref2)
    assert ring_mismatches(ns2, off2, off2, c_off2, A2, B2, got2) == []


def test_batch_larger_than_the_staged_workspace(ctx):
    """1024 products at n = 57637 (staged workspace of about 54 MB, more than
    the scratch holds) run in their one-workgroup class: same results."""
    n, count = 57637, 1024
    W = oracle.words(n)
    A = inputs.dense_batch(n, count, inputs.SEED_BASE + 33, 0).ravel()
    B = inputs.dense_batch(n, count, inputs.SEED_BASE + 33, 1).ravel()
    off = np.arange(count, dtype=np.uint64) * W
    items = gf2x.make_items(n, gf2x.KIND_CYCLIC, off, off, off)
    print("case noalloc n=%d count=%d" % (n, count), flush=True)
    got, ref = _both(ctx, items, A, B, count * W)
    assert np.array_equal(got, ref)


def test_size_limit_and_arguments(ctx):
    dX = empty_dev(8)
    too_many = np.zeros(65537, dtype=gf2x.ITEM_DTYPE)
    too_many["n_bits"] = 1
    with pytest.raises(gf2x.Gf2xError) as e:
        ctx.mul_batched_noalloc(too_many, dX, dX, dX)
    assert e.value.code == gf2x.GF2X_ENOMEM
    with pytest.raises(gf2x.Gf2xError) as e:
        ctx.mul_batched_noalloc(gf2x.make_items(100, 7, 0, 0, 0), dX, dX, dX)
    assert e.value.code == gf2x.GF2X_EINVAL
    ctx.mul_batched_noalloc(np.zeros(0, dtype=gf2x.ITEM_DTYPE), dX, dX, dX)  # empty: no-op
