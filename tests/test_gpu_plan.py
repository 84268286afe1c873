"""Recorded batches (gf2x_plan_*) and the bounded graph cache of
GF2X_USE_GRAPH: replays equal the oracle on every item, a replay's host
cost does not grow with the number of items, and many distinct graph
batches under a small budget keep working (least recently used graphs are
released)."""
import time

import numpy as np
import pytest

from paper_2201_10473_amd import gf2x, inputs, serve
from tests.gpu_util import empty_dev, from_dev, to_dev
from tests.oracle_check import ring_mismatches

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    c = gf2x.Context(0)
    yield c
    c.close()


def test_plan_replays_equal_oracle(ctx):
    """A plan over a mixed batch (six sizes, staged and direct classes),
    replayed three times with eager work in between; the items array is
    overwritten after the plan is made (the plan keeps its own copy)."""
    import torch
    count = 600
    ns, off, A, B = serve.make_requests(count, inputs.SEED_BASE + 21)
    items = gf2x.make_items(ns, gf2x.KIND_CYCLIC, off, off, off)
    dA, dB, dC = to_dev(A), to_dev(B), empty_dev(len(A))
    print("case plan mixed count=%d" % count, flush=True)
    with ctx.plan(items, dC, dA, dB) as plan:
        items["n_bits"] = 1  # not read again by the plan
        scratch = empty_dev(len(A))
        for rep in range(3):
            dC.fill_(0)
            plan.launch()
            ctx.mul_cyclic(scratch[:1], dA[:1], dB[:1], 64)  # eager work between replays
            torch.cuda.synchronize()
            C = from_dev(dC)
            assert ring_mismatches(ns, off, off, off, A, B, C) == [], rep


def test_empty_plan_and_errors(ctx):
    import torch
    dX = empty_dev(8)
    with ctx.plan(np.zeros(0, dtype=gf2x.ITEM_DTYPE), dX, dX, dX) as plan:
        plan.launch()
    torch.cuda.synchronize()
    bad = gf2x.make_items(100, 7, 0, 0, 0)
    with pytest.raises(gf2x.Gf2xError) as e:
        ctx.plan(bad, dX, dX, dX)
    assert e.value.code == gf2x.GF2X_EINVAL


def _host_launch_us(plan, reps=200):
    import torch
    plan.launch()
    torch.cuda.synchronize()
    t = []
    for _ in range(reps):
        t0 = time.perf_counter()
        plan.launch()
        t.append(time.perf_counter() - t0)
        torch.cuda.synchronize()
    return 1e6 * float(np.median(t))


def test_plan_launch_host_cost_does_not_grow_with_items(ctx):
    """Host time of one replay: 16 items and 16384 items of the same size
    (tiny products, so the device is idle between replays)."""
    n = 64
    times = {}
    for count in (16, 16384):
        off = np.arange(count, dtype=np.uint64)
        items = gf2x.make_items(n, gf2x.KIND_CYCLIC, off, off, off)
        dA = to_dev(inputs.dense_batch(n, count, 5, 0).ravel())
        dB = to_dev(inputs.dense_batch(n, count, 5, 1).ravel())
        dC = empty_dev(count)
        with ctx.plan(items, dC, dA, dB) as plan:
            times[count] = _host_launch_us(plan)
    print("host us per replay: %s" % times, flush=True)
    assert times[16384] < 2.0 * times[16] + 20.0, times


def test_graph_cache_is_bounded_under_a_small_budget():
    """100 distinct GF2X_USE_GRAPH batches (different item arrays) of staged
    products under a 24 MiB budget, each replayed twice: every call works and
    every result equals the oracle."""
    import torch
    n, count = 57637, 24
    W = (n + 63) // 64
    A = inputs.dense_batch(n, count, 9, 0)
    B = inputs.dense_batch(n, count, 9, 1)
    dA, dB, dC = to_dev(A.ravel()), to_dev(B.ravel()), empty_dev(count * W)
    off = np.arange(count, dtype=np.uint64) * W
    ref = None
    with gf2x.Context(0, hbm_budget_bytes=24 << 20) as c:
        arrays = [gf2x.make_items(n, gf2x.KIND_CYCLIC, off, off, off) for _ in range(100)]
        print("case graph cache: 100 batches x 2 replays", flush=True)
        for rep in range(2):
            for k, items in enumerate(arrays):
                dC.fill_(0)
                c.mul_batched(items, dC, dA, dB, gf2x.USE_GRAPH)
                torch.cuda.synchronize()
                C = from_dev(dC)
                if ref is None:
                    ns = np.full(count, n, dtype=np.uint32)
                    assert ring_mismatches(ns, off, off, off, A.ravel(), B.ravel(), C) == []
                    ref = C.copy()
                assert np.array_equal(C, ref), (rep, k)
