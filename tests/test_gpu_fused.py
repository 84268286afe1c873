"""One persistent launch over a batch of uneven sizes (GF2X_FUSED): every
item equal to the oracle, in a direct call, in graph replays and in a
recorded plan replayed several times (the work queue resets itself), and
the sizes and kinds it refuses."""
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


def test_fused_mixed_sizes_all_forms(ctx):
    import torch
    count = 900
    ns, off, A, B = serve.make_requests(count, inputs.SEED_BASE + 51)
    items = gf2x.make_items(ns, gf2x.KIND_CYCLIC, off, off, off)
    dA, dB = to_dev(A), to_dev(B)
    for how in ("call", "graph", "plan"):
        dC = empty_dev(len(A))
        print("case fused %s count=%d" % (how, count), flush=True)
        for rep in range(3):
            dC.fill_(0)
            if how == "call":
                ctx.mul_batched(items, dC, dA, dB, gf2x.FUSED)
            elif how == "graph":
                ctx.mul_batched(items, dC, dA, dB, gf2x.FUSED | gf2x.USE_GRAPH)
            else:
                if rep == 0:
                    plan = ctx.plan(items, dC, dA, dB, gf2x.FUSED)
                plan.launch()
            torch.cuda.synchronize()
            C = from_dev(dC)
            assert ring_mismatches(ns, off, off, off, A, B, C) == [], (how, rep)
        if how == "plan":
            plan.close()


def test_fused_full_kind_and_ragged_count(ctx):
    import torch
    sizes = [12323, 57637, 17669, 40973, 24659, 35851, 57637]
    W = [oracle.words(n) for n in sizes]
    a_off = np.concatenate([[0], np.cumsum(W)[:-1]]).astype(np.uint64)
    c_off = 2 * a_off
    A = np.concatenate([inputs.dense(n, 7, i, 0) for i, n in enumerate(sizes)])
    B = np.concatenate([inputs.dense(n, 7, i, 1) for i, n in enumerate(sizes)])
    items = gf2x.make_items(np.array(sizes, np.uint32), gf2x.KIND_FULL, a_off, a_off, c_off)
    dC = empty_dev(2 * len(A))
    ctx.mul_batched(items, dC, to_dev(A), to_dev(B), gf2x.FUSED)
    torch.cuda.synchronize()
    C = from_dev(dC)
    for i, n in enumerate(sizes):
        a, b = A[a_off[i]:a_off[i] + W[i]], B[a_off[i]:a_off[i] + W[i]]
        assert np.array_equal(C[c_off[i]:c_off[i] + 2 * W[i]], oracle.mul(a, b, n)), i


def test_fused_refuses_other_classes(ctx):
    dX = empty_dev(4096)
    for kinds, n in ((gf2x.KIND_CYCLIC, 100), (gf2x.sparse_kind(3), 17669)):
        items = gf2x.make_items(n, kinds, 0, 0, 0)
        with pytest.raises(gf2x.Gf2xError) as e:
            ctx.mul_batched(items, dX, dX, dX, gf2x.FUSED)
        assert e.value.code == gf2x.GF2X_ENOTSUP
