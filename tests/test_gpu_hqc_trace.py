"""The HQC-shaped trace: chains of 1, 2 or 3 dependent ring products at the
three HQC sizes, served with each product submitted once its predecessor has
completed.  Every served chain equals the same chain recomputed with batched
launches and the oracle applied step by step."""
import numpy as np
import pytest

import oracle
from paper_2201_10473_amd import gf2x, hqc_trace, inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    c = gf2x.Context(0)
    yield c
    c.close()


def test_trace_chains_match_batched_and_oracle(ctx):
    count = 600
    print("case hqc_trace rate=20000 count=%d" % count, flush=True)
    res, trace = hqc_trace.run(ctx, 20000, count, inputs.SEED_BASE + 11)
    kinds, ns, length, W, X, xo, R, ro = trace
    assert res["operations"] == count
    assert res["products"] == int(length.sum())
    assert sum(v["count"] for v in res["per_kind"].values()) == count
    for v in res["per_kind"].values():
        assert 0 < v["p50_us"] <= v["p99_us"]
    # a longer chain cannot finish sooner than its own first product could
    assert res["per_kind"]["decaps"]["p50_us"] >= res["per_kind"]["keygen"]["p50_us"]
    assert hqc_trace.check_against_batched(ctx, trace) == int(length.sum())
    for op in range(count):
        n, w, L = int(ns[op]), int(W[op]), int(length[op])
        x0 = int(xo[op])
        acc = X[x0:x0 + w]
        for k in range(1, L + 1):
            acc = oracle.mul_cyclic(acc, X[x0 + k * w:x0 + (k + 1) * w], n)
            r0 = int(ro[op]) + (k - 1) * w
            assert np.array_equal(acc, R[r0:r0 + w]), (op, k)

