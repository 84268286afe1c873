"""The serving loop (continuous batching under an HBM budget) and the mixed
workload: every served result equals the oracle and the same product
computed in a plain batched launch, a sample equals the product computed
alone, and the admission limits hold."""
import numpy as np
import pytest

import oracle
from paper_2201_10473_amd import gf2x, inputs, serve
from tests.oracle_check import ring_mismatches

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    c = gf2x.Context(0)
    yield c
    c.close()


def _oracle_all(bufs):
    """Every served result against the oracle."""
    ns, off, A, B, C = bufs
    bad = ring_mismatches(ns, off, off, off, A, B, C)
    assert bad == [], ("served results differ from the oracle", bad[:10])
    return len(ns)


def _alone(ctx, n, a, b):
    import torch
    from tests.gpu_util import empty_dev, from_dev, to_dev
    C = empty_dev(len(a))
    ctx.mul_cyclic(C, to_dev(a), to_dev(b), n)
    torch.cuda.synchronize()
    return from_dev(C)


def test_served_equals_alone_batched_and_oracle(ctx):
    print("case serving rate=50000 count=3000", flush=True)
    res, (ns, off, A, B, C) = serve.run(ctx, 50000, 3000, inputs.SEED_BASE + 5)
    assert res["server"]["completed"] == 3000 and res["server"]["admitted"] == 3000
    assert res["server"]["phased_batches"] > 0  # small batches run as three phase kernels
    assert serve.check_against_batched(ctx, ns, off, A, B, C) == 3000
    rng = np.random.default_rng(0)
    for i in rng.choice(3000, 30, replace=False):  # 1% re-run alone
        n = int(ns[i])
        W = (n + 63) // 64
        sl = slice(int(off[i]), int(off[i]) + W)
        assert np.array_equal(_alone(ctx, n, A[sl], B[sl]), C[sl]), i
    assert _oracle_all((ns, off, A, B, C)) == 3000
    # latencies are measured from scheduled arrival and are positive
    assert res["p50_us"] > 0 and res["p99_us"] >= res["p50_us"]


def test_high_rate_batches_overlap(ctx):
    print("case serving rate=500000 count=20000", flush=True)
    res, bufs = serve.run(ctx, 500000, 20000, inputs.SEED_BASE + 6)
    st = res["server"]
    assert st["completed"] == 20000
    assert st["max_batch_seen"] > 1          # arrivals joined running work as batches
    assert st["max_slots_busy"] >= 2         # batches on different streams in flight together
    serve.check_against_batched(ctx, *bufs)
    _oracle_all(bufs)


def test_burst_takes_batches_above_the_staged_threshold(ctx):
    """1000 requests submitted at once are admitted as batches of several
    hundred, which run one workgroup per product (direct classes), while a
    trickle runs staged classes; both give the batched launch's results."""
    print("case serving burst count=1000", flush=True)
    ns, off, A, B = serve.make_requests(1000, inputs.SEED_BASE + 12)
    C = np.zeros_like(A)
    with gf2x.Server(ctx) as srv:
        srv.submit(ns, A, off, B, off, C, off)
        srv.drain()
        st = srv.stats()
    assert st["completed"] == 1000
    assert st["max_batch_seen"] > 256
    assert serve.check_against_batched(ctx, ns, off, A, B, C) == 1000
    _oracle_all((ns, off, A, B, C))


def test_sixteen_streams_default_budget(ctx):
    """With 16 slots the default budget holds the staged workspace for smaller
    batches only; results still equal the batched launch."""
    print("case serving streams=16 rate=100000 count=4000", flush=True)
    res, bufs = serve.run(ctx, 100000, 4000, inputs.SEED_BASE + 13, streams=16)
    assert res["server"]["completed"] == 4000
    assert serve.check_against_batched(ctx, *bufs) == 4000
    _oracle_all(bufs)


def test_tiny_hbm_budget_backpressure(ctx):
    """A budget of one largest request per stream: every batch holds one
    request, nothing is dropped, results are unchanged."""
    W = (57637 + 63) // 64
    per_req = 40 + 3 * W * 8
    print("case serving tiny budget", flush=True)
    res, bufs = serve.run(ctx, 200000, 400, inputs.SEED_BASE + 7, hbm_budget_bytes=4 * per_req, streams=4,
                          warm=False)
    st = res["server"]
    assert st["max_batch"] == 1 and st["max_batch_seen"] == 1
    assert st["completed"] == 400 and st["batches"] == 400
    assert st["hbm_bytes"] <= 4 * per_req + 4 * 256
    serve.check_against_batched(ctx, *bufs)
    _oracle_all(bufs)


def test_budget_too_small_and_queue_full(ctx):
    with pytest.raises(gf2x.Gf2xError) as e:
        gf2x.Server(ctx, hbm_budget_bytes=1000, streams=4)
    assert e.value.code == gf2x.GF2X_ENOMEM
    ns, off, A, B = serve.make_requests(12, 3)
    C = np.zeros_like(A)
    far = None
    with gf2x.Server(ctx, max_pending=10) as srv:
        far = np.full(12, srv.now_ns() + int(50e6), dtype=np.uint64)  # 50 ms in the future
        with pytest.raises(gf2x.Gf2xError) as e:
            srv.submit(ns, A, off, B, off, C, off, far)
        assert e.value.code == gf2x.GF2X_EAGAIN
        first = srv.submit(ns[:10], A, off[:10], B, off[:10], C, off[:10], far[:10])
        srv.drain()
        done = srv.completion(first, 10)
        assert (done >= far[:10]).all()      # nothing admitted before its arrival time
        assert srv.stats()["refused"] == 12
    with pytest.raises(gf2x.Gf2xError):
        gf2x.Server(ctx, max_bits=gf2x.GF2X_MAX_BITS + 1)


def test_mixed_workload_graph(ctx):
    """The mixed workload: 8192 products, n uniform over the six sizes, half
    dense x sparse, in one graph-captured launch sequence; every item equal
    to the oracle, the first sparse items also to the rotation closed form."""
    import torch
    from tests import brute
    from tests.gpu_util import empty_dev, from_dev, parity_rows, to_dev
    count = 8192
    seed = inputs.SEED_BASE + 4
    ns, off, A, B = serve.make_requests(count, seed)
    sparse_items = np.arange(1, count, 2)
    pos_of = {}
    for i in sparse_items[:64]:  # sparse operands for the first 64 odd items, kept for the closed form
        n = int(ns[i])
        pos = inputs.sparse_positions(n, inputs.sparse_weight_for(n), seed, int(i))
        pos_of[int(i)] = pos
    for i in sparse_items:
        n = int(ns[i])
        W = (n + 63) // 64
        pos = pos_of.get(int(i)) or inputs.sparse_positions(n, inputs.sparse_weight_for(n), seed, int(i))
        B[int(off[i]):int(off[i]) + W] = inputs.from_positions(n, pos)
    items = gf2x.make_items(ns, gf2x.KIND_CYCLIC, off, off, off)
    dA, dB, dC = to_dev(A), to_dev(B), empty_dev(len(A))
    for _ in range(2):
        ctx.mul_batched(items, dC, dA, dB, gf2x.USE_GRAPH)
        torch.cuda.synchronize()
    C = from_dev(dC)
    for n in inputs.RING_SIZES:
        idx = np.nonzero(ns == n)[0]
        W = (n + 63) // 64
        rows = lambda X: X[(off[idx][:, None] + np.arange(W)[None, :]).astype(np.int64)]
        assert np.array_equal(parity_rows(rows(C)), parity_rows(rows(A)) & parity_rows(rows(B)))
    bad = ring_mismatches(ns, off, off, off, A, B, C)
    assert bad == [], ("mixed items differ from the oracle", bad[:10])
    for i, pos in list(pos_of.items())[:16]:
        n = int(ns[i])
        W = (n + 63) // 64
        sl = slice(int(off[i]), int(off[i]) + W)
        xa = brute.words_to_int(A[sl])
        expect = 0
        for q in pos:
            expect ^= brute.rotate(xa, q, n)
        assert brute.words_to_int(C[sl]) == expect, i


def test_completion_stamps_are_released_once_read(ctx):
    """A stamp is returned once; once every earlier stamp has been returned
    too, the server drops it and a second read gives 1 (done, not kept)."""
    ns, off, A, B = serve.make_requests(50, inputs.SEED_BASE + 14)
    C = np.zeros_like(A)
    with gf2x.Server(ctx) as srv:
        first = srv.submit(ns, A, off, B, off, C, off)
        srv.drain()
        done = srv.completion(first, 50)
        assert (done > 1).all()
        again = srv.completion(first, 50)
        assert (again == 1).all()
        second = srv.submit(ns[:5], A, off[:5], B, off[:5], C, off[:5])
        srv.drain()
        assert (srv.completion(second, 5) > 1).all()
        with pytest.raises(gf2x.Gf2xError):
            srv.completion(second, 6)  # a ticket not yet issued
    assert ring_mismatches(ns, off, off, off, A, B, C) == []
