"""Parity of the HIP path (through the C ABI) with the CPU oracle.

Bit-exact comparison on seeded inputs: every ring size of the workloads, the
edge sizes of the ABI, every schedule class, ragged tails, full products,
and batched launches at full workload sizes (every item against the oracle,
computed over a pool of host threads)."""
import os

import numpy as np
import pytest

import oracle
from paper_2201_10473_amd import gf2x, inputs
from tests.gpu_util import empty_dev, from_dev, parity_rows, to_dev
from tests.oracle_check import ring_mismatches, ring_rows

pytestmark = pytest.mark.gpu

RING = inputs.RING_SIZES
SEED = inputs.SEED_BASE


@pytest.fixture(scope="module")
def ctx():
    import torch

    assert torch.cuda.is_available()
    c = gf2x.Context(0)
    yield c
    c.close()


def _single(ctx, n, a, b, kind):
    import torch

    W = oracle.words(n)
    A, B = to_dev(a), to_dev(b)
    C = empty_dev(W if kind == gf2x.KIND_CYCLIC else 2 * W)
    if kind == gf2x.KIND_CYCLIC:
        ctx.mul_cyclic(C, A, B, n)
    else:
        ctx.mul(C, A, B, n)
    torch.cuda.synchronize()
    return from_dev(C)


@pytest.mark.parametrize("n", RING)
def test_ring_sizes_single(ctx, n):
    print("case ring single n=%d" % n, flush=True)
    for item in range(3):
        a = inputs.dense(n, SEED + 1, item, 0)
        b = inputs.dense(n, SEED + 1, item, 1)
        assert np.array_equal(_single(ctx, n, a, b, gf2x.KIND_CYCLIC), oracle.mul_cyclic(a, b, n))
    assert np.array_equal(_single(ctx, n, a, b, gf2x.KIND_FULL), oracle.mul(a, b, n))


EDGE = [1, 2, 3, 31, 32, 33, 63, 64, 65, 127, 128, 129, 255, 256, 257, 1000, 4095, 4096, 4097, 8191, 8193,
        13311, 13313, 18239, 18241, 36095, 36097, 59137, 63743, 63745, 100000, gf2x.GF2X_MAX_BITS]


@pytest.mark.parametrize("n", EDGE)
def test_edge_sizes(ctx, n):
    print("case edge n=%d" % n, flush=True)
    a = inputs.dense(n, SEED + 2, n, 0)
    b = inputs.dense(n, SEED + 2, n, 1)
    assert np.array_equal(_single(ctx, n, a, b, gf2x.KIND_CYCLIC), oracle.mul_cyclic(a, b, n))
    assert np.array_equal(_single(ctx, n, a, b, gf2x.KIND_FULL), oracle.mul(a, b, n))


def test_degenerate_operands(ctx):
    n = 17669
    W = oracle.words(n)
    zero = np.zeros(W, dtype=np.uint64)
    ones = inputs.dense(n, 0, 0, 0) | np.uint64(0xFFFFFFFFFFFFFFFF)
    ones[-1] &= inputs.top_mask(n)
    one = zero.copy()
    one[0] = 1
    a = inputs.dense(n, SEED + 3, 0, 0)
    for x, y in ((zero, a), (a, zero), (one, a), (ones, ones), (ones, a), (a, a)):
        assert np.array_equal(_single(ctx, n, x, y, gf2x.KIND_CYCLIC), oracle.mul_cyclic(x, y, n))


def test_input_bits_above_n_ignored(ctx):
    for n in (17669, 57637, 100):
        a = inputs.dense(n, SEED + 4, 0, 0)
        b = inputs.dense(n, SEED + 4, 0, 1)
        ja, jb = a.copy(), b.copy()
        ja[-1] |= ~inputs.top_mask(n)
        jb[-1] |= ~inputs.top_mask(n)
        assert np.array_equal(_single(ctx, n, ja, jb, gf2x.KIND_CYCLIC), oracle.mul_cyclic(a, b, n))
        assert np.array_equal(_single(ctx, n, ja, jb, gf2x.KIND_FULL), oracle.mul(a, b, n))


def _class_names():
    import ctypes
    lib = gf2x.load()
    seen = {}
    # probe the default table and the tuner-visible names via schedule_info on many sizes
    for n in range(32, gf2x.GF2X_MAX_BITS + 1, 32):
        s = ctypes.c_uint32()
        name = ctypes.create_string_buffer(64)
        lib.gf2x_schedule_info(None, n, ctypes.byref(s), None, None, name, 64)
        seen.setdefault(name.value.decode(), s.value)
    return seen


ALL_CLASSES = [
    ("U4", 4), ("U8", 8), ("K2^1.U8", 16), ("K2^2.U8", 32), ("K2^3.U8", 64), ("K2^4.U8", 128),
    ("K2^5.U8", 256), ("K2^5.U13", 416), ("T3.K2^4.U9", 426), ("T3.K2^5.U5", 474), ("T3.K2^5.U6", 570),
    ("T3.K2^4.U12", 570), ("T3.T3.K2^5.U3", 840), ("T3.K2^5.U9", 858), ("T3.T3.K2^5.U4", 1128),
    ("T3.T3.K2^5.U5", 1416), ("T3.T3.K2^4.U13", 1848), ("T3.T3.K2^5.U7", 1992), ("T3.T3.K2^5.U10", 2856),
    ("T3.T3.T3.K2^5.U4", 3378), ("T3.T3.T3.K2^5.U5", 4242),
    ("T3.K2^5.U7", 666), ("T3.K2^5.U4", 378), ("K2^5.U6", 192), ("K2^5.U9", 288),
    ("T4.K2^5.U9", 1140), ("T4.T3.K2^5.U5", 1884), ("T4.T3.K2^5.U4", 1500), ("K3.K2^5.U6", 576),
    ("K3.K2^5.U9", 864), ("K3.T3.K2^5.U5", 1422), ("K5.K2^5.U9", 1440), ("K5.K2^5.U6", 960),
    ("T3m.K2^5.U6", 570), ("T3m.K2^5.U5", 474), ("T3m.K2^5.U9", 858),
    ("T4m.K2^5.U9", 1140), ("T4m.T3.K2^5.U5", 1884), ("T4m.T3.K2^5.U4", 1500), ("T3m.T3.K2^5.U5", 1416),
    ("T3m.T3.K2^5.U4", 1128),
    ("G.T3.T3.K2^5.U4", 1128), ("G.T3.T3.K2^5.U5", 1416), ("G.T3.T3.K2^5.U7", 1992), ("G.T3.K2^5.U6", 570),
    ("G.T3.K2^5.U9", 858), ("G.T3.T3.T3.K2^5.U5", 4242),
    ("G.T4.T3.K2^5.U5", 1884), ("G.T4.T3.K2^5.U4", 1500), ("G.T4.K2^5.U9", 1140),
    ("G.T5.T3.K2^5.U4", 1850), ("G.T5.K2^5.U9", 1400),
]


@pytest.mark.parametrize("name,S", ALL_CLASSES)
def test_every_schedule_class(tmp_path, name, S):
    """Force each class through a tuner table and check a full-size and a ragged n,
    as single products (staged classes across several workgroups) and as a batch."""
    import torch
    ns = sorted({min(S * 32, gf2x.GF2X_MAX_BITS), max(1, min(S * 32, gf2x.GF2X_MAX_BITS) - 37)})
    table = tmp_path / "tune.txt"
    # the class serves batches and single products (a staged class then spreads
    # one product over several workgroups); a staged name in the direct column
    # is ignored, so device-resident items fall back to its direct form
    table.write_text("".join("%d %s %s %s\n" % ((n + 31) // 32, name, name, name) for n in ns))
    with gf2x.Context(0, tune_cache=str(table)) as c:
        for n in ns:
            assert c.schedule_info(n)[3] == name
            print("case class %s n=%d" % (name, n), flush=True)
            a = inputs.dense(n, SEED + 5, S, 0)
            b = inputs.dense(n, SEED + 5, S, 1)
            assert np.array_equal(_single(c, n, a, b, gf2x.KIND_CYCLIC), oracle.mul_cyclic(a, b, n))
            assert np.array_equal(_single(c, n, a, b, gf2x.KIND_FULL), oracle.mul(a, b, n))
            # a small batch, where staged classes take their staged path
            for kind in (gf2x.KIND_CYCLIC, gf2x.KIND_FULL):
                A, B, (C,) = _batched(c, n, 5, SEED + 5, kind=kind)
                for i in range(5):
                    ref = oracle.mul_cyclic(A[i], B[i], n) if kind == gf2x.KIND_CYCLIC else oracle.mul(A[i], B[i], n)
                    assert np.array_equal(C[i], ref), (name, n, kind, i)


def _batched(ctx, n, count, seed, kind=gf2x.KIND_CYCLIC, flags=0, reps=1):
    import torch
    W = oracle.words(n)
    A = inputs.dense_batch(n, count, seed, 0)
    B = inputs.dense_batch(n, count, seed, 1)
    cw = W if kind == gf2x.KIND_CYCLIC else 2 * W
    items = gf2x.make_items(n, kind, np.arange(count) * W, np.arange(count) * W, np.arange(count) * cw)
    dA, dB, dC = to_dev(A.ravel()), to_dev(B.ravel()), empty_dev(count * cw)
    outs = []
    for _ in range(reps):
        ctx.mul_batched(items, dC, dA, dB, flags)
        torch.cuda.synchronize()
        outs.append(from_dev(dC).reshape(count, cw))
    return A, B, outs


@pytest.mark.parametrize("n", [17669, 57637])
def test_batched_full_workload(ctx, n):
    """4096 products in one persistent launch (the batched workload): every
    item equal to the oracle."""
    count = 4096
    print("case batched n=%d count=%d" % (n, count), flush=True)
    A, B, (C,) = _batched(ctx, n, count, SEED + 2)
    assert np.array_equal(parity_rows(C), parity_rows(A) & parity_rows(B))
    ref = ring_rows(A, B, n)
    bad = np.nonzero((ref != C).any(axis=1))[0]
    assert len(bad) == 0, ("items differ from the oracle", bad[:10])


def test_batched_ragged_and_full_kind(ctx):
    n = 12323
    A, B, (C,) = _batched(ctx, n, 37, SEED + 6, kind=gf2x.KIND_FULL)
    for i in range(37):
        assert np.array_equal(C[i], oracle.mul(A[i], B[i], n))


def test_batched_graph_replays(ctx):
    n = 24659
    A, B, outs = _batched(ctx, n, 300, SEED + 7, flags=gf2x.USE_GRAPH, reps=3)
    for C in outs[1:]:
        assert np.array_equal(C, outs[0])
    for i in (0, 1, 150, 299):
        assert np.array_equal(outs[0][i], oracle.mul_cyclic(A[i], B[i], n))


def test_single_products_staged_and_captured(ctx):
    """Single products at sizes whose lowest-latency class is staged (several
    workgroups per product), eager and captured in a HIP graph (where the
    product is one launch of the direct class); every replay, with eager work
    in between, equals the oracle."""
    import torch
    for n in (17669, 57637):
        W = oracle.words(n)
        a = inputs.dense(n, SEED + 9, n, 0)
        b = inputs.dense(n, SEED + 9, n, 1)
        ref = oracle.mul_cyclic(a, b, n)
        dA, dB, dC = to_dev(a), to_dev(b), empty_dev(W)
        print("case single eager n=%d schedule %s" % (n, ctx.schedule_info(n)[3]), flush=True)
        ctx.mul_cyclic(dC, dA, dB, n)
        torch.cuda.synchronize()
        assert np.array_equal(from_dev(dC), ref)
        dG = empty_dev(W)
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):
            ctx.mul_cyclic(dG, dA, dB, n)  # warm-up outside the capture
        torch.cuda.current_stream().wait_stream(side)
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        print("case single captured n=%d" % n, flush=True)
        with torch.cuda.graph(g):
            ctx.mul_cyclic(dG, dA, dB, n)
        for rep in range(3):
            dG.zero_()
            ctx.mul_cyclic(dC, dB, dA, n)  # eager work between replays
            g.replay()
            torch.cuda.synchronize()
            assert np.array_equal(from_dev(dG), ref), (n, rep)
            assert np.array_equal(from_dev(dC), ref), (n, rep)


def test_batched_calls_refuse_stream_capture(ctx):
    """Batched products (host or device descriptors) and batched inverses on a
    stream under capture return GF2X_ENOTSUP and record nothing; the capture
    stays valid, and the same calls work eagerly afterwards."""
    import torch
    n, count = 12323, 4
    W = oracle.words(n)
    A = inputs.dense_batch(n, count, SEED + 10, 0)
    B = inputs.dense_batch(n, count, SEED + 10, 1)
    offs = np.arange(count) * W
    items = gf2x.make_items(n, gf2x.KIND_CYCLIC, offs, offs, offs)
    d_items = torch.from_numpy(items.view(np.uint8).copy()).cuda()
    dA, dB, dC = to_dev(A.ravel()), to_dev(B.ravel()), empty_dev(count * W)
    marker = torch.zeros(8, dtype=torch.int64, device="cuda")
    calls = {
        "host items": lambda: ctx.mul_batched(items, dC, dA, dB),
        "host items, graph": lambda: ctx.mul_batched(items, dC, dA, dB, gf2x.USE_GRAPH),
        "device items": lambda: ctx.mul_batched(d_items, dC, dA, dB, gf2x.ITEMS_ON_DEVICE, count=count),
        "inverse": lambda: ctx.inv_cyclic_batched(items, dC, dA),
    }
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    print("case batched calls under capture", flush=True)
    codes = {}
    with torch.cuda.graph(g):
        marker.add_(1)
        for name, call in calls.items():
            try:
                call()
                codes[name] = gf2x.GF2X_OK
            except gf2x.Gf2xError as e:
                codes[name] = e.code
    assert codes == {name: gf2x.GF2X_ENOTSUP for name in calls}, codes
    g.replay()
    torch.cuda.synchronize()
    assert int(marker[0]) == 1
    print("case batched calls eager after capture", flush=True)
    ctx.mul_batched(items, dC, dA, dB)
    torch.cuda.synchronize()
    C = from_dev(dC).reshape(count, W)
    for i in range(count):
        assert np.array_equal(C[i], oracle.mul_cyclic(A[i], B[i], n)), i


def test_batched_device_items(ctx):
    """Device-resident descriptors over a batch that mixes all six ring sizes
    (so every group of direct classes computes products) plus a few edge
    sizes and full products: every item equal to the oracle."""
    import torch
    rng = np.random.default_rng(8)
    sizes = [RING[i % 6] for i in range(240)] + [1, 65, 4097, 100000]
    sizes = [sizes[i] for i in rng.permutation(len(sizes))]
    kinds = [gf2x.KIND_FULL if i % 11 == 3 else gf2x.KIND_CYCLIC for i in range(len(sizes))]
    a_off, c_off, ao, co = [], [], 0, 0
    for n, k in zip(sizes, kinds):
        W = oracle.words(n)
        a_off.append(ao)
        c_off.append(co)
        ao += W
        co += W if k == gf2x.KIND_CYCLIC else 2 * W
    Abuf = np.zeros(ao, dtype=np.uint64)
    Bbuf = np.zeros(ao, dtype=np.uint64)
    for p, n in enumerate(sizes):
        W = oracle.words(n)
        Abuf[a_off[p]:a_off[p] + W] = inputs.dense(n, SEED + 8, p, 0)
        Bbuf[a_off[p]:a_off[p] + W] = inputs.dense(n, SEED + 8, p, 1)
    items = gf2x.make_items(np.array(sizes, np.uint32), np.array(kinds, np.uint32), a_off, a_off, c_off)
    d_items = torch.from_numpy(items.view(np.uint8).copy()).cuda()
    dA, dB, dC = to_dev(Abuf), to_dev(Bbuf), empty_dev(co)
    print("case device items, %d items of mixed sizes" % len(sizes), flush=True)
    ctx.mul_batched(d_items, dC, dA, dB, gf2x.ITEMS_ON_DEVICE, count=len(sizes))
    torch.cuda.synchronize()
    C = from_dev(dC)
    ring = [p for p in range(len(sizes)) if kinds[p] == gf2x.KIND_CYCLIC]
    sel = lambda xs: [xs[p] for p in ring]
    assert ring_mismatches(sel(sizes), sel(a_off), sel(a_off), sel(c_off), Abuf, Bbuf, C) == []
    for p in range(len(sizes)):
        if kinds[p] == gf2x.KIND_FULL:
            n, W = sizes[p], oracle.words(sizes[p])
            ref = oracle.mul(Abuf[a_off[p]:a_off[p] + W], Bbuf[a_off[p]:a_off[p] + W], n)
            assert np.array_equal(C[c_off[p]:c_off[p] + 2 * W], ref), p


def test_invalid_device_descriptors_are_counted(ctx):
    """Device-resident descriptors with n = 0, n above the maximum or an
    unknown kind are skipped (outputs untouched) and counted; the valid ones
    are computed."""
    import torch
    n = 12323
    W = oracle.words(n)
    A = inputs.dense_batch(n, 2, SEED + 11, 0)
    B = inputs.dense_batch(n, 2, SEED + 11, 1)
    items = gf2x.make_items(np.array([n, 0, n, gf2x.GF2X_MAX_BITS + 1, n], np.uint32),
                            np.array([0, 0, 7, 0, 0], np.uint32), [0, 0, 0, 0, W], [0, 0, 0, 0, W],
                            [0, W, 2 * W, 3 * W, 4 * W])
    d_items = torch.from_numpy(items.view(np.uint8).copy()).cuda()
    dC = empty_dev(5 * W)
    ctx.device_item_errors()  # clears any count left by earlier calls
    ctx.mul_batched(d_items, dC, to_dev(A.ravel()), to_dev(B.ravel()), gf2x.ITEMS_ON_DEVICE, count=5)
    assert ctx.device_item_errors() == 3
    assert ctx.device_item_errors() == 0
    C = from_dev(dC).reshape(5, W)
    assert np.array_equal(C[0], oracle.mul_cyclic(A[0], B[0], n))
    assert np.array_equal(C[4], oracle.mul_cyclic(A[1], B[1], n))
    untouched = np.full(W, 0x5A5A5A5A5A5A5A5A, dtype=np.uint64)
    for i in (1, 2, 3):
        assert np.array_equal(C[i], untouched), i


def test_mixed_batch_with_sparse_operands(ctx):
    """Mixed sizes, half dense x dense and half dense x sparse, one launch.
    Sparse items are also checked against the rotation closed form."""
    import torch
    from tests import brute
    count = 96
    rng = np.random.default_rng(4)
    sizes = [RING[int(u)] for u in rng.integers(0, 6, count)]
    offs, off = [], 0
    for n in sizes:
        offs.append(off)
        off += oracle.words(n)
    Abuf = np.zeros(off, dtype=np.uint64)
    Bbuf = np.zeros(off, dtype=np.uint64)
    sparse_pos = {}
    for p, n in enumerate(sizes):
        W = oracle.words(n)
        Abuf[offs[p]:offs[p] + W] = inputs.dense(n, SEED + 4, p, 0)
        if p % 2:
            pos = inputs.sparse_positions(n, inputs.sparse_weight_for(n), SEED + 4, p)
            sparse_pos[p] = pos
            Bbuf[offs[p]:offs[p] + W] = inputs.from_positions(n, pos)
        else:
            Bbuf[offs[p]:offs[p] + W] = inputs.dense(n, SEED + 4, p, 1)
    items = gf2x.make_items(sizes, gf2x.KIND_CYCLIC, offs, offs, offs)
    dA, dB, dC = to_dev(Abuf), to_dev(Bbuf), empty_dev(off)
    ctx.mul_batched(items, dC, dA, dB)
    torch.cuda.synchronize()
    C = from_dev(dC)
    assert ring_mismatches(sizes, offs, offs, offs, Abuf, Bbuf, C) == []
    for p, n in enumerate(sizes):
        W = oracle.words(n)
        a, c = Abuf[offs[p]:offs[p] + W], C[offs[p]:offs[p] + W]
        if p in sparse_pos:
            xa = brute.words_to_int(a)
            expect = 0
            for q in sparse_pos[p]:
                expect ^= brute.rotate(xa, q, n)
            assert brute.words_to_int(c) == expect


def test_determinism_across_orders(ctx):
    """Same products computed in a different item order and grid give identical words."""
    import torch
    n = 17669
    count = 600
    W = oracle.words(n)
    A = inputs.dense_batch(n, count, SEED + 9, 0)
    B = inputs.dense_batch(n, count, SEED + 9, 1)
    dA, dB = to_dev(A.ravel()), to_dev(B.ravel())
    perm = np.random.default_rng(1).permutation(count)
    outs = []
    for order in (np.arange(count), perm, perm[:7]):
        items = gf2x.make_items(n, gf2x.KIND_CYCLIC, order * W, order * W, order * W)
        dC = empty_dev(count * W)
        ctx.mul_batched(items, dC, dA, dB)
        torch.cuda.synchronize()
        outs.append((order, from_dev(dC).reshape(count, W)))
    base = outs[0][1]
    for order, C in outs[1:]:
        assert np.array_equal(C[order], base[order])


def _shared(ctx, n, count, seed, flags):
    import torch
    W = oracle.words(n)
    h = inputs.dense(n, seed, 0, 0)
    R = inputs.dense_batch(n, count, seed, 1)
    items = gf2x.make_items(n, gf2x.KIND_CYCLIC, 0, np.arange(count) * W, np.arange(count) * W)
    dH, dR, dC = to_dev(h), to_dev(R.ravel()), empty_dev(count * W)
    ctx.mul_batched(items, dC, dH, dR, gf2x.SHARED_A | flags)
    torch.cuda.synchronize()
    return h, R, from_dev(dC).reshape(count, W)


@pytest.mark.parametrize("n,count", [(35851, 1024), (57637, 512)])
def test_shared_operand_toeplitz_and_packed(ctx, n, count):
    """The shared-operand workload through the int8-MFMA Toeplitz path and the
    bit-packed path: identical words, every item equal to the oracle."""
    print("case shared n=%d count=%d" % (n, count), flush=True)
    h, R, Ct = _shared(ctx, n, count, SEED + 3, gf2x.FORCE_TOEPLITZ)
    _, _, Cp = _shared(ctx, n, count, SEED + 3, gf2x.FORCE_PACKED)
    assert np.array_equal(Ct, Cp)
    ref = ring_rows(np.broadcast_to(h, R.shape), R, n)
    bad = np.nonzero((ref != Ct).any(axis=1))[0]
    assert len(bad) == 0, ("items differ from the oracle", bad[:10])


@pytest.mark.parametrize("n,count", [(1, 5), (63, 3), (64, 64), (65, 65), (1000, 130), (12323, 7), (17669, 100)])
def test_toeplitz_ragged(ctx, n, count):
    h, R, C = _shared(ctx, n, count, SEED + 5, gf2x.FORCE_TOEPLITZ)
    for i in range(count):
        assert np.array_equal(C[i], oracle.mul_cyclic(h, R[i], n)), i


def test_toeplitz_ignores_bits_above_n(ctx):
    import torch
    n, count = 17669, 70
    W = oracle.words(n)
    h = inputs.dense(n, SEED + 6, 0, 0)
    R = inputs.dense_batch(n, count, SEED + 6, 1)
    hj, Rj = h.copy(), R.copy()
    hj[-1] |= ~inputs.top_mask(n)
    Rj[:, -1] |= ~inputs.top_mask(n)
    items = gf2x.make_items(n, gf2x.KIND_CYCLIC, 0, np.arange(count) * W, np.arange(count) * W)
    dC = empty_dev(count * W)
    ctx.mul_batched(items, dC, to_dev(hj), to_dev(Rj.ravel()), gf2x.SHARED_A | gf2x.FORCE_TOEPLITZ)
    torch.cuda.synchronize()
    C = from_dev(dC).reshape(count, W)
    for i in (0, 33, 69):
        assert np.array_equal(C[i], oracle.mul_cyclic(h, R[i], n))


def test_argument_errors(ctx):
    import torch
    n = 100
    W = oracle.words(n)
    A = to_dev(np.zeros(W, dtype=np.uint64))
    C = empty_dev(2 * W)
    with pytest.raises(gf2x.Gf2xError) as e:
        ctx.mul_cyclic(C, A, A, 0)
    assert e.value.code == gf2x.GF2X_EINVAL
    with pytest.raises(gf2x.Gf2xError):
        ctx.mul_cyclic(C, A, A, gf2x.GF2X_MAX_BITS + 1)
    with pytest.raises(gf2x.Gf2xError):
        ctx.mul_cyclic(A, A, C, n)  # c overlaps a
    with pytest.raises(gf2x.Gf2xError):
        ctx.mul_cyclic(C.data_ptr() + 4, A, A, n)  # misaligned
    bad = gf2x.make_items(n, 7, 0, 0, 0)
    with pytest.raises(gf2x.Gf2xError):
        ctx.mul_batched(bad, C, A, A)
    with pytest.raises(gf2x.Gf2xError) as e:
        ctx.mul_batched(gf2x.make_items(n, 0, 0, 0, 0), C, A, A, gf2x.FORCE_TOEPLITZ)
    assert e.value.code == gf2x.GF2X_ENOTSUP
    two = gf2x.make_items(n, 0, [0, 1], 0, 0)  # SHARED_A with different a_off
    with pytest.raises(gf2x.Gf2xError) as e:
        ctx.mul_batched(two, C, A, A, gf2x.SHARED_A)
    assert e.value.code == gf2x.GF2X_EINVAL
    ctx.mul_batched(np.zeros(0, dtype=gf2x.ITEM_DTYPE), C, A, A)  # empty batch is a no-op


def test_overlapping_ranges_are_refused(ctx):
    """Host items: an output range that overlaps another item's output or any
    operand range is refused with GF2X_EINVAL (shared operands are allowed),
    on the plain call, the graph path, plans and the allocation-free call."""
    import torch

    n = 1000
    W = oracle.words(n)
    dX = empty_dev(16 * W)
    ok = gf2x.make_items(n, gf2x.KIND_CYCLIC, 0, 0, [8 * W, 9 * W])  # a, b shared, outputs apart
    ctx.mul_batched(ok, dX, dX, dX)
    cases = [
        gf2x.make_items(n, gf2x.KIND_CYCLIC, 0, 0, [8 * W, 9 * W - 1]),  # outputs overlap by one word
        gf2x.make_items(n, gf2x.KIND_FULL, 0, 0, [8 * W, 9 * W]),  # full outputs are 2 W words
        gf2x.make_items(n, gf2x.KIND_CYCLIC, [0, 8 * W + 3], 0, [8 * W, 10 * W]),  # a read from an output
        gf2x.make_items(n, gf2x.KIND_CYCLIC, 0, [0, 11 * W - 1], [8 * W, 10 * W]),  # b reaches into an output
        gf2x.make_items(n, gf2x.KIND_CYCLIC, 0, 0, [10 * W, 12 * W, 8 * W, 10 * W + 5]),  # unsorted; 1st and 4th overlap
        gf2x.make_items(n, gf2x.sparse_kind(5), 0, 10 * W + 2, [8 * W, 10 * W]),  # positions inside an output
    ]
    for items in cases:
        for flags in (0, gf2x.USE_GRAPH):
            with pytest.raises(gf2x.Gf2xError) as e:
                ctx.mul_batched(items, dX, dX, dX, flags)
            assert e.value.code == gf2x.GF2X_EINVAL
        with pytest.raises(gf2x.Gf2xError) as e:
            ctx.plan(items, dX, dX, dX)
        assert e.value.code == gf2x.GF2X_EINVAL
        with pytest.raises(gf2x.Gf2xError) as e:
            ctx.mul_batched_noalloc(items, dX, dX, dX)
        assert e.value.code == gf2x.GF2X_EINVAL
    # outputs in descending order, apart: accepted
    ctx.mul_batched(gf2x.make_items(n, gf2x.KIND_CYCLIC, 0, 0, [12 * W, 10 * W, 8 * W]), dX, dX, dX)
    torch.cuda.synchronize()
