"""Open-loop serving workload: Poisson arrivals of ring products of mixed n.

    python -m paper_2201_10473_amd.serve --rate 100000 --count 20000

Each request is one ring product with n drawn uniformly from the six ring
sizes and dense operands seeded by its request index.  All arrival times are
drawn up front (exponential gaps at the given rate) and handed to the
library's server, which admits each request no earlier than its arrival; the
latency of a request is its completion stamp minus its scheduled arrival.
"""
import argparse
import json
import sys

import numpy as np

from paper_2201_10473_amd import gf2x, inputs


def make_requests(count, seed, sizes=inputs.RING_SIZES):
    """Per request: n, and operand / result offsets into flat uint64 buffers."""
    rng = np.random.default_rng(seed)
    ns = np.asarray(sizes, dtype=np.uint32)[rng.integers(0, len(sizes), count)]
    W = (ns.astype(np.uint64) + 63) // 64
    off = np.concatenate([[0], np.cumsum(W)[:-1]]).astype(np.uint64)
    total = int(W.sum())
    A = np.zeros(total, dtype=np.uint64)
    B = np.zeros(total, dtype=np.uint64)
    for n in sizes:
        idx = np.nonzero(ns == n)[0]
        if len(idx) == 0:
            continue
        w = (n + 63) // 64
        blockA = inputs.dense_items(n, idx, seed, 0)
        blockB = inputs.dense_items(n, idx, seed, 1)
        pos = (off[idx][:, None] + np.arange(w, dtype=np.uint64)[None, :]).ravel()
        A[pos] = blockA.ravel()
        B[pos] = blockB.ravel()
    return ns, off, A, B


def warm_up(srv, seed, requests=None, rate=0.0, count=0):
    """Before the timed run, and not part of the measurement: a few requests
    of every size through the server (loads every kernel the workload uses),
    then a replay of the first `count` timed requests at `rate`.  The first
    replay in a process runs slower for its first tens of milliseconds (its
    p99 is several ms higher); the timed replay measures the steady state."""
    ns, off, A, B = make_requests(6 * 8, seed, sizes=inputs.RING_SIZES)
    C = np.zeros_like(A)
    srv.submit(ns, A, off, B, off, C, off)
    srv.drain()
    if requests is not None and rate > 0 and count > 0:
        rns, rA, roff, rB, rC = requests
        k = min(count, len(rns))
        gaps = np.random.default_rng(seed).exponential(1.0 / rate, k)
        arrival = (srv.now_ns() + int(0.005 * 1e9) + np.cumsum(gaps) * 1e9).astype(np.uint64)
        srv.submit(rns[:k], rA, roff[:k], rB, roff[:k], rC, roff[:k], arrival)
        srv.drain()


def run(ctx, rate, count, seed, hbm_budget_bytes=0, streams=0, start_delay_s=0.01, warm=True, max_batch=0,
        warm_requests=None):
    """Replay a Poisson process of `count` requests at `rate` per second."""
    ns, off, A, B = make_requests(count, seed)
    # write every page of the result buffer now: fresh zero pages are mapped
    # on first write, which would otherwise be timed inside the first batches
    C = np.empty_like(A)
    C.fill(0)
    rng = np.random.default_rng(seed + 1)
    gaps = rng.exponential(1.0 / rate, count)
    with gf2x.Server(ctx, hbm_budget_bytes=hbm_budget_bytes, streams=streams, max_batch=max_batch) as srv:
        if warm:
            # warm-up replay: 0.3 s of traffic at the same rate (at least 2000 requests)
            k = warm_requests if warm_requests is not None else max(2000, int(rate * 0.3))
            warm_up(srv, seed + 2, (ns, A, off, B, C), rate, k)
            base = srv.stats()
        else:
            base = None
        t0 = srv.now_ns() + int(start_delay_s * 1e9)
        arrival = (t0 + np.cumsum(gaps) * 1e9).astype(np.uint64)
        first = srv.submit(ns, A, off, B, off, C, off, arrival)
        srv.drain()
        done = srv.completion(first, count)
        stats = srv.stats()
        if base:  # counters of the timed requests only
            for k in ("submitted", "admitted", "completed", "batches", "launches", "phased_batches",
                      "host_pack_ns", "host_issue_ns", "host_retire_ns"):
                stats[k] -= base[k]
    lat_us = (done.astype(np.int64) - arrival.astype(np.int64)) / 1e3
    span_s = (int(done.max()) - int(arrival.min())) / 1e9
    per_n = {}
    for n in sorted(set(ns.tolist())):
        sel = lat_us[ns == n]
        per_n[str(n)] = {
            "count": int(len(sel)),
            "p50_us": round(float(np.percentile(sel, 50)), 1),
            "p99_us": round(float(np.percentile(sel, 99)), 1),
        }
    result = {
        "offered_rate": rate,
        "requests": count,
        "achieved_rate": round(count / span_s, 1),
        "p50_us": round(float(np.percentile(lat_us, 50)), 1),
        "p99_us": round(float(np.percentile(lat_us, 99)), 1),
        "per_n": per_n,
        "server": {k: int(v) for k, v in stats.items()},
        # where the longest scheduler iteration fell: ms after the first arrival
        "loop_busy_max_at_ms": round((int(stats["loop_busy_max_at_ns"]) - int(arrival.min())) / 1e6, 3),
    }
    return result, (ns, off, A, B, C)


def check_against_batched(ctx, ns, off, A, B, C):
    """Every served result equals the same product computed in one batched
    launch (same operands, no mix); returns the number of requests checked."""
    import torch

    count = len(ns)
    items = gf2x.make_items(ns, gf2x.KIND_CYCLIC, off, off, off)
    dA = torch.from_numpy(A.view(np.int64)).cuda()
    dB = torch.from_numpy(B.view(np.int64)).cuda()
    dC = torch.zeros(len(A), dtype=torch.int64, device="cuda")
    ctx.mul_batched(items, dC, dA, dB)
    torch.cuda.synchronize()
    ref = dC.cpu().numpy().view(np.uint64)
    if not np.array_equal(ref, C):
        bad = np.nonzero(ref != C)[0]
        raise AssertionError("served results differ from the batched launch at %d words" % len(bad))
    return count


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--rate", type=float, default=100000)
    ap.add_argument("--count", type=int, default=20000)
    ap.add_argument("--seed", type=int, default=inputs.SEED_BASE + 5)
    ap.add_argument("--budget-mib", type=int, default=256)
    ap.add_argument("--streams", type=int, default=0)
    ap.add_argument("--max-batch", type=int, default=0)
    args = ap.parse_args()
    with gf2x.Context(0) as ctx:
        res, bufs = run(ctx, args.rate, args.count, args.seed, args.budget_mib << 20, args.streams,
                        max_batch=args.max_batch)
        check_against_batched(ctx, *bufs)
    print(json.dumps(res))
    return 0


if __name__ == "__main__":
    sys.exit(main())
