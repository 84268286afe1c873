"""HQC-shaped serving trace: operations that are chains of dependent ring
products, through the continuous-batching server.

    python -m paper_2201_10473_amd.hqc_trace --rate 20000 --count 10000

An operation is a key generation, an encapsulation or a decapsulation at one
of the three HQC ring sizes (n = 17669, 35851, 57637), drawn uniformly.  Its
products form a chain of 1, 2 or 3 products: product k multiplies the result
of product k - 1 by a fresh operand, so it can only be submitted once the
previous one has completed.  (This keeps only the shape of the KEM's work: the
number of dependent ring products per operation.  Nothing else of HQC is
computed.)  Operations arrive as a Poisson process.  The first product of
each is submitted when its arrival time comes, carrying that time; the driver
submits each next product as soon as it sees the previous one completed.  The latency of an
operation runs from its arrival to the completion of its last product.
"""
import argparse
import json
import sys
import time

import numpy as np

from paper_2201_10473_amd import gf2x, inputs

HQC_SIZES = (17669, 35851, 57637)
CHAIN = {"keygen": 1, "encaps": 2, "decaps": 3}


def make_trace(count, seed):
    """Per operation: kind, n, and its operand / result words.  Operand 0 is
    the chain's first left operand; operand k (k >= 1) the right operand of
    product k; result k is written at res_off[op] + (k - 1) * W."""
    rng = np.random.default_rng(seed)
    kinds = np.array(list(CHAIN))[rng.integers(0, len(CHAIN), count)]
    ns = np.asarray(HQC_SIZES, dtype=np.uint32)[rng.integers(0, len(HQC_SIZES), count)]
    length = np.array([CHAIN[k] for k in kinds], dtype=np.int64)
    W = ((ns.astype(np.int64) + 63) // 64)
    opnd_words = W * (length + 1)
    res_words = W * length
    opnd_off = np.concatenate([[0], np.cumsum(opnd_words)[:-1]]).astype(np.uint64)
    res_off = np.concatenate([[0], np.cumsum(res_words)[:-1]]).astype(np.uint64)
    X = np.zeros(int(opnd_words.sum()), dtype=np.uint64)
    for i in range(count):
        n, w = int(ns[i]), int(W[i])
        for k in range(int(length[i]) + 1):
            X[int(opnd_off[i]) + k * w:int(opnd_off[i]) + (k + 1) * w] = inputs.dense(n, seed, i, k)
    R = np.empty(int(res_words.sum()), dtype=np.uint64)
    R.fill(0)  # map every page now, not inside the timed run
    return kinds, ns, length, W.astype(np.uint64), X, opnd_off, R, res_off


def _timer_slack(ns):
    """Set this thread's Linux timer slack (how late a sleep may end); returns
    the previous value, or None where it cannot be set."""
    try:
        import ctypes
        libc = ctypes.CDLL(None, use_errno=True)
        old = libc.prctl(30, 0, 0, 0, 0)  # PR_GET_TIMERSLACK
        if old < 0 or libc.prctl(29, ctypes.c_ulong(ns), 0, 0, 0) != 0:  # PR_SET_TIMERSLACK
            return None
        return old
    except (OSError, AttributeError):
        return None


def drive(srv, trace, arrival):
    """Serve the trace's operations through `srv` (a gf2x.Server, or any object
    with its submit / completion / now_ns methods).  The driver plays the
    clients: an operation's first product is submitted once its arrival time
    has come (stamped with that time), each next product once the previous one
    has completed.  The server admits its queue in order, so nothing queued may
    lie in the future.  Returns the completion stamp of each operation's last
    product and the number of products submitted."""
    kinds, ns, length, W, X, xo, R, ro = trace
    # the polls below sleep 10 us; with the default 50 us slack every link
    # of a chain would wait for the driver rather than for the server
    old_slack = _timer_slack(1)
    try:
        return _drive(srv, ns, length, W, X, xo, R, ro, arrival)
    finally:
        if old_slack is not None:
            _timer_slack(old_slack)


def _drive(srv, ns, length, W, X, xo, R, ro, arrival):
    count = len(ns)
    active = []  # submissions in flight: [first ticket, operations, steps, handled]
    done_at = np.zeros(count, dtype=np.uint64)
    products = 0
    nf = 0  # operations whose first product has been submitted
    while nf < count or active:
        upto = int(np.searchsorted(arrival, srv.now_ns(), side="right"))
        idle = upto == nf
        if upto > nf:
            o = np.arange(nf, upto)
            tf = srv.submit(ns[o], X, xo[o], X, xo[o] + W[o], R, ro[o], arrival[o])
            active.append([tf, o, np.ones(len(o), dtype=np.int64), np.zeros(len(o), dtype=bool)])
            products += len(o)
            nf = upto
        nxt_op, nxt_step = [], []
        for sub in active:
            tf, ops, steps, handled = sub
            stamps = srv.completion(tf, len(ops))
            new = (stamps != 0) & ~handled
            if not new.any():
                continue
            handled |= new
            o, st = ops[new], steps[new]
            last = st == length[o]
            done_at[o[last]] = stamps[new][last]
            nxt_op.append(o[~last])
            nxt_step.append(st[~last] + 1)
        active = [sub for sub in active if not sub[3].all()]
        ops = np.concatenate(nxt_op) if nxt_op else np.zeros(0, dtype=np.int64)
        if len(ops):
            steps = np.concatenate(nxt_step)
            k = steps.astype(np.uint64)
            # product k: result of product k-1 times operand k
            tf = srv.submit(ns[ops], R, ro[ops] + (k - 2) * W[ops], X, xo[ops] + k * W[ops], R,
                            ro[ops] + (k - 1) * W[ops])
            active.append([tf, ops, steps, np.zeros(len(ops), dtype=bool)])
            products += len(ops)
        elif idle:
            time.sleep(10e-6)
    return done_at, products


def arrivals(srv, rate, count, seed, start_delay_s=0.01):
    gaps = np.random.default_rng(seed).exponential(1.0 / rate, count)
    return (srv.now_ns() + int(start_delay_s * 1e9) + np.cumsum(gaps) * 1e9).astype(np.uint64)


def summarize(trace, arrival, done_at, products, rate):
    kinds = trace[0]
    count = len(kinds)
    lat_us = (done_at.astype(np.int64) - arrival.astype(np.int64)) / 1e3
    span_s = (int(done_at.max()) - int(arrival.min())) / 1e9
    per = {}
    for kind in CHAIN:
        sel = kinds == kind
        if not sel.any():
            continue
        per[kind] = {"count": int(sel.sum()), "products_per_op": CHAIN[kind],
                     "p50_us": round(float(np.percentile(lat_us[sel], 50)), 1),
                     "p99_us": round(float(np.percentile(lat_us[sel], 99)), 1)}
    return {"offered_op_rate": rate, "operations": count, "products": int(products),
            "achieved_op_rate": round(count / span_s, 1), "products_per_s": round(products / span_s, 1),
            "per_kind": per}


def run(ctx, rate, count, seed, warm=True):
    """Replay a Poisson process of `count` operations at `rate` per second.
    Before the timed replay, untimed: every size once, then 0.1 s of the same
    traffic (at least 1000 operations, a trace of its own)."""
    trace = make_trace(count, seed)
    with gf2x.Server(ctx) as srv:
        if warm:
            kinds, ns, length, W, X, xo, R, ro = trace
            wk = min(count, 64)
            srv.submit(ns[:wk], X, xo[:wk], X, xo[:wk] + W[:wk], R, ro[:wk])
            srv.drain()
            wtrace = make_trace(max(1000, int(rate * 0.1)), seed + 2)
            drive(srv, wtrace, arrivals(srv, rate, len(wtrace[1]), seed + 3))
            srv.drain()
            base = srv.stats()["batches"]
        else:
            base = 0
        arrival = arrivals(srv, rate, count, seed + 1)
        done_at, products = drive(srv, trace, arrival)
        srv.drain()
        batches = srv.stats()["batches"] - base
    result = summarize(trace, arrival, done_at, products, rate)
    result["server_batches"] = int(batches)
    return result, trace


def check_against_batched(ctx, trace):
    """Recompute every chain step by step with batched launches (no server,
    no interleaving) and compare with the served results; returns the number
    of products compared."""
    import torch

    kinds, ns, length, W, X, xo, R, ro = trace
    dX = torch.from_numpy(X.view(np.int64)).cuda()
    dR = torch.zeros(len(R), dtype=torch.int64, device="cuda")
    for k in range(1, int(length.max()) + 1):
        ops = np.nonzero(length >= k)[0]
        ku = np.uint64(k)
        left_base = dX if k == 1 else dR
        left_off = xo[ops] if k == 1 else ro[ops] + (ku - np.uint64(2)) * W[ops]
        items = gf2x.make_items(ns[ops], gf2x.KIND_CYCLIC, left_off, xo[ops] + ku * W[ops],
                                ro[ops] + (ku - np.uint64(1)) * W[ops])
        if k == 1:
            ctx.mul_batched(items, dR, dX, dX)
        else:
            # left operands are results of step k-1 (in dR), right ones in dX
            ctx.mul_batched(items, dR, left_base, dX)
        torch.cuda.synchronize()
    ref = dR.cpu().numpy().view(np.uint64)
    if not np.array_equal(ref, R):
        bad = np.nonzero(ref != R)[0]
        raise AssertionError("served chains differ from the batched recomputation at %d words" % len(bad))
    return int(length.sum())


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--rate", type=float, default=20000)
    ap.add_argument("--count", type=int, default=10000)
    ap.add_argument("--seed", type=int, default=inputs.SEED_BASE + 11)
    args = ap.parse_args()
    with gf2x.Context(0) as ctx:
        res, trace = run(ctx, args.rate, args.count, args.seed)
        res["checked_products"] = check_against_batched(ctx, trace)
    print(json.dumps(res))
    return 0


if __name__ == "__main__":
    sys.exit(main())
