"""Whole-batch checks against the CPU oracle: every item of a batch, spread
over a pool of host threads (the C oracle releases the GIL while it runs).

Test infrastructure: only the tests import this module."""
import os
from concurrent.futures import ThreadPoolExecutor

import numpy as np

import oracle


def threads():
    """Host threads for the oracle: the cores this process may use, at most 16."""
    return max(1, min(16, len(os.sched_getaffinity(0))))


def ring_rows(A, B, n):
    """Oracle ring products of the row pairs of A and B ((count, words(n)) arrays)."""
    A = np.ascontiguousarray(A, dtype=np.uint64)
    B = np.ascontiguousarray(B, dtype=np.uint64)
    count = A.shape[0]
    if count == 0:
        return np.zeros_like(A)
    k = min(threads(), count)
    bounds = np.linspace(0, count, k + 1).astype(int)
    out = np.zeros_like(A)

    def work(j):
        lo, hi = bounds[j], bounds[j + 1]
        if hi > lo:
            out[lo:hi] = oracle.mul_cyclic_many(A[lo:hi], B[lo:hi], n)

    with ThreadPoolExecutor(max_workers=k) as ex:
        list(ex.map(work, range(k)))
    return out


def _rows(buf, offs, W):
    idx = np.asarray(offs, dtype=np.int64)[:, None] + np.arange(W, dtype=np.int64)[None, :]
    return buf[idx]


def ring_mismatches(ns, a_off, b_off, c_off, Abuf, Bbuf, Cbuf):
    """Indices of the ring-product items whose result words in Cbuf differ
    from the oracle; items may mix sizes (grouped by n for the oracle)."""
    ns = np.asarray(ns)
    a_off, b_off, c_off = (np.asarray(x, dtype=np.uint64) for x in (a_off, b_off, c_off))
    bad = []
    for n in sorted(set(int(x) for x in ns.tolist())):
        idx = np.nonzero(ns == n)[0]
        W = oracle.words(n)
        ref = ring_rows(_rows(Abuf, a_off[idx], W), _rows(Bbuf, b_off[idx], W), n)
        got = _rows(Cbuf, c_off[idx], W)
        diff = np.nonzero((ref != got).any(axis=1))[0]
        bad.extend(int(i) for i in idx[diff])
    return sorted(bad)


def full_rows(A, B, n):
    """Oracle full products (2 * words(n) words each) of the row pairs."""
    return np.stack([oracle.mul(A[i], B[i], n) for i in range(A.shape[0])]) if A.shape[0] else np.zeros(
        (0, 2 * oracle.words(n)), dtype=np.uint64)
