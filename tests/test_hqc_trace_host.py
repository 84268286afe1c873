"""Host side of the HQC-shaped trace: the operation mix, the buffer layout
(operands and results of different operations never overlap) and seeding."""
import numpy as np

from paper_2201_10473_amd import hqc_trace, inputs


def test_trace_layout_and_seeding():
    tr = hqc_trace.make_trace(300, inputs.SEED_BASE + 11)
    kinds, ns, length, W, X, xo, R, ro = tr
    assert set(kinds.tolist()) == set(hqc_trace.CHAIN)
    assert set(ns.tolist()) == set(hqc_trace.HQC_SIZES)
    assert all(length[i] == hqc_trace.CHAIN[k] for i, k in enumerate(kinds))
    assert np.array_equal(W, (ns.astype(np.uint64) + 63) // 64)
    # operation i owns operands [xo, xo + W*(L+1)) and results [ro, ro + W*L), back to back
    assert np.array_equal(xo[1:], xo[:-1] + W[:-1] * (length[:-1] + 1).astype(np.uint64))
    assert np.array_equal(ro[1:], ro[:-1] + W[:-1] * length[:-1].astype(np.uint64))
    assert len(X) == int(xo[-1] + W[-1] * np.uint64(length[-1] + 1))
    assert len(R) == int(ro[-1] + W[-1] * np.uint64(length[-1]))
    assert not R.any()
    # operands are the seeded dense generator's, bits >= n clear
    for i in (0, 7, 299):
        w, n = int(W[i]), int(ns[i])
        for k in range(int(length[i]) + 1):
            blk = X[int(xo[i]) + k * w:int(xo[i]) + (k + 1) * w]
            assert np.array_equal(blk, inputs.dense(n, inputs.SEED_BASE + 11, i, k))
            assert int(blk[-1]) >> (n % 64) == 0
    again = hqc_trace.make_trace(300, inputs.SEED_BASE + 11)
    for x, y in zip(tr, again):
        assert np.array_equal(x, y)


class InOrderServer:
    """Stand-in for gf2x.Server with the same admission rule: the queue is
    served in submission order and its head only once its arrival time has
    passed.  Its "product" is the word-wise XOR of the operands, enough to
    check which operands and results each request touches."""

    def __init__(self):
        self.queue = []
        self.done = []
        self.head = 0

    def now_ns(self):
        import time
        return time.monotonic_ns()

    def submit(self, n_bits, a, a_off, b, b_off, c, c_off, arrival_ns=None):
        first = len(self.done)
        now = self.now_ns()
        for i in range(len(n_bits)):
            t = int(arrival_ns[i]) if arrival_ns is not None else now
            self.queue.append((int(n_bits[i]), a, int(a_off[i]), b, int(b_off[i]), c, int(c_off[i]), t))
            self.done.append(0)
        return first

    def _pump(self):
        now = self.now_ns()
        while self.head < len(self.queue) and self.queue[self.head][7] <= now:
            n, a, ao, b, bo, c, co, _ = self.queue[self.head]
            w = (n + 63) // 64
            c[co:co + w] = a[ao:ao + w] ^ b[bo:bo + w]
            self.done[self.head] = now
            self.head += 1

    def completion(self, first, count):
        self._pump()
        return np.array(self.done[first:first + count], dtype=np.uint64)


def test_driver_chains_and_no_head_of_line_wait():
    count, rate = 300, 3000.0
    tr = hqc_trace.make_trace(count, inputs.SEED_BASE + 11)
    kinds, ns, length, W, X, xo, R, ro = tr
    srv = InOrderServer()
    arrival = hqc_trace.arrivals(srv, rate, count, inputs.SEED_BASE + 12, start_delay_s=0.002)
    done_at, products = hqc_trace.drive(srv, tr, arrival)
    assert products == int(length.sum()) == len(srv.queue)
    assert (done_at >= arrival).all()
    # result k of each chain is operand 0 ^ ... ^ operand k under the stand-in product
    for i in range(count):
        w, x0, r0 = int(W[i]), int(xo[i]), int(ro[i])
        acc = X[x0:x0 + w].copy()
        for k in range(1, int(length[i]) + 1):
            acc ^= X[x0 + k * w:x0 + (k + 1) * w]
            assert np.array_equal(R[r0 + (k - 1) * w:r0 + k * w], acc), (i, k)
    # each next product is submitted on completion of the previous one, not
    # behind first products that have not arrived yet: chains finish in a
    # small part of the 100 ms trace
    lat_ms = (done_at.astype(np.int64) - arrival.astype(np.int64)) / 1e6
    span_ms = (int(done_at.max()) - int(arrival.min())) / 1e6
    assert np.median(lat_ms[length == 3]) < 0.1 * span_ms, (np.median(lat_ms[length == 3]), span_ms)
    res = hqc_trace.summarize(tr, arrival, done_at, products, rate)
    assert sum(v["count"] for v in res["per_kind"].values()) == count
