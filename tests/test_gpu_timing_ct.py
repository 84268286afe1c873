"""Timing side of the constant-time check (the instruction-counter side is
paper_2201_10473_amd/ct_check.py under rocprofv3): a Welch t-test between
launch times of ring products with one fixed operand set and with varying
random operand sets, classes interleaved at random, top 10% of each class
cropped (the dudect method of Reparaz, Balasch and Verbauwhede, DATE 2017).

The fixed set is itself uniformly random (same Hamming-weight statistics as
the varying sets).  Degenerate operands such as all-zero words do run a few
percent faster with the identical instruction stream: the chip's clock
management reacts to the power drawn by toggling bits.  That effect is
measured and printed by test_all_zero_power_effect_is_reported, not asserted
away: it is outside what the kernels' control flow and addressing can
control."""
import numpy as np
import pytest

from paper_2201_10473_amd import gf2x, inputs

pytestmark = pytest.mark.gpu


def welch_t(x, y):
    x, y = np.asarray(x, float), np.asarray(y, float)
    return (x.mean() - y.mean()) / np.sqrt(x.var(ddof=1) / len(x) + y.var(ddof=1) / len(y))


def _timings(n, count, fixed_kind, reps, seed):
    import torch
    W = (n + 63) // 64
    rng = np.random.default_rng(n + count + seed)
    if fixed_kind == "zero":
        fixed = (np.zeros((count, W), dtype=np.uint64),) * 2
    else:
        fixed = (inputs.dense_batch(n, count, seed + 100, 0), inputs.dense_batch(n, count, seed + 100, 1))
    # the random class draws from 8 distinct random operand sets
    sets = [(inputs.dense_batch(n, count, seed + k, 0), inputs.dense_batch(n, count, seed + k, 1)) for k in range(8)]
    dev = lambda x: torch.from_numpy(np.ascontiguousarray(x).ravel().view(np.int64)).cuda()
    F = (dev(fixed[0]), dev(fixed[1]))
    R = [(dev(a), dev(b)) for a, b in sets]
    # both classes are copied into the same operand buffers right before each
    # timed launch, so that they see the same memory and cache state
    A, B = torch.empty_like(F[0]), torch.empty_like(F[1])
    C = torch.zeros(count * W, dtype=torch.int64, device="cuda")
    items = gf2x.make_items(n, gf2x.KIND_CYCLIC, np.arange(count) * W, np.arange(count) * W, np.arange(count) * W)
    times = {0: [], 1: []}
    with gf2x.Context(0) as ctx:
        def launch(cls, k):
            a, b = F if cls == 0 else R[k % 8]
            A.copy_(a)
            B.copy_(b)
            s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            s.record()
            if count == 1:
                ctx.mul_cyclic(C, A, B, n)
            else:
                ctx.mul_batched(items, C, A, B)
            e.record()
            return s, e
        for k in range(20):
            launch(1, k)
        torch.cuda.synchronize()
        for k, cls in enumerate(rng.integers(0, 2, 2 * reps)):
            s, e = launch(int(cls), k)
            torch.cuda.synchronize()
            times[int(cls)].append(s.elapsed_time(e))
    crop = lambda v: np.sort(v)[: int(0.9 * len(v))]
    return times, welch_t(crop(times[0]), crop(times[1]))


@pytest.mark.parametrize("n,count", [(17669, 1), (17669, 1024), (57637, 256)])
def test_fixed_vs_random_timing(n, count):
    print("case ct timing n=%d count=%d" % (n, count), flush=True)
    times, t = _timings(n, count, "random", 600 if count == 1 else 200, 11)
    print("n=%d count=%d mean fixed %.4f ms random %.4f ms t=%.2f" % (
        n, count, np.mean(times[0]), np.mean(times[1]), t), flush=True)
    # dudect flags |t| > 4.5 as a possible and |t| > 10 as a definite leak; the
    # definite threshold keeps GPU clock noise from failing the suite, and
    # still catches an effect of the size the all-zero case shows (|t| ~ 16-26)
    assert abs(t) < 10


def test_all_zero_power_effect_is_reported():
    """All-zero operands against random ones: printed for the record (the
    difference, if any, comes from clock management, not from the code)."""
    times, t = _timings(17669, 1024, "zero", 200, 13)
    print("all-zero vs random, n=17669 x 1024: mean %.4f vs %.4f ms, t=%.2f" % (
        np.mean(times[0]), np.mean(times[1]), t), flush=True)
    assert np.isfinite(t)
