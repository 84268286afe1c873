"""Throughput of ring products in F2[X]/(X^n - 1) on one MI355X.

Workload (one step): 4096 independent dense x dense ring products at
n = 17669 (277 uint64 words per operand), uniform seeded operands, all in
one persistent launch (a recorded plan replayed once per step).
Reported value: products per second over the timed steps, inputs already
resident in HBM.

Also measured (reported under "extra"): the same batch at n = 57637, and
both sizes as 4096 back-to-back single-product launches (one per product)
for the batched / one-per-launch factor.

roofline: the dominant kernel is the batched product kernel; it is bound by
VALU integer throughput.  achieved = modelled algorithmic lane-ops of the
schedule (base-case bit operations plus XOR passes, as reported by
gf2x_schedule_info) x products per launch / mean launch time, measured with
one pair of HIP events on the launch stream around the timed steps (their
span over the step count); peak = 256 CU x 4 SIMD
x 32 lanes per clock x 2.4 GHz = 78.6 T lane-ops/s (a SIMD issues one 32-bit
wave64 op every two clocks).

cpu_baseline: the CPU oracle (word schoolbook + fold) timed on the host
over a bounded sample of the same workload: all usable cores (at most 16
threads), and one thread pinned to one core; the CPU model is reported.  A
separate line times the oracle's fast mode (the CPU's PCLMULQDQ for the
64x64 carry-less multiply) on the same sample.
"""
import argparse
import json
import os
import sys
import tempfile
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "products/sec at n=17669 & 57637 (batched vs one-per-launch); % int-op roofline"
VALU_PEAK = 256 * 4 * 32 * 2.4e9  # int32 lane-ops per second: 256 CU x 4 SIMD x 32 lanes per clock
INT8_PEAK = 5.0e15  # dense int8 matrix ops per second (2 per multiply-add)
BATCH = 4096


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def make_batch(n, count, seed):
    import numpy as np
    import torch

    from paper_2201_10473_amd import gf2x, inputs

    W = gf2x.words(n)
    A = inputs.dense_batch(n, count, seed, 0)
    B = inputs.dense_batch(n, count, seed, 1)
    items = gf2x.make_items(n, gf2x.KIND_CYCLIC, np.arange(count) * W, np.arange(count) * W, np.arange(count) * W)
    dA = torch.from_numpy(A.ravel().view(np.int64)).cuda()
    dB = torch.from_numpy(B.ravel().view(np.int64)).cuda()
    dC = torch.zeros(count * W, dtype=torch.int64, device="cuda")
    return A, B, items, dA, dB, dC


def time_batched(ctx, n, count, steps, warmup, seed):
    import torch

    from paper_2201_10473_amd import gf2x

    A, B, items, dA, dB, dC = make_batch(n, count, seed)
    stream = torch.cuda.current_stream()
    plan = ctx.plan(items, dC, dA, dB)
    # warm-up: the requested steps, and at least ~0.5 s of device work so the
    # engine clock has settled before the timed region
    t0 = time.perf_counter()
    done = 0
    while done < max(warmup, 1) or time.perf_counter() - t0 < 0.5:
        plan.launch(stream)
        torch.cuda.synchronize()
        done += 1
    # one pair of HIP events on the launch stream around the timed steps: their
    # span over the step count is the average launch duration
    s_ev, e_ev = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s_ev.record(stream)
    for _ in range(steps):
        plan.launch(stream)
    e_ev.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    launch_ms = s_ev.elapsed_time(e_ev) / steps
    plan.close()
    return {"A": A, "B": B, "C": dC, "wall_s": wall, "launch_ms": launch_ms, "items": items}


def time_paper_method(ctx, count=4096, seeds=10, reps=20, warmup=3):
    """The measurement method of the paper's Appendix E, per ring size: for
    each of `seeds` seeded batches, `warmup` untimed replays, then the minimum
    over `reps` timed replays (HIP events around the whole batch on the launch
    stream); the minima are averaged over the seeds."""
    import numpy as np
    import torch

    from paper_2201_10473_amd import inputs

    stream = torch.cuda.current_stream()
    out = {}
    for n in inputs.RING_SIZES:
        # every seed's operands are resident before the first timed replay, and
        # 0.3 s of replays settle the engine clock after the uploads
        batches = [make_batch(n, count, inputs.SEED_BASE + 100 + k)[2:] for k in range(seeds)]
        items, dA, dB, dC = batches[0]
        with ctx.plan(items, dC, dA, dB) as plan:
            t0 = time.perf_counter()
            while time.perf_counter() - t0 < 0.3:
                plan.launch(stream)
                torch.cuda.synchronize()
        mins = []
        for items, dA, dB, dC in batches:
            with ctx.plan(items, dC, dA, dB) as plan:
                for _ in range(warmup):
                    plan.launch(stream)
                ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
                      for _ in range(reps)]
                for s_ev, e_ev in ev:
                    s_ev.record(stream)
                    plan.launch(stream)
                    e_ev.record(stream)
                torch.cuda.synchronize()
                mins.append(min(s_ev.elapsed_time(e_ev) for s_ev, e_ev in ev))
        del batches
        ms = float(np.mean(mins))
        out[str(n)] = {"batch": count, "ms_per_batch": round(ms, 4), "products_per_s": round(count / (ms * 1e-3), 1),
                       "min_ms_over_seeds": round(min(mins), 4), "max_ms_over_seeds": round(max(mins), 4),
                       "schedule": ctx.schedule_info(n)[3]}
    return out


def time_one_per_launch(ctx, n, count, seed):
    import torch

    from paper_2201_10473_amd import gf2x

    A, B, items, dA, dB, dC = make_batch(n, count, seed)
    W = gf2x.words(n)
    stream = torch.cuda.current_stream()
    base_c, base_a, base_b = dC.data_ptr(), dA.data_ptr(), dB.data_ptr()
    s = stream.cuda_stream
    for i in range(8):  # warm-up
        ctx.mul_cyclic(base_c + 8 * W * i, base_a + 8 * W * i, base_b + 8 * W * i, n, s)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(count):
        off = 8 * W * i
        ctx.mul_cyclic(base_c + off, base_a + off, base_b + off, n, s)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    return {"A": A, "B": B, "C": dC, "wall_s": wall}


def time_shared(ctx, n, count, flags, steps, seed):
    """Shared-operand batch (one h, `count` vectors r_i) through the path pinned by flags."""
    import numpy as np
    import torch

    from paper_2201_10473_amd import gf2x, inputs

    W = gf2x.words(n)
    h = inputs.dense(n, seed, 0, 0)
    R = inputs.dense_batch(n, count, seed, 1)
    items = gf2x.make_items(n, gf2x.KIND_CYCLIC, 0, np.arange(count) * W, np.arange(count) * W)
    dH = torch.from_numpy(h.view(np.int64)).cuda()
    dR = torch.from_numpy(R.ravel().view(np.int64)).cuda()
    dC = torch.zeros(count * W, dtype=torch.int64, device="cuda")
    f = gf2x.SHARED_A | flags
    t0 = time.perf_counter()
    while time.perf_counter() - t0 < 0.3:
        ctx.mul_batched(items, dC, dH, dR, f)
        torch.cuda.synchronize()
    s_ev, e_ev = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    s_ev.record()
    for _ in range(steps):
        ctx.mul_batched(items, dC, dH, dR, f)
    e_ev.record()
    torch.cuda.synchronize()
    ms = s_ev.elapsed_time(e_ev) / steps
    C = dC.cpu().numpy().view(np.uint64).reshape(count, W)
    return ms, h, R, C


def time_mixed(ctx, steps, seed, count=8192):
    """The mixed workload: n uniform over the six ring sizes, odd items dense x
    sparse (weight by size level), all in one graph-captured launch sequence."""
    import numpy as np
    import torch

    from paper_2201_10473_amd import gf2x, inputs, serve

    ns, off, A, B = serve.make_requests(count, seed)
    for i in range(1, count, 2):
        n = int(ns[i])
        W = (n + 63) // 64
        B[int(off[i]):int(off[i]) + W] = inputs.sparse(n, inputs.sparse_weight_for(n), seed, i)
    items = gf2x.make_items(ns, gf2x.KIND_CYCLIC, off, off, off)
    dA = torch.from_numpy(A.view(np.int64)).cuda()
    dB = torch.from_numpy(B.view(np.int64)).cuda()
    dC = torch.zeros(len(A), dtype=torch.int64, device="cuda")
    t0 = time.perf_counter()
    while time.perf_counter() - t0 < 0.3:
        ctx.mul_batched(items, dC, dA, dB, gf2x.USE_GRAPH)
        torch.cuda.synchronize()
    s_ev, e_ev = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    s_ev.record()
    for _ in range(steps):
        ctx.mul_batched(items, dC, dA, dB, gf2x.USE_GRAPH)
    e_ev.record()
    torch.cuda.synchronize()
    ms = s_ev.elapsed_time(e_ev) / steps
    C = dC.cpu().numpy().view(np.uint64)
    for i in (0, 1, count - 1):
        n = int(ns[i])
        W = (n + 63) // 64
        sl = slice(int(off[i]), int(off[i]) + W)
        if not np.array_equal(C[sl], single_product(ctx, A[sl], B[sl], n)):
            raise AssertionError("mixed workload item %d differs from the single-product path" % i)
    ops = sum(ctx.schedule_info(int(n))[2] for n in ns)
    # the same batch as one persistent launch (work queue over the direct classes)
    dF = torch.zeros(len(A), dtype=torch.int64, device="cuda")
    ms_fused = _plan_ms(ctx, items, dF, dA, dB, steps, gf2x.FUSED)
    if not torch.equal(dF, dC):
        raise AssertionError("mixed workload: fused launch differs from the per-class launches")
    return {"products": count, "ms_per_launch": round(ms, 4), "products_per_s": round(count / (ms * 1e-3), 1),
            "valu_frac": round(ops / (ms * 1e-3) / VALU_PEAK, 4),
            "fused_ms_per_launch": round(ms_fused, 4), "fused_products_per_s": round(count / (ms_fused * 1e-3), 1)}


def _plan_ms(ctx, items, dC, dA, dB, steps, flags=0):
    """Mean device time of one replay of a recorded batch (HIP events on the
    launch stream), after at least 0.3 s of warm-up replays."""
    import torch

    stream = torch.cuda.current_stream()
    with ctx.plan(items, dC, dA, dB, flags) as plan:
        t0 = time.perf_counter()
        while time.perf_counter() - t0 < 0.3:
            plan.launch(stream)
            torch.cuda.synchronize()
        s_ev, e_ev = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        s_ev.record(stream)
        for _ in range(steps):
            plan.launch(stream)
        e_ev.record(stream)
        torch.cuda.synchronize()
    return s_ev.elapsed_time(e_ev) / steps


def time_sparse(ctx, steps, seed, count=4096):
    """Dense x sparse ring products at each ring size (weights of the mixed
    workload), through the constant-time rotation barrel (sparse kind, the
    positions as input) and through the dense path (the sparse operand as a
    dense polynomial); both checked equal on every item."""
    import numpy as np
    import torch

    from paper_2201_10473_amd import gf2x, inputs

    out = {}
    for n in inputs.RING_SIZES:
        w = inputs.sparse_weight_for(n)
        W = gf2x.words(n)
        A = inputs.dense_batch(n, count, seed, 0)
        pos = [inputs.sparse_positions(n, w, seed, i) for i in range(count)]
        P = np.zeros(count * ((w + 1) // 2), dtype=np.uint64)
        P.view(np.uint32).reshape(count, -1)[:, :w] = np.asarray(pos, dtype=np.uint32)
        S = np.stack([inputs.from_positions(n, p) for p in pos])
        off = np.arange(count, dtype=np.uint64) * W
        poff = np.arange(count, dtype=np.uint64) * ((w + 1) // 2)
        sp_items = gf2x.make_items(n, gf2x.sparse_kind(w), off, poff, off)
        de_items = gf2x.make_items(n, gf2x.KIND_CYCLIC, off, off, off)
        dA = torch.from_numpy(A.ravel().view(np.int64)).cuda()
        dP = torch.from_numpy(P.view(np.int64)).cuda()
        dS = torch.from_numpy(S.ravel().view(np.int64)).cuda()
        dC1 = torch.zeros(count * W, dtype=torch.int64, device="cuda")
        dC2 = torch.zeros(count * W, dtype=torch.int64, device="cuda")
        ms_sp = _plan_ms(ctx, sp_items, dC1, dA, dP, steps)
        ms_de = _plan_ms(ctx, de_items, dC2, dA, dS, steps)
        if not torch.equal(dC1, dC2):
            raise AssertionError("sparse and dense paths disagree at n=%d" % n)
        out[str(n)] = {"weight": w, "batch": count, "sparse_ms": round(ms_sp, 4), "dense_ms": round(ms_de, 4),
                       "sparse_products_per_s": round(count / (ms_sp * 1e-3), 1),
                       "dense_products_per_s": round(count / (ms_de * 1e-3), 1),
                       "sparse_over_dense": round(ms_de / ms_sp, 3)}
        log("  n=%d w=%d: sparse %.3f ms, dense %.3f ms per %d products" % (n, w, ms_sp, ms_de, count))
    return out


def time_mixed_sparse(ctx, steps, seed, count=8192):
    """The mixed workload with its dense x sparse half given as positions
    (sparse kind): one recorded plan, every result equal to the same
    workload computed with the sparse operands as dense polynomials."""
    import numpy as np
    import torch

    from paper_2201_10473_amd import gf2x, inputs, serve

    ns, off, A, B = serve.make_requests(count, seed)
    pos_words, pos_off, sp_kind = [], [], []
    total = len(B)
    for i in range(1, count, 2):
        n = int(ns[i])
        w = inputs.sparse_weight_for(n)
        p = inputs.sparse_positions(n, w, seed, i)
        W = (n + 63) // 64
        B[int(off[i]):int(off[i]) + W] = inputs.from_positions(n, p)
        words = np.zeros((w + 1) // 2, dtype=np.uint64)
        words.view(np.uint32)[:w] = np.asarray(p, dtype=np.uint32)
        pos_words.append(words)
        pos_off.append(total)
        total += len(words)
        sp_kind.append(gf2x.sparse_kind(w))
    Bs = np.concatenate([B] + pos_words)
    kinds = np.zeros(count, dtype=np.uint32)
    kinds[1::2] = sp_kind
    b_off = off.copy()
    b_off[1::2] = pos_off
    items_sp = gf2x.make_items(ns, kinds, off, b_off, off)
    items_de = gf2x.make_items(ns, gf2x.KIND_CYCLIC, off, off, off)
    dA = torch.from_numpy(A.view(np.int64)).cuda()
    dB = torch.from_numpy(Bs.view(np.int64)).cuda()
    dC1 = torch.zeros(len(A), dtype=torch.int64, device="cuda")
    dC2 = torch.zeros(len(A), dtype=torch.int64, device="cuda")
    ms_sp = _plan_ms(ctx, items_sp, dC1, dA, dB, steps)
    ms_de = _plan_ms(ctx, items_de, dC2, dA, dB, steps)
    if not torch.equal(dC1, dC2):
        raise AssertionError("mixed workload: sparse-kind and dense results differ")
    return {"products": count, "ms_per_launch": round(ms_sp, 4), "products_per_s": round(count / (ms_sp * 1e-3), 1),
            "dense_path_ms_per_launch": round(ms_de, 4), "speedup_over_dense_path": round(ms_de / ms_sp, 3)}


def single_latency(ctx, n, calls, warmup, seed):
    """One product per call, each call synchronized: median device time (HIP
    events) and median host round trip, after `warmup` untimed calls."""
    import numpy as np
    import torch

    from paper_2201_10473_amd import gf2x, inputs

    W = gf2x.words(n)
    a = inputs.dense(n, seed, 0, 0)
    b = inputs.dense(n, seed, 0, 1)
    dA = torch.from_numpy(a.view(np.int64)).cuda()
    dB = torch.from_numpy(b.view(np.int64)).cuda()
    dC = torch.zeros(W, dtype=torch.int64, device="cuda")
    for _ in range(warmup):
        ctx.mul_cyclic(dC, dA, dB, n)
    torch.cuda.synchronize()
    dev, host = [], []
    for _ in range(calls):
        s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        t0 = time.perf_counter()
        s.record()
        ctx.mul_cyclic(dC, dA, dB, n)
        e.record()
        e.synchronize()
        host.append(time.perf_counter() - t0)
        dev.append(s.elapsed_time(e))
    items = gf2x.make_items(n, gf2x.KIND_CYCLIC, 0, 0, 0)
    dR = torch.zeros(W, dtype=torch.int64, device="cuda")
    ctx.mul_batched(items, dR, dA, dB)
    torch.cuda.synchronize()
    if not torch.equal(dC, dR):
        raise AssertionError("single product at n=%d differs from the batched path" % n)
    return {"n": n, "calls": calls, "median_device_us": round(1e3 * float(np.median(dev)), 2),
            "median_host_us": round(1e6 * float(np.median(host)), 2),
            "schedule": single_schedule(n)}


def direct_class(n):
    """The fastest direct class (one workgroup per product) of n: the third
    column of the packaged schedule table."""
    from paper_2201_10473_amd import gf2x

    w = (n + 31) // 32
    for line in open(gf2x.DEFAULT_TUNE_CACHE):
        f = line.split()
        if f and not line.startswith("#") and int(f[0]) == w and len(f) >= 3:
            return f[2]
    raise RuntimeError("no direct class for n=%d in the schedule table" % n)


def single_schedule(n):
    """The class a single product of n bits runs in: the fourth column of the
    packaged schedule table (the lowest single-product latency measured), else
    the direct class of the third column, else the batch class."""
    from paper_2201_10473_amd import gf2x

    w = (n + 31) // 32
    try:
        for line in open(gf2x.DEFAULT_TUNE_CACHE):
            f = line.split()
            if f and not line.startswith("#") and int(f[0]) == w and len(f) >= 2:
                return f[min(len(f), 4) - 1]
    except (OSError, ValueError):
        pass
    return None


def time_inverse(ctx, n, seed, batch=1024, reps=10):
    """gf2x_inv_cyclic_batched on odd-weight operands: median device time of
    one inverse and of a batch; two results checked by a * inv(a) = 1."""
    import numpy as np
    import torch

    from paper_2201_10473_amd import gf2x, inputs

    W = gf2x.words(n)
    A = inputs.dense_batch(n, batch, seed, 0)
    A[:, -1] &= inputs.top_mask(n)
    weight = np.count_nonzero(np.unpackbits(A.view(np.uint8), axis=1), axis=1)
    A[:, 0] ^= (weight % 2 == 0).astype(np.uint64)  # odd weight: invertible for this n
    out = {"n": n}
    for count in (1, batch):
        off = np.arange(count, dtype=np.uint64) * W
        items = gf2x.make_items(n, gf2x.KIND_CYCLIC, off, off, off)
        dA = torch.from_numpy(A[:count].ravel().view(np.int64)).cuda()
        dC = torch.zeros(count * W, dtype=torch.int64, device="cuda")
        for _ in range(3):
            ctx.inv_cyclic_batched(items, dC, dA)
        torch.cuda.synchronize()
        ts = []
        for _ in range(reps):
            s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            s.record()
            ctx.inv_cyclic_batched(items, dC, dA)
            e.record()
            e.synchronize()
            ts.append(s.elapsed_time(e))
        C = dC.cpu().numpy().view(np.uint64).reshape(count, W)
        unit = np.zeros(W, dtype=np.uint64)
        unit[0] = 1
        for i in {0, count - 1}:
            if not np.array_equal(single_product(ctx, A[i], C[i], n), unit):
                raise AssertionError("inverse %d at n=%d: a * inv(a) != 1" % (i, n))
        ms = float(np.median(ts))
        key = "single" if count == 1 else "batch_%d" % count
        out[key] = {"ms": round(ms, 4), "inverses_per_s": round(count / (ms * 1e-3), 1)}
    return out


def single_product(ctx, a, b, n):
    """a * b mod (X^n - 1) through gf2x_mul_cyclic (host words in and out)."""
    import numpy as np
    import torch

    W = (n + 63) // 64
    dA = torch.from_numpy(np.ascontiguousarray(a).view(np.int64)).cuda()
    dB = torch.from_numpy(np.ascontiguousarray(b).view(np.int64)).cuda()
    dC = torch.zeros(W, dtype=torch.int64, device="cuda")
    ctx.mul_cyclic(dC, dA, dB, n)
    torch.cuda.synchronize()
    return dC.cpu().numpy().view(np.uint64)


def check_sample(ctx, res, n, count, k=6):
    """Sanity checks of a timed batch (exactness against the oracle is what
    the tests establish): every item against the evaluation-at-1 invariant
    (the parity of a product is the product of the parities), and k items
    against the single-product entry point, which runs other classes and
    kernels.  Returns the results as host words."""
    import numpy as np

    W = (n + 63) // 64
    C = res["C"].cpu().numpy().view(np.uint64).reshape(count, W)
    A, B = res["A"], res["B"]
    par = lambda X: (np.bitwise_count(X).sum(axis=1) & 1)
    if not np.array_equal(par(C), par(A) & par(B)):
        raise AssertionError("parity invariant failed at n=%d" % n)
    for i in np.linspace(0, count - 1, k).astype(int):
        if not np.array_equal(C[i], single_product(ctx, A[i], B[i], n)):
            raise AssertionError("item %d differs from the single-product path at n=%d" % (i, n))
    return C


def cpu_model():
    """CPU model name of the host (from /proc/cpuinfo), or None."""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def cpu_baseline(n, seed, target_s=12.0):
    """Oracle throughput on the host over a bounded sample of the workload:
    all usable cores (a thread pool, at most 16 threads) and one thread pinned
    to one core."""
    from concurrent.futures import ThreadPoolExecutor

    import numpy as np

    import oracle
    from paper_2201_10473_amd import inputs

    oracle.load()
    cpus = sorted(os.sched_getaffinity(0))
    threads = max(1, min(16, len(cpus)))
    A = inputs.dense_batch(n, 1, seed, 0)
    B = inputs.dense_batch(n, 1, seed, 1)
    t0 = time.perf_counter()
    oracle.mul_cyclic_many(A, B, n)
    one = time.perf_counter() - t0
    per_thread = max(1, int(target_s / threads / max(one, 1e-4)))
    per_thread = min(per_thread, BATCH // threads if BATCH >= threads else 1)
    total = per_thread * threads
    A = inputs.dense_batch(n, total, seed, 0)
    B = inputs.dense_batch(n, total, seed, 1)

    def work(t):
        sl = slice(t * per_thread, (t + 1) * per_thread)
        return oracle.mul_cyclic_many(A[sl], B[sl], n)

    t0 = time.perf_counter()
    with ThreadPoolExecutor(max_workers=threads) as ex:
        portable = list(ex.map(work, range(threads)))
    wall = time.perf_counter() - t0
    # the fast mode (the CPU's carry-less multiply), reported on its own line:
    # the whole seeded batch, repeated for at least a second; the products the
    # portable run computed are checked against it
    fast = None
    Af = inputs.dense_batch(n, BATCH, seed, 0)
    Bf = inputs.dense_batch(n, BATCH, seed, 1)
    per_fast = (BATCH + threads - 1) // threads

    def work_fast(t):
        sl = slice(t * per_fast, min(BATCH, (t + 1) * per_fast))
        return oracle.mul_cyclic_many_pclmul(Af[sl], Bf[sl], n)

    reps = 0
    t0 = time.perf_counter()
    with ThreadPoolExecutor(max_workers=threads) as ex:
        while True:
            fast_res = list(ex.map(work_fast, range(threads)))
            reps += 1
            if any(r is None for r in fast_res) or time.perf_counter() - t0 >= 1.0:
                break
    wall_fast = time.perf_counter() - t0
    if all(r is not None for r in fast_res):
        if not np.array_equal(np.concatenate(fast_res)[:total], np.concatenate(portable)):
            raise AssertionError("the oracle's PCLMULQDQ mode differs from its portable mode")
        fast = {"value": round(reps * BATCH / wall_fast, 2), "unit": "products/s", "cores": threads,
                "kind": "oracle with the CPU's PCLMULQDQ for the 64x64 carry-less multiply (word schoolbook)",
                "sample": "the %d-product batch at n=%d, %d times; its first %d products equal the portable mode's"
                % (BATCH, n, reps, total)}
    # one thread pinned to one core, on a sample of about 3 s
    k1 = max(1, min(total, int(3.0 / max(one, 1e-4))))
    pinned = os.sched_getaffinity(0)
    try:
        os.sched_setaffinity(0, {cpus[0]})
        t0 = time.perf_counter()
        oracle.mul_cyclic_many(A[:k1], B[:k1], n)
        wall1 = time.perf_counter() - t0
    finally:
        os.sched_setaffinity(0, pinned)
    return {
        "value": round(total / wall, 2),
        "unit": "products/s",
        "cores": threads,
        "kind": "oracle",
        "sample": "%d ring products at n=%d (the first %d pairs of the seeded batch), %d threads x %d products"
        % (total, n, total, threads, per_thread),
        "single_core": {"value": round(k1 / wall1, 2), "unit": "products/s", "cores": 1,
                        "sample": "%d ring products at n=%d on one thread pinned to cpu %d" % (k1, n, cpus[0])},
        "fast_mode_pclmul": fast,
        "host_cpus_usable": len(cpus),
        "nproc": os.cpu_count(),
        "cpu_model": cpu_model(),
    }


def kernel_sources():
    """The files that define the batched kernels and their launch: the device
    headers, the kernel translation units and the launchers (not the host API,
    the server or the Toeplitz path), in name order."""
    csrc = os.path.join(ROOT, "paper_2201_10473_amd", "csrc")
    keep = ("gf2x_device.hpp", "gf2x_product.hpp", "gf2x_internal.hpp", "gf2x_launch.hpp", "gf2x_kern_direct.hpp",
            "gf2x_kernels.hip")
    return [os.path.join(csrc, f) for f in sorted(os.listdir(csrc)) if f in keep or f.startswith("gf2x_kern_")]


def traffic_from_profile(kernel_key):
    """HBM bytes per launch measured with rocprofv3 --pmc (FETCH_SIZE, WRITE_SIZE),
    if a summary for the current kernel sources is committed under profiles/."""
    import hashlib

    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    try:
        data = json.load(open(path))
    except Exception:
        return None
    h = hashlib.sha256()
    for path in kernel_sources():
        h.update(open(path, "rb").read())
    entry = data.get(kernel_key)
    if not entry or entry.get("sources_sha256") != h.hexdigest():
        return None
    return entry.get("bytes_per_launch")


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-one-per-launch", action="store_true")
    ap.add_argument("--only-n", type=int, default=0, help="time only this ring size (profiling runs)")
    ap.add_argument("--no-serving", action="store_true")
    ap.add_argument("--serving-requests", type=int, default=0,
                    help="requests per serving rate (default 100000)")
    ap.add_argument("--calibrate-copy-mib", type=int, default=0,
                    help="also run one device copy of this many MiB (calibrates HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU; multi-GPU runs are not part of this library's benchmark "
              "(independent products shard by item with no exchange).", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2201_10473_amd import gf2x, inputs

    if not torch.cuda.is_available():
        print("no GPU visible", file=sys.stderr)
        sys.exit(1)
    ctx = gf2x.Context(0)
    seed = inputs.SEED_BASE + 2
    if args.calibrate_copy_mib:
        nbytes = args.calibrate_copy_mib << 20
        src = torch.ones(nbytes // 8, dtype=torch.int64, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        log("calibration copy: %d bytes read, %d bytes written" % (nbytes, nbytes))
    sizes = [args.only_n] if args.only_n else [17669, 57637]
    results = {}
    for n in sizes:
        s, base, ops, name = ctx.schedule_info(n)
        log("batched n=%d schedule=%s ops/product=%d" % (n, name, ops))
        r = time_batched(ctx, n, BATCH, args.steps, args.warmup, seed)
        C_batched = check_sample(ctx, r, n, BATCH)
        res = {
            "schedule": name,
            "padded_words32": s,
            "lane_ops_per_product": ops,
            "launch_ms": r["launch_ms"],
            "products_per_s": BATCH * args.steps / r["wall_s"],
            "ms_per_step": 1e3 * r["wall_s"] / args.steps,
        }
        res["valu_frac"] = ops * BATCH / (res["launch_ms"] * 1e-3) / VALU_PEAK
        if not args.no_one_per_launch and not args.only_n:
            # one kernel launch per product: a context whose single-product
            # class is the direct class of n (one workgroup, one launch)
            direct = direct_class(n)
            with tempfile.NamedTemporaryFile("w", suffix=".txt", delete=False) as f:
                f.write("%d %s %s %s\n" % ((n + 31) // 32, name, direct, direct))
                table = f.name
            try:
                with gf2x.Context(0, tune_cache=table) as dctx:
                    log("one-per-launch n=%d (one %s launch per product)" % (n, direct))
                    o = time_one_per_launch(dctx, n, BATCH, seed)
            finally:
                os.unlink(table)
            # same seeded operands as the batched run: every result must match it
            if not np.array_equal(o["C"].cpu().numpy().view(np.uint64).reshape(BATCH, -1), C_batched):
                raise AssertionError("one-per-launch results differ from the batched launch at n=%d" % n)
            res["one_per_launch_class"] = direct
            res["one_per_launch_products_per_s"] = BATCH / o["wall_s"]
            res["batched_over_one_per_launch"] = res["products_per_s"] / res["one_per_launch_products_per_s"]
            log("one-per-launch n=%d through gf2x_mul_cyclic (lowest-latency class %s)" % (n, single_schedule(n)))
            o = time_one_per_launch(ctx, n, BATCH, seed)
            if not np.array_equal(o["C"].cpu().numpy().view(np.uint64).reshape(BATCH, -1), C_batched):
                raise AssertionError("single-product results differ from the batched launch at n=%d" % n)
            res["single_call_class"] = single_schedule(n)
            res["single_call_products_per_s"] = BATCH / o["wall_s"]
        results[n] = res
        log("n=%d: %.0f products/s, launch %.3f ms, VALU frac %.3f" % (n, res["products_per_s"], res["launch_ms"], res["valu_frac"]))

    shared = {}
    if not args.only_n:
        for n, count in ((35851, 1024), (57637, 512)):
            log("shared-operand n=%d x %d: packed vs Toeplitz int8 MFMA" % (n, count))
            ms_p, h, R, Cp = time_shared(ctx, n, count, gf2x.FORCE_PACKED, 10, seed + 1)
            ms_t, _, _, Ct = time_shared(ctx, n, count, gf2x.FORCE_TOEPLITZ, 10, seed + 1)
            # two independent device paths (bit-packed Karatsuba/Toom, int8 MFMA)
            if not np.array_equal(Cp, Ct):
                raise AssertionError("Toeplitz and packed paths disagree at n=%d" % n)
            macs = float(n) * n * count  # one int8 multiply-add per matrix entry
            shared[str(n)] = {
                "batch": count,
                "packed_products_per_s": round(count / (ms_p * 1e-3), 1),
                "toeplitz_products_per_s": round(count / (ms_t * 1e-3), 1),
                "toeplitz_over_packed": round(ms_p / ms_t, 4),
                "toeplitz_mfma_frac": round(2 * macs / (ms_t * 1e-3) / INT8_PEAK, 4),
            }
            log("  packed %.3f ms, toeplitz %.3f ms" % (ms_p, ms_t))

    mixed = None
    paper_method = None
    sparse = None
    mixed_sparse = None
    serving = []
    trace = None
    single = None
    inverse = None
    if not args.only_n:
        log("the paper's method (Appendix E): six ring sizes, 10 seeds x min over 20 replays of a 4096 batch")
        paper_method = time_paper_method(ctx)
        log("  %s" % {n: r["ms_per_batch"] for n, r in paper_method.items()})
        log("single product latency n=12323 (1000 calls after 100 warm-ups)")
        single = single_latency(ctx, 12323, 1000, 100, inputs.SEED_BASE + 1)
        log("  %s" % single)
        log("mixed workload: 8192 products, six sizes, half dense x sparse")
        mixed = time_mixed(ctx, 10, inputs.SEED_BASE + 4)
        log("  %s" % mixed)
        log("dense x sparse: constant-time rotation barrel vs the dense path, 4096 products per size")
        sparse = time_sparse(ctx, 10, inputs.SEED_BASE + 14)
        log("mixed workload with the sparse half as positions (sparse kind)")
        mixed_sparse = time_mixed_sparse(ctx, 10, inputs.SEED_BASE + 4)
        log("  %s" % mixed_sparse)
        log("inverses in F2[X]/(X^12323 - 1): one, and a batch of 1024")
        inverse = time_inverse(ctx, 12323, inputs.SEED_BASE + 9)
        log("  %s" % inverse)
        if not args.no_serving:
            from paper_2201_10473_amd import serve

            # the server gets a context of its own, as a serving process would
            with gf2x.Context(0) as sctx:
                runs = [(rate, 0) for rate in (10000, 30000, 100000, 300000, 500000)] + [(100000, 8 << 20)]
                for rate, budget in runs:
                    log("serving: Poisson %d req/s%s" % (rate, ", 8 MiB budget" if budget else ""))
                    count = args.serving_requests or 100000
                    res, bufs = serve.run(sctx, rate, count, inputs.SEED_BASE + 5, hbm_budget_bytes=budget)
                    serve.check_against_batched(sctx, *bufs)
                    res["hbm_budget_bytes"] = budget or 256 << 20
                    serving.append(res)
                    st = res["server"]
                    log("  achieved %.0f req/s p50 %.1f us p99 %.1f us; batches %d (%d phased), host per batch "
                        "pack %.1f issue %.1f retire %.1f us; max batch %.0f us, device %.0f us, loop %.0f us"
                        % (res["achieved_rate"], res["p50_us"], res["p99_us"], st["batches"], st["phased_batches"],
                           st["host_pack_ns"] / 1e3 / max(1, st["batches"]),
                           st["host_issue_ns"] / 1e3 / max(1, st["batches"]),
                           st["host_retire_ns"] / 1e3 / max(1, st["batches"]), st["batch_max_ns"] / 1e3,
                           st["device_max_ns"] / 1e3, st["loop_busy_max_ns"] / 1e3))
                    log("  longest issue %.0f us: copies in %.0f, launches %.0f, copy back and event %.0f us (maxima)"
                        % (st["host_issue_max_ns"] / 1e3, st["host_issue_copy_max_ns"] / 1e3,
                           st["host_issue_launch_max_ns"] / 1e3, st["host_issue_tail_max_ns"] / 1e3))
                from paper_2201_10473_amd import hqc_trace

                log("HQC-shaped trace: 5000 operations (chains of 1-3 dependent products), 20000 op/s")
                trace, tbufs = hqc_trace.run(sctx, 20000, 5000, inputs.SEED_BASE + 11)
                trace["checked_products"] = hqc_trace.check_against_batched(sctx, tbufs)
                log("  %s" % trace["per_kind"])

    head = sizes[0]
    main_res = results[head]
    achieved = main_res["lane_ops_per_product"] * BATCH / (main_res["launch_ms"] * 1e-3)
    roof = {
        "bound": "alu",
        "achieved": round(achieved / 1e12, 4),
        "peak": round(VALU_PEAK / 1e12, 4),
        "unit": "Tlane-op/s",
        "frac": round(achieved / VALU_PEAK, 4),
        "traffic": traffic_from_profile("batched_n%d" % head),
        "kernel": "gf2x::k_batched<%s>" % main_res["schedule"],
    }
    out = {
        "metric": METRIC,
        "value": round(main_res["products_per_s"], 1),
        "unit": "products/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(main_res["ms_per_step"], 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic",
        "config": {
            "workload": "%d independent dense x dense ring products in F2[X]/(X^%d - 1), uniform seeded "
            "operands of %d uint64 words, one persistent launch per step (plan replay)"
            % (BATCH, head, (head + 63) // 64),
            "n": head,
            "batch": BATCH,
            "schedule": main_res["schedule"],
        },
        "roofline": roof,
        "extra": dict(
            {str(n): {k: (round(v, 4) if isinstance(v, float) else v) for k, v in r.items()}
             for n, r in results.items()},
            shared_operand=shared,
            paper_method=paper_method,
            single_product=single,
            inverse=inverse,
            mixed=mixed,
            mixed_sparse_kind=mixed_sparse,
            sparse=sparse,
            serving=serving,
            hqc_trace=trace,
        ),
    }
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle) n=%d" % head)
        out["cpu_baseline"] = cpu_baseline(head, seed)
    print(json.dumps(out), flush=True)
    ctx.close()


if __name__ == "__main__":
    main()
