"""Constant-time check by hardware counters.

A product's control flow, loop bounds and memory addresses depend only on n,
so its kernels must execute exactly the same instructions whatever the
operand bits are.  `run` launches the same workload once per operand class
(all-zero, all-one, random, sparse) -- a 1024-item batch of ring products at
each ring size, single-product launches (a staged and a one-workgroup
class), device-resident descriptors, the fused launch, a batch of inverses,
a shared-operand Toeplitz batch, a batch of dense x sparse products whose
position sets are the classes (all at 0, all at n - 1, random, clustered),
and a batch through the serving loop (the phase kernels) -- and `analyze`
compares the instruction counters rocprofv3 recorded for those dispatches,
kernel by kernel; every counter must be equal across the four classes.

    rocprofv3 --pmc SQ_INSTS_VALU SQ_INSTS_SALU SQ_INSTS_LDS SQ_INSTS_VMEM_RD \\
        SQ_INSTS_VMEM_WR SQ_INSTS_SMEM SQ_INSTS_BRANCH SQ_INSTS_LDS_ATOMIC \\
        -d OUT -o ct --output-format csv -- python -m paper_2201_10473_amd.ct_check run
    python -m paper_2201_10473_amd.ct_check analyze OUT/ct_counter_collection.csv
"""
import argparse
import csv
import json
import sys

import numpy as np

CLASSES = ("zero", "ones", "random", "sparse")


def operands(kind, n, count, seed):
    from paper_2201_10473_amd import inputs

    W = (n + 63) // 64
    if kind == "zero":
        return np.zeros((count, W), dtype=np.uint64)
    if kind == "ones":
        x = np.full((count, W), 0xFFFFFFFFFFFFFFFF, dtype=np.uint64)
        x[:, -1] &= inputs.top_mask(n)
        return x
    if kind == "random":
        return inputs.dense_batch(n, count, seed, 0)
    return np.stack([inputs.sparse(n, inputs.sparse_weight_for(n), seed, i) for i in range(count)])


# A product of n = 1 runs the one-word class, which no workload here uses:
# its dispatch marks the start of each run in the counter trace.
MARKER = "ParK2<0, 4>"


def run(count=1024, seed=7):
    import torch

    from paper_2201_10473_amd import gf2x, inputs

    order = []
    with gf2x.Context(0) as ctx:
        dM = torch.zeros(4, dtype=torch.int64, device="cuda")
        # the server of the last workload is created before the first marker:
        # its set-up launches (page warm-up) belong to no run
        srv = gf2x.Server(ctx, streams=1)

        def mark():
            torch.cuda.synchronize()
            ctx.mul_cyclic(dM[2:], dM[:1], dM[1:2], 1)
            torch.cuda.synchronize()

        for n in inputs.RING_SIZES:
            W = (n + 63) // 64
            items = gf2x.make_items(n, gf2x.KIND_CYCLIC, np.arange(count) * W, np.arange(count) * W,
                                    np.arange(count) * W)
            dC = torch.zeros(count * W, dtype=torch.int64, device="cuda")
            for kind in CLASSES:
                mark()
                A = operands(kind, n, count, seed)
                B = operands(kind, n, count, seed + 1)
                dA = torch.from_numpy(A.ravel().view(np.int64)).cuda()
                dB = torch.from_numpy(B.ravel().view(np.int64)).cuda()
                torch.cuda.synchronize()
                ctx.mul_batched(items, dC, dA, dB)
                torch.cuda.synchronize()
                order.append(("batched", n, kind))
        n = 17669
        W = (n + 63) // 64
        dC = torch.zeros(W, dtype=torch.int64, device="cuda")
        for kind in CLASSES:
            mark()
            A = operands(kind, n, 1, seed)
            dA = torch.from_numpy(A.ravel().view(np.int64)).cuda()
            torch.cuda.synchronize()
            ctx.mul_cyclic(dC, dA, dA, n)
            torch.cuda.synchronize()
            order.append(("single", n, kind))
        n = 12323  # one workgroup (k_single)
        W = (n + 63) // 64
        dC = torch.zeros(W, dtype=torch.int64, device="cuda")
        for kind in CLASSES:
            mark()
            A = operands(kind, n, 1, seed)
            dA = torch.from_numpy(A.ravel().view(np.int64)).cuda()
            torch.cuda.synchronize()
            ctx.mul_cyclic(dC, dA, dA, n)
            torch.cuda.synchronize()
            order.append(("single", n, kind))
        # device-resident descriptors (k_mixed), then the fused launch, over
        # 16 items of each ring size
        ns = np.repeat(np.asarray(inputs.RING_SIZES, dtype=np.uint32), 16)
        Ws = (ns.astype(np.uint64) + 63) // 64
        offs = np.concatenate([[0], np.cumsum(Ws)[:-1]]).astype(np.uint64)
        items = gf2x.make_items(ns, gf2x.KIND_CYCLIC, offs, offs, offs)
        d_items = torch.from_numpy(items.view(np.uint8).copy()).cuda()
        dC = torch.zeros(int(Ws.sum()), dtype=torch.int64, device="cuda")
        for flags, name in ((gf2x.ITEMS_ON_DEVICE, "device items"), (gf2x.FUSED, "fused")):
            for kind in CLASSES:
                mark()
                A = np.concatenate([operands(kind, int(n), 1, seed + i)[0] for i, n in enumerate(ns)])
                dA = torch.from_numpy(A.view(np.int64)).cuda()
                torch.cuda.synchronize()
                if flags == gf2x.ITEMS_ON_DEVICE:
                    ctx.mul_batched(d_items, dC, dA, dA, flags, count=len(ns))
                else:
                    ctx.mul_batched(items, dC, dA, dA, flags)
                torch.cuda.synchronize()
                order.append((name, 0, kind))
        # inverses (Itoh-Tsujii: permutation launches and batched products)
        n, count = 12323, 16
        W = (n + 63) // 64
        off = np.arange(count, dtype=np.uint64) * W
        items = gf2x.make_items(n, gf2x.KIND_CYCLIC, off, off, off)
        dC = torch.zeros(count * W, dtype=torch.int64, device="cuda")
        for kind in CLASSES:
            mark()
            A = operands(kind, n, count, seed)
            dA = torch.from_numpy(A.ravel().view(np.int64)).cuda()
            torch.cuda.synchronize()
            ctx.inv_cyclic_batched(items, dC, dA)
            torch.cuda.synchronize()
            order.append(("inverse", n, kind))
        # dense x sparse: the secret is the position set
        for n, count in ((17669, 64), (57637, 1024)):
            w = inputs.sparse_weight_for(n)
            W = (n + 63) // 64
            A = inputs.dense_batch(n, count, seed, 0)
            dA = torch.from_numpy(A.ravel().view(np.int64)).cuda()
            dC = torch.zeros(count * W, dtype=torch.int64, device="cuda")
            per = (w + 1) // 2
            items = gf2x.make_items(n, gf2x.sparse_kind(w), np.arange(count) * W, np.arange(count) * per,
                                    np.arange(count) * W)
            for kind in CLASSES:
                mark()
                P = np.zeros((count, 2 * per), dtype=np.uint32)
                for i in range(count):
                    if kind == "zero":
                        P[i, :w] = 0
                    elif kind == "ones":
                        P[i, :w] = n - 1
                    elif kind == "random":
                        P[i, :w] = inputs.sparse_positions(n, w, seed, i)
                    else:  # clustered: w consecutive positions
                        P[i, :w] = (np.arange(w) + 17 * i) % n
                dP = torch.from_numpy(P.view(np.int64).ravel().copy()).cuda()
                torch.cuda.synchronize()
                ctx.mul_batched(items, dC, dA, dP)
                torch.cuda.synchronize()
                order.append(("sparse", n, kind))
        n, count = 35851, 256
        W = (n + 63) // 64
        items = gf2x.make_items(n, gf2x.KIND_CYCLIC, 0, np.arange(count) * W, np.arange(count) * W)
        dC = torch.zeros(count * W, dtype=torch.int64, device="cuda")
        for kind in CLASSES:
            mark()
            h = operands(kind, n, 1, seed)
            R = operands(kind, n, count, seed + 1)
            dH = torch.from_numpy(h.ravel().view(np.int64)).cuda()
            dR = torch.from_numpy(R.ravel().view(np.int64)).cuda()
            torch.cuda.synchronize()
            ctx.mul_batched(items, dC, dH, dR, gf2x.SHARED_A | gf2x.FORCE_TOEPLITZ)
            torch.cuda.synchronize()
            order.append(("toeplitz", n, kind))
        # the serving loop: 4 requests of each ring size, submitted together,
        # run as one batch of three phase kernels
        ns = np.repeat(np.asarray(inputs.RING_SIZES, dtype=np.uint32), 4)
        Ws = (ns.astype(np.uint64) + 63) // 64
        offs = np.concatenate([[0], np.cumsum(Ws)[:-1]]).astype(np.uint64)
        C = np.zeros(int(Ws.sum()), dtype=np.uint64)
        with srv:
            for kind in CLASSES:
                mark()
                A = np.concatenate([operands(kind, int(n), 1, seed + i)[0] for i, n in enumerate(ns)])
                torch.cuda.synchronize()
                srv.submit(ns, A, offs, A, offs, C, offs)
                srv.drain()
                order.append(("serving", 0, kind))
            st = srv.stats()
        if st["batches"] != len(CLASSES):
            print("serving batches split: %d" % st["batches"], file=sys.stderr)
    print(json.dumps(order))


def analyze(path):
    rows = [r for r in csv.DictReader(open(path)) if "gf2x" in r["Kernel_Name"] and "prepare" not in r["Kernel_Name"]
            and "fill" not in r["Kernel_Name"]]
    by_dispatch = {}
    for r in rows:
        d = int(r["Dispatch_Id"])
        by_dispatch.setdefault(d, {"kernel": r["Kernel_Name"].split("(")[0]})[r["Counter_Name"]] = float(
            r["Counter_Value"])
    # runs: the dispatches after each marker, up to the next one; every
    # workload is four consecutive runs (zero, ones, random, sparse) that must
    # launch the same kernels with the same counts
    runs = []
    for d in sorted(by_dispatch):
        x = by_dispatch[d]
        if MARKER in x["kernel"]:
            runs.append([])
        elif runs:
            runs[-1].append(x)
    if len(runs) % 4:
        print("unexpected number of runs: %d" % len(runs))
        return 1
    ok = True
    counters = sorted(k for k in runs[0][0] if k != "kernel")
    print("| workload kernel | counter | zero | ones | random | sparse | equal |")
    print("|---|---|---|---|---|---|---|")
    rows_out = 0
    for g in range(0, len(runs), 4):
        grp = runs[g:g + 4]
        if len(set(len(r) for r in grp)) != 1 or any(
                [x["kernel"] for x in r] != [x["kernel"] for x in grp[0]] for r in grp):
            print("| workload %d | kernel sequence differs between classes | | | | | NO |" % (g // 4))
            ok = False
            continue
        # one row per kernel and counter: the sum over the run's dispatches of that kernel
        kernels = []
        for x in grp[0]:
            if x["kernel"] not in kernels:
                kernels.append(x["kernel"])
        for kern in kernels:
            for c in counters:
                vals = [sum(x.get(c, 0.0) for x in r if x["kernel"] == kern) for r in grp]
                eq = len(set(vals)) == 1
                ok &= eq
                rows_out += 1
                print("| %s | %s | %s | %s | %s | %s | %s |" % (kern.replace("void ", "")[:60], c,
                                                               *["%.0f" % v for v in vals], "yes" if eq else "NO"))
    print("%d rows, %d workloads: %s" % (rows_out, len(runs) // 4, "ALL EQUAL" if ok else "MISMATCH"))
    return 0 if ok else 1


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("mode", choices=("run", "analyze"))
    ap.add_argument("path", nargs="?")
    args = ap.parse_args()
    if args.mode == "run":
        run()
        return 0
    return analyze(args.path)


if __name__ == "__main__":
    sys.exit(main())
