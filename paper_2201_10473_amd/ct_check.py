"""Constant-time check by hardware counters.

A product's control flow, loop bounds and memory addresses depend only on n,
so its kernels must execute exactly the same instructions whatever the
operand bits are.  `run` launches the same workload once per operand class
(all-zero, all-one, random, sparse) -- a 1024-item batch of ring products at
each ring size, one single-product launch, and one shared-operand Toeplitz
batch -- and `analyze` compares the instruction counters rocprofv3 recorded for
those dispatches, kernel by kernel; every counter must be equal across the
four classes.

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


def run(count=1024, seed=7):
    import torch

    from paper_2201_10473_amd import gf2x, inputs

    order = []
    with gf2x.Context(0) as ctx:
        for n in inputs.RING_SIZES:
            W = (n + 63) // 64
            items = gf2x.make_items(n, gf2x.KIND_CYCLIC, np.arange(count) * W, np.arange(count) * W,
                                    np.arange(count) * W)
            dC = torch.zeros(count * W, dtype=torch.int64, device="cuda")
            for kind in CLASSES:
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
            A = operands(kind, n, 1, seed)
            dA = torch.from_numpy(A.ravel().view(np.int64)).cuda()
            torch.cuda.synchronize()
            ctx.mul_cyclic(dC, dA, dA, n)
            torch.cuda.synchronize()
            order.append(("single", n, kind))
        n, count = 35851, 256
        W = (n + 63) // 64
        items = gf2x.make_items(n, gf2x.KIND_CYCLIC, 0, np.arange(count) * W, np.arange(count) * W)
        dC = torch.zeros(count * W, dtype=torch.int64, device="cuda")
        for kind in CLASSES:
            h = operands(kind, n, 1, seed)
            R = operands(kind, n, count, seed + 1)
            dH = torch.from_numpy(h.ravel().view(np.int64)).cuda()
            dR = torch.from_numpy(R.ravel().view(np.int64)).cuda()
            torch.cuda.synchronize()
            ctx.mul_batched(items, dC, dH, dR, gf2x.SHARED_A | gf2x.FORCE_TOEPLITZ)
            torch.cuda.synchronize()
            order.append(("toeplitz", n, kind))
    print(json.dumps(order))


def analyze(path):
    rows = [r for r in csv.DictReader(open(path)) if "gf2x" in r["Kernel_Name"] and "prepare" not in r["Kernel_Name"]
            and "convert" not in r["Kernel_Name"] and "fill" not in r["Kernel_Name"]]
    by_dispatch = {}
    for r in rows:
        d = int(r["Dispatch_Id"])
        by_dispatch.setdefault(d, {"kernel": r["Kernel_Name"].split("(")[0]})[r["Counter_Name"]] = float(
            r["Counter_Value"])
    # A workload may launch several kernels (the staged classes launch four),
    # so the dispatches are grouped per kernel: each launch of a workload runs
    # every one of its kernels once, in the order zero, ones, random, sparse.
    per_kernel = {}
    for d in sorted(by_dispatch):
        per_kernel.setdefault(by_dispatch[d]["kernel"], []).append(by_dispatch[d])
    for kern, lst in per_kernel.items():
        if len(lst) % 4:
            print("unexpected dispatch count %d for %s" % (len(lst), kern))
            return 1
    ok = True
    counters = sorted(k for k in next(iter(per_kernel.values()))[0] if k != "kernel")
    print("| workload kernel | counter | zero | ones | random | sparse | equal |")
    print("|---|---|---|---|---|---|---|")
    for kern, lst in per_kernel.items():
        for g in range(0, len(lst), 4):
            grp = lst[g:g + 4]
            name = kern.replace("void ", "")
            for c in counters:
                vals = [x.get(c) for x in grp]
                eq = len(set(vals)) == 1
                ok &= eq
                print("| %s | %s | %s | %s | %s | %s | %s |" % (name[:60], c, *["%.0f" % v for v in vals],
                                                               "yes" if eq else "NO"))
    print("ALL EQUAL" if ok else "MISMATCH")
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
