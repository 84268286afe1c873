"""Measure the schedule table for the ring sizes on the local GPU and write it.

    python -m paper_2201_10473_amd.tune [--out FILE] [--batch 4096] [sizes...]

The timing loop runs inside the library (gf2x_tune); this script only picks
the sizes and the output file (default: the packaged tune_gfx950.txt).
"""
import argparse
import sys

from paper_2201_10473_amd import gf2x, inputs


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("sizes", nargs="*", type=int, default=list(inputs.RING_SIZES))
    ap.add_argument("--out", default=gf2x.DEFAULT_TUNE_CACHE)
    ap.add_argument("--batch", type=int, default=4096)
    args = ap.parse_args()
    with gf2x.Context(0, tune_cache=None) as ctx:
        for n in args.sizes:
            print("tuning n=%d (default %s)" % (n, ctx.schedule_info(n)[3]), flush=True)
            ctx.tune([n], batch=args.batch)
            print("  -> %s" % ctx.schedule_info(n)[3], flush=True)
        ctx.tune([], batch=args.batch, out_path=args.out)
    print("wrote", args.out)
    return 0


if __name__ == "__main__":
    sys.exit(main())
