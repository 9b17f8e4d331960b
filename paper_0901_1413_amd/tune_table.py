"""Write a tuning table for the current device with the library's tuner (gfq_tune).

Batch mode: every (field, m class, l class) that products of sides 64..4096 fall in
(classes are powers of two; the tuner times each at the geometric middle of the class).
Plain mode: square products 512 .. 8192 and the rectangular 16384 x 2048 x 16384 shape, then
the Strassen-Winograd levels for square products of 4096, 8192 and 16384.
The table is text (one entry per line) and is loaded with gfq.tune_load.

    python -m paper_0901_1413_amd.tune_table [--out paper_0901_1413_amd/tuning/gfx950.txt]
"""
from __future__ import annotations

import argparse
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))


def mid(b: int) -> int:
    """Geometric middle of the size class (2^(b-1), 2^b]."""
    return max(1, int(round(2 ** (b - 0.5))))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=os.path.join(HERE, "tuning", "gfx950.txt"))
    ap.add_argument("--fields", default="3,4,5,7,8,9")
    ap.add_argument("--batch-classes", default="6,7,8,9,10,11,12", help="log2 classes of m and l for batch mode")
    ap.add_argument("--plain", action="store_true", help="also tune the plain single-product shapes")
    args = ap.parse_args()
    sys.path.insert(0, os.path.dirname(HERE))
    import torch

    from paper_0901_1413_amd import gfq

    torch.cuda.set_device(0)
    gfq.load()
    gfq.tune_clear()
    fields = [int(x) for x in args.fields.split(",")]
    classes = [int(x) for x in args.batch_classes.split(",")]
    t0 = time.time()
    for q in fields:
        for bm in classes:
            for bl in classes:
                c = gfq.tune(q, mid(bm), mid(bl), 512, batch=True)
                print(f"batch q={q} m~{mid(bm)} l~{mid(bl)}: {c}", flush=True)
    if args.plain:
        shapes = [(s, s, s) for s in (512, 1024, 2048, 4096, 8192)] + [(16384, 2048, 16384)]
        for q in fields:
            for (m, l, n) in shapes:
                c = gfq.tune(q, m, l, n)
                print(f"plain q={q} {m}x{l}x{n}: {c}", flush=True)
        # Strassen-Winograd levels for the large square classes (after the plain entries, which
        # the leaves' configurations come from)
        for q in fields:
            for s in (4096, 8192, 16384):
                lev = gfq.tune_sw(q, s, s, s)
                print(f"sw q={q} {s}^3: {lev} levels", flush=True)
    os.makedirs(os.path.dirname(args.out), exist_ok=True)
    gfq.tune_save(args.out)
    print(f"wrote {args.out} in {time.time() - t0:.1f} s", flush=True)


if __name__ == "__main__":
    main()
