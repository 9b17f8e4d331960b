"""Benchmark of the bitsliced Four-Russians product on one MI355X.

Workload: the plain single products over F_3 and F_5, A and B 8192 x 8192 with i.i.d.
uniform entries (seeded).  One step is the whole path for both products: pack A and B
(uint8 -> bit-planes), the Four-Russians product (and the partial-sum kernel when the
inner dimension is split), unpack C.  Inputs are resident in HBM before timing starts.

Printed: one JSON line with field-ops/s (2 m l n / t) for the whole step, the roofline of
the dominant kernel (the product kernel of the field that takes longest), and the CPU
oracle timed on a bounded row sample of the same products (its rows are also compared
bit-exactly with the GPU product).

    python bench.py [--gpus 1] [--steps K] [--warmup W]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

M = L = N = 8192
FIELDS = (3, 5)
PEAK_VALU_OPS = 256 * 64 * 2.4e9          # 32-bit VALU lane-operations per second
PEAK_HBM = 8.0e12

# Per-unit operation counts of the method on gfx950 (three-input bitwise instructions).
# A unit is (row of C, slab of k rows of B, 32-column word).  Accumulate: carry-save
# additions of the D alpha-scaled table rows (2 instructions per residue bit and addend).
# Table build: one field addition per table entry and word.  Finish: per output word.
C_ACC = {3: 8, 4: 3, 5: 24, 7: 18}
C_ADD = {3: 6, 4: 2, 5: 13, 7: 11}
C_FIN = {3: 8, 4: 0, 5: 30, 7: 15}
# The paper's two-input operation counts (Sections 4.1 and 4.2) for the same units.
C_ACC_PAPER = {3: 12, 4: 4, 5: 60, 7: 51}
C_ADD_PAPER = {3: 6, 4: 2, 5: 20, 7: 17}


# HBM traffic of the product kernels from rocprofv3 FETCH_SIZE / WRITE_SIZE passes on this
# workload, scaled by the same counters on a 1 GiB device copy (reads x 2.0, writes x 1.0);
# valid only while the kernel sources hash to `src` (otherwise the roofline reports null).
KERNEL_SOURCES = ("gfq_m4rm.hip", "gfq_device.h", "gfq_field.h", "gfq_internal.h")
MEASURED_TRAFFIC = {
    3: {"src": "928ca375c42b3e04", "read_mib": 643.1, "write_mib": 32.0},
    5: {"src": "928ca375c42b3e04", "read_mib": 248.2, "write_mib": 24.0},
}


def kernel_source_hash():
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_0901_1413_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def algorithmic_ops(q, m, l, n, k, acc, add, fin=None):
    S = -(-l // k)
    W = -(-n // 32)
    ops = S * W * (m * acc[q] + ((1 << k) - 1) * add[q])
    if fin:
        ops += m * W * fin[q]
    return ops


def percentile(xs, p):
    xs = sorted(xs)
    i = min(len(xs) - 1, max(0, int(round(p / 100.0 * (len(xs) - 1)))))
    return xs[i]


def cpu_baseline(torch, gfq, oracle, data, seconds=10.0):
    """Time the oracle on the first rows of A for each field (about `seconds` in total) and
    compare those rows with the GPU product."""
    import numpy as np
    per_field = seconds / len(FIELDS)
    total_ops, total_t, rows_done, match = 0.0, 0.0, {}, True
    for q in FIELDS:
        A, B, Cgpu = data[q]["A"], data[q]["B"], data[q]["C_host"]
        r0, t_used = 0, 0.0
        chunk = 32
        while t_used < per_field and r0 < M:
            r1 = min(M, r0 + chunk)
            t0 = time.perf_counter()
            Cs = oracle.matmul(q, A[r0:r1], B)
            dt = time.perf_counter() - t0
            t_used += dt
            total_ops += 2.0 * (r1 - r0) * L * N
            match = match and bool(np.array_equal(Cs, Cgpu[r0:r1]))
            r0 = r1
            chunk = min(1024, chunk * 2)
        total_t += t_used
        rows_done[q] = r0
    return {
        "value": total_ops / total_t,
        "unit": "field-ops/s",
        "cores": oracle.max_threads(),
        "kind": "oracle",
        "sample": ", ".join(f"F_{q}: rows 0..{rows_done[q] - 1} of A times all of B" for q in FIELDS)
                  + "; schoolbook i-t-j loop, int32 accumulation, OpenMP over rows",
        "sample_rows_match_gpu": match,
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--copy-mb", type=int, default=0,
                    help="first run one device-to-device copy of this many MiB (a kernel of known "
                         "traffic that calibrates hardware memory counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported: the library drives one "
              f"MI355X and reports that GPU's throughput", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_0901_1413_amd import gfq, inputs

    torch.cuda.set_device(0)
    dev = torch.device("cuda", 0)
    gfq.load()

    if args.copy_mb:
        src = torch.ones(args.copy_mb << 20, dtype=torch.uint8, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    data = {}
    for q in FIELDS:
        A, B = inputs.pair(q, M, L, N, cfg=2, idx=q)
        cfg = gfq.choose_config(q, M, L, N)
        data[q] = {
            "A": A, "B": B, "cfg": cfg,
            "Ad": torch.from_numpy(A).to(dev), "Bd": torch.from_numpy(B).to(dev),
            "Ap": gfq.empty_packed(q, M, L), "Bp": gfq.empty_packed(q, L, N), "Cp": gfq.empty_packed(q, M, N),
            "Cd": torch.empty((M, N), dtype=torch.uint8, device=dev),
        }
    torch.cuda.synchronize()

    def step(record=None):
        for q in FIELDS:
            d = data[q]
            e0 = torch.cuda.Event(enable_timing=True) if record is not None else None
            e1 = torch.cuda.Event(enable_timing=True) if record is not None else None
            if e0 is not None:
                e0.record()
            gfq.pack(q, d["Ad"], out=d["Ap"])
            gfq.pack(q, d["Bd"], out=d["Bp"])
            gfq.matmul(q, d["Ap"], d["Bp"], M, L, N, out=d["Cp"])
            gfq.unpack(q, d["Cp"], M, N, out=d["Cd"])
            if e1 is not None:
                e1.record()
                record.append((q, e0, e1))

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()

    # timed region: K steps, per-product events, library events around every kernel
    per_product = []
    kernel_ms = {q: [] for q in FIELDS}
    t_start = torch.cuda.Event(enable_timing=True)
    t_end = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t_start.record()
    for _ in range(args.steps):
        step(per_product)
    t_end.record()
    torch.cuda.synchronize()
    total_ms = t_start.elapsed_time(t_end)

    # product-kernel durations, measured in separate passes with library timing on
    gfq.set_timing(True)
    for q in FIELDS:
        d = data[q]
        gfq.timing_read()
        for _ in range(max(3, min(args.steps, 10))):
            gfq.matmul(q, d["Ap"], d["Bp"], M, L, N, out=d["Cp"])
        torch.cuda.synchronize()
        t = gfq.timing_read()
        kernel_ms[q] = {"product_ms": t["product_ms"] / t["product_launches"],
                        "reduce_ms": (t["reduce_ms"] / t["reduce_launches"]) if t["reduce_launches"] else 0.0}
    gfq.set_timing(False)

    ops_per_step = sum(2.0 * M * L * N for _ in FIELDS)
    ms_per_step = total_ms / args.steps
    value = ops_per_step / (ms_per_step * 1e-3)
    lat = {}
    for q in FIELDS:
        xs = [e0.elapsed_time(e1) for (qq, e0, e1) in per_product if qq == q]
        lat[f"F_{q}"] = {"p50_ms": round(percentile(xs, 50), 4), "p99_ms": round(percentile(xs, 99), 4)}

    rooflines = []
    src_hash = kernel_source_hash()
    for q in FIELDS:
        c = data[q]["cfg"]
        dur = kernel_ms[q]["product_ms"] * 1e-3
        ops = algorithmic_ops(q, M, L, N, c["k"], C_ACC, C_ADD)
        ops_paper = algorithmic_ops(q, M, L, N, c["k"], C_ACC_PAPER, C_ADD_PAPER)
        ach = ops / dur
        rooflines.append({
            "kernel": f"m4rm_kernel<F_{q}>", "bound": "alu",
            "achieved": round(ach / 1e12, 3), "peak": round(PEAK_VALU_OPS / 1e12, 3), "unit": "Tops/s",
            "frac": round(ach / PEAK_VALU_OPS, 4),
            "traffic": (round((MEASURED_TRAFFIC[q]["read_mib"] + MEASURED_TRAFFIC[q]["write_mib"]) * 2 ** 20)
                        if MEASURED_TRAFFIC.get(q, {}).get("src") == src_hash else None),
            "avg_ms": round(kernel_ms[q]["product_ms"], 4),
            "partial_sum_ms": round(kernel_ms[q]["reduce_ms"], 4),
            "paper_op_frac": round(ops_paper / dur / PEAK_VALU_OPS, 4),
            "config": c,
        })
    dominant = max(rooflines, key=lambda r: r["avg_ms"])

    out = {
        "metric": "GF(q) matmul field-ops/s (2mln/t) batched vs plain, 1 MI355X; p99 latency",
        "value": value,
        "unit": "field-ops/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic",
        "config": {"workload": "plain products F_3 and F_5, A and B 8192x8192, uniform entries; "
                               "step = pack A, pack B, Four-Russians product, unpack C for both fields",
                   "fields": list(FIELDS), "m": M, "l": L, "n": N,
                   "kernel_config": {f"F_{q}": data[q]["cfg"] for q in FIELDS}},
        "roofline": {k: dominant[k] for k in ("bound", "achieved", "peak", "unit", "frac", "traffic")},
        "roofline_kernels": rooflines,
        "latency_per_product": lat,
    }
    if not args.no_cpu:
        for q in FIELDS:
            data[q]["C_host"] = data[q]["Cd"].cpu().numpy()
        import oracle
        out["cpu_baseline"] = cpu_baseline(torch, gfq, oracle, data)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
