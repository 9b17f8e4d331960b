"""Benchmark of the bitsliced Four-Russians product on one MI355X.

Headline workload (the `value`): the plain single products over F_3 and F_5, A and B
8192 x 8192 with i.i.d. uniform entries (seeded).  One step is the whole path for both
products: pack A and B (uint8 -> bit-planes), the Four-Russians product (and the
partial-sum kernel when the inner dimension is split), unpack C.  Inputs are resident in
HBM before timing starts.

Printed: one JSON line with field-ops/s (2 m l n / t) for the whole step, the roofline of
the dominant kernel (the product kernel of the field that takes longest) and of the F_3
product, the machine rates the rooflines are quoted against (derived from the unit counts
and clock, and microbenchmarked in the run: v_bitop3_b32 lane operations, 128-bit LDS
reads, HBM copy), the CPU oracle timed on a bounded row sample of the same products on all
host threads and on one (its rows are also compared bit-exactly with the GPU product), and
sections for the other workloads:
  c1       F_3 512^3: per-product latency p50/p99 and the oracle's time for the product
  c2_k     the 8192^3 products with the slab width k swept 4..10 (each bit-exact)
  mfma     comparison only: the same 8192^3 products as exact int8 matrix-core GEMMs
           (torch._int_mm, int32 accumulation) reduced mod p, checked against this path
  c3       F_7 and GF(4), A 16384 x 2048 times B 2048 x 16384, dense and 10% density
  ext      GF(8) and F_9 products (row-wise and matrix-level routes)
  sw       Strassen-Winograd levels over the product
  c4       4096 products of mixed fields and log-uniform shapes: one batched launch
           (captured in a HIP graph) against one plain launch per product; every product
           against the oracle
  c5       served requests with Poisson arrivals: continuous batching against serial
           plain launches over the same trace, latency p50/p99 and throughput; every
           request with n <= 1024 and 2% of the others against the oracle, Freivalds' check
           on all

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--only c1,c5] [--c5-requests N]
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
# 32-bit VALU lane operations per second: 256 CUs x 128 lanes per clock x 2.4 GHz, the rate
# behind the published fp32 vector peak (157.3 TFLOP/s = 78.6e12 lane FMAs); the v_bitop3_b32
# microbenchmark issues 1.62 wave64 instructions per CU and clock, so one per clock (64
# lanes) would understate it
PEAK_VALU_OPS = 256 * 128 * 2.4e9
PEAK_LDS = 256 * 256 * 2.4e9              # LDS bytes per second: 64 banks x 4 B per clock per CU
PEAK_HBM = 8.0e12
SECTIONS = ("c1", "c2_k", "mfma", "c3", "ext", "sw", "c4", "c4_slices", "c5")

# Per-unit operation counts of the method on gfx950 (three-input bitwise instructions).
# A unit is (row of C, slab of k rows of B, 32-column word).  Accumulate: the slab's D
# alpha-scaled table rows into a carry-save accumulator, one full adder (2 instructions)
# per addend bit (F_3 4 bits, F_7 9; F_5 9 bits plus one half adder; GF(4) 3 XORs; GF(8)
# 6 XORs; F_9 8 bits).  Table build: one field addition per table entry and word.  Finish:
# per output word.
C_ACC = {3: 8, 4: 3, 5: 20, 7: 18, 8: 6, 9: 32}
C_ADD = {3: 4, 4: 2, 5: 8, 7: 11, 8: 3, 9: 8}
# The paper's two-input operation counts (Sections 4.1 and 4.2) for the same units.
C_ACC_PAPER = {3: 12, 4: 4, 5: 60, 7: 51}
C_ADD_PAPER = {3: 6, 4: 2, 5: 20, 7: 17}
# LDS words per unit: the slab's gathers read D table rows of GP planes per row of C and
# word; the table holds PT planes per entry.  Row-wise routes (variant 0) and the
# matrix-level routes of GF(4), GF(8), F_9 (variant 1).
LDS_GEOM = {(3, 0): (2, 2, 2), (4, 0): (2, 2, 2), (5, 0): (3, 3, 3), (7, 0): (3, 3, 3), (8, 0): (3, 3, 3),
            (9, 0): (4, 4, 4), (4, 1): (3, 1, 3), (8, 1): (6, 1, 6), (9, 1): (6, 2, 6)}


# HBM traffic of the product kernels from rocprofv3 FETCH_SIZE / WRITE_SIZE passes on this
# workload, scaled by the same counters on a 1 GiB device copy (reads x 2.0, writes x 1.0);
# valid only while the kernel sources hash to `src` (otherwise the roofline reports null).
KERNEL_SOURCES = ("gfq_m4rm_launch.h", "gfq_m4rm_tile.h", "gfq_device.h", "gfq_field.h", "gfq_internal.h")
MEASURED_TRAFFIC = {
    3: {"src": "f52dc466b8f6a7bd", "read_mib": 54.3, "write_mib": 64.0},
    5: {"src": "f52dc466b8f6a7bd", "read_mib": 129.3, "write_mib": 96.0},
}


def kernel_source_hash():
    """Hash of the product kernels' code (comments and whitespace removed, so that only a
    change of code invalidates the measured traffic)."""
    import hashlib
    import re
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_0901_1413_amd", "csrc", f), encoding="utf-8") as fh:
            text = fh.read()
        text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
        text = re.sub(r"//[^\n]*", " ", text)
        h.update(" ".join(text.split()).encode())
    return h.hexdigest()[:16]


def algorithmic_ops(q, m, l, n, k, acc, add, fin=None):
    S = -(-l // k)
    W = -(-n // 32)
    ops = S * W * (m * acc[q] + ((1 << k) - 1) * add[q])
    if fin:
        ops += m * W * fin[q]
    return ops


def algorithmic_lds_bytes(q, m, l, n, k, variant=0):
    """LDS bytes the method moves: every row's gathers for every slab and word, plus every
    table entry written once per slab and column strip."""
    D, GP, PT = LDS_GEOM[(q, variant)]
    S = -(-l // k)
    W = -(-n // 32)
    return 4.0 * S * W * (m * D * GP + (1 << k) * PT)


def rooflines(q, m, l, n, cfg, product_ms, peaks=None):
    """VALU and LDS fractions of one product launch: algorithmic work over the launch's time,
    against the derived peaks (VALU: 256 CUs x 128 lanes x 2.4 GHz; LDS: 256 B per clock per
    CU) and, where measured in this run, the microbenchmarked ones."""
    dur = product_ms * 1e-3
    variant = cfg.get("variant", 0)
    ops = algorithmic_ops(q, m, l, n, cfg["k"], C_ACC, C_ADD) if variant == 0 else None
    lds = algorithmic_lds_bytes(q, m, l, n, cfg["k"], variant)
    r = {"lds_TBps": round(lds / dur / 1e12, 3), "lds_frac_of_spec": round(lds / dur / PEAK_LDS, 4)}
    if ops is not None:
        r["alu_frac"] = round(ops / dur / PEAK_VALU_OPS, 4)
    if peaks:
        if ops is not None:
            r["alu_frac_of_measured"] = round(ops / dur / peaks["valu_lane_ops_per_s"], 4)
        r["lds_frac_of_measured"] = round(lds / dur / peaks["lds_bytes_per_s"], 4)
    return r


def rooflines_extra(q, m, l, n, cfg, product_ms, ctx):
    r = rooflines(q, m, l, n, cfg, product_ms, getattr(ctx, "peaks", None))
    r.pop("alu_frac", None)                     # the entry's frac
    return r


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def section_peaks(ctx, reps=3):
    """Microbenchmarked machine rates (gfq_probe_*): best of reps runs each."""
    gfq = ctx.gfq
    best = {}
    for kind, kw in (("valu", {"blocks": 2048, "iters": 4096}), ("lds", {"blocks": 2048, "iters": 256}),
                     ("copy", {"nbytes": 1 << 30})):
        gfq.probe(kind, **kw)                       # warm-up
        best[kind] = max(gfq.probe(kind, **kw)["rate"] for _ in range(reps))
    clk_cu = 2.4e9 * 256
    return {"valu_lane_ops_per_s": best["valu"], "valu_frac_of_derived": round(best["valu"] / PEAK_VALU_OPS, 4),
            "lds_bytes_per_s": best["lds"], "lds_bytes_per_clk_per_cu": round(best["lds"] / clk_cu, 1),
            "hbm_copy_bytes_per_s": best["copy"], "hbm_frac_of_8TBps": round(best["copy"] / PEAK_HBM, 4),
            "derived": {"valu_lane_ops_per_s": PEAK_VALU_OPS, "lds_bytes_per_s": PEAK_LDS, "hbm_bytes_per_s": PEAK_HBM},
            "probes": "v_bitop3_b32 in 17 independent chains per lane; 128-bit LDS reads, each 16-lane group one "
                      "256-byte row (the gathers' shape); 128-bit device copy of 1 GiB (reads + writes)"}


def percentile(xs, p):
    xs = sorted(xs)
    if not xs:
        return None
    i = min(len(xs) - 1, max(0, int(round(p / 100.0 * (len(xs) - 1)))))
    return xs[i]


def warm(torch, fn, seconds=0.25):
    """Run fn for `seconds` of wall time before a timed block: after host work (input
    generation, oracle checks) the GPU idles and its clock must ramp up again."""
    t0 = time.perf_counter()
    while time.perf_counter() - t0 < seconds:
        for _ in range(4):
            fn()
        torch.cuda.synchronize()


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


class Ctx:
    def __init__(self, torch, gfq, inputs, oracle_mod):
        self.torch, self.gfq, self.inputs, self.oracle = torch, gfq, inputs, oracle_mod
        self.dev = torch.device("cuda", 0)

    def up(self, x):
        import numpy as np
        return self.torch.from_numpy(np.ascontiguousarray(x)).to(self.dev)

    def events(self, n):
        return [self.torch.cuda.Event(enable_timing=True) for _ in range(n)]


def cpu_baseline(ctx, data, seconds=10.0, single_thread_seconds=2.0):
    """Time the oracle on the first rows of A for each field (about `seconds` in total, all
    host threads) and compare those rows with the GPU product; then on one thread, on the
    last rows (about `single_thread_seconds`)."""
    import numpy as np
    oracle = ctx.oracle
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
    # one thread: blocks of 8 rows from the end of A
    one_ops, one_t, one_rows = 0.0, 0.0, {}
    for q in FIELDS:
        A, B, Cgpu = data[q]["A"], data[q]["B"], data[q]["C_host"]
        r1, t_used = M, 0.0
        while t_used < single_thread_seconds / len(FIELDS) and r1 > 0:
            r0 = max(0, r1 - 8)
            t0 = time.perf_counter()
            Cs = oracle.matmul(q, A[r0:r1], B, threads=1)
            t_used += time.perf_counter() - t0
            one_ops += 2.0 * (r1 - r0) * L * N
            match = match and bool(np.array_equal(Cs, Cgpu[r0:r1]))
            r1 = r0
        one_t += t_used
        one_rows[q] = M - r1
    return {
        "value": total_ops / total_t,
        "unit": "field-ops/s",
        "cores": oracle.max_threads(),
        "kind": "oracle",
        "sample": ", ".join(f"F_{q}: rows 0..{rows_done[q] - 1} of A times all of B" for q in FIELDS)
                  + "; schoolbook i-t-j loop, int32 accumulation, OpenMP over rows",
        "cpu_model": cpu_model(),
        "single_thread": {"value": one_ops / one_t, "unit": "field-ops/s", "threads": 1,
                          "sample": ", ".join(f"F_{q}: the last {one_rows[q]} rows of A times all of B"
                                              for q in FIELDS)},
        "sample_rows_match_gpu": match,
    }


# ------------------------------------------------------------------------------------
# headline: F_3 and F_5 8192^3, whole path
# ------------------------------------------------------------------------------------

def headline(ctx, args):
    torch, gfq, inputs = ctx.torch, ctx.gfq, ctx.inputs
    data = {}
    for q in FIELDS:
        A, B = inputs.pair(q, M, L, N, cfg=2, idx=q)
        cfg = gfq.choose_config(q, M, L, N)
        data[q] = {
            "A": A, "B": B, "cfg": cfg,
            "Ad": ctx.up(A), "Bd": ctx.up(B),
            "Ap": gfq.empty_packed(q, M, L), "Bp": gfq.empty_packed(q, L, N), "Cp": gfq.empty_packed(q, M, N),
            "Cd": torch.empty((M, N), dtype=torch.uint8, device=ctx.dev),
        }
    torch.cuda.synchronize()

    def step(record=None):
        for q in FIELDS:
            d = data[q]
            e0, e1 = ctx.events(2) if record is not None else (None, None)
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

    per_product = []
    t_start, t_end = ctx.events(2)
    torch.cuda.synchronize()
    t_start.record()
    for _ in range(args.steps):
        step(per_product)
    t_end.record()
    torch.cuda.synchronize()
    total_ms = t_start.elapsed_time(t_end)

    # product-kernel durations, measured in separate passes with library timing on
    kernel_ms = {}
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

    ms_per_step = total_ms / args.steps
    value = sum(2.0 * M * L * N for _ in FIELDS) / (ms_per_step * 1e-3)
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
        tr = MEASURED_TRAFFIC.get(q, {})
        rooflines.append({
            "kernel": f"m4rm_kernel<F_{q}>", "bound": "alu",
            "achieved": round(ach / 1e12, 3), "peak": round(PEAK_VALU_OPS / 1e12, 3), "unit": "Tops/s",
            "frac": round(ach / PEAK_VALU_OPS, 4),
            "traffic": (round((tr["read_mib"] + tr["write_mib"]) * 2 ** 20) if tr.get("src") == src_hash else None),
            "algorithmic_hbm_bytes": (M * L + L * N + M * N) * {3: 2, 5: 3}[q] // 8,
            "avg_ms": round(kernel_ms[q]["product_ms"], 4),
            "partial_sum_ms": round(kernel_ms[q]["reduce_ms"], 4),
            # the paper's two-input operation count over the same time, per issued lane
            # instruction of the peak: one three-input instruction does up to two of them, so
            # this ratio is no roofline fraction and may exceed 1
            "paper_two_input_ops_per_peak_instruction": round(ops_paper / dur / PEAK_VALU_OPS, 4),
            **rooflines_extra(q, M, L, N, c, kernel_ms[q]["product_ms"], ctx),
            "config": c,
        })
    dominant = max(rooflines, key=lambda r: r["avg_ms"])
    f3 = next(r for r in rooflines if r["kernel"] == "m4rm_kernel<F_3>")
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
        "roofline_F_3": {k: f3[k] for k in ("bound", "achieved", "peak", "unit", "frac", "traffic")},
        "roofline_kernels": rooflines,
        "latency_per_product": lat,
    }
    return out, data


# ------------------------------------------------------------------------------------
# c1: F_3 512^3
# ------------------------------------------------------------------------------------

def section_c1(ctx, reps=200):
    import numpy as np
    torch, gfq, inputs = ctx.torch, ctx.gfq, ctx.inputs
    n = 512
    A, B = inputs.pair(3, n, n, n, cfg=1, idx=0)
    Ad, Bd = ctx.up(A), ctx.up(B)
    Ap, Bp, Cp = gfq.empty_packed(3, n, n), gfq.empty_packed(3, n, n), gfq.empty_packed(3, n, n)
    Cd = torch.empty((n, n), dtype=torch.uint8, device=ctx.dev)

    def path():
        gfq.pack(3, Ad, out=Ap)
        gfq.pack(3, Bd, out=Bp)
        gfq.matmul(3, Ap, Bp, n, n, n, out=Cp)
        gfq.unpack(3, Cp, n, n, out=Cd)

    for _ in range(10):
        path()
    torch.cuda.synchronize()
    # the same path captured once into a HIP graph (one graph launch instead of five kernel
    # launches); a first eager pass on the capture stream creates that stream's workspace
    graph = torch.cuda.CUDAGraph()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        path()
        side.synchronize()
        with torch.cuda.graph(graph, stream=side):
            path()
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    res = {}
    for name, fn in (("path", path), ("path_graph", graph.replay),
                     ("product", lambda: gfq.matmul(3, Ap, Bp, n, n, n, out=Cp))):
        ev = ctx.events(2 * reps)
        for i in range(reps):
            ev[2 * i].record()
            fn()
            ev[2 * i + 1].record()
        torch.cuda.synchronize()
        xs = [ev[2 * i].elapsed_time(ev[2 * i + 1]) for i in range(reps)]
        res[name] = {"p50_us": round(percentile(xs, 50) * 1e3, 2), "p99_us": round(percentile(xs, 99) * 1e3, 2),
                     "field_ops_per_s_at_p50": 2.0 * n ** 3 / (percentile(xs, 50) * 1e-3)}
    t0 = time.perf_counter()
    want = ctx.oracle.matmul(3, A, B)
    t_or = time.perf_counter() - t0
    Cd.zero_()
    graph.replay()
    torch.cuda.synchronize()
    graph_exact = bool(np.array_equal(Cd.cpu().numpy(), want))
    path()
    torch.cuda.synchronize()
    del graph
    return {"workload": "F_3 A, B 512x512 uniform", "reps": reps, **res,
            "bit_exact_vs_oracle": bool(np.array_equal(Cd.cpu().numpy(), want)),
            "graph_replay_bit_exact": graph_exact,
            "oracle_ms": round(t_or * 1e3, 2), "oracle_cores": ctx.oracle.max_threads(),
            "config": gfq.choose_config(3, n, n, n)}


# ------------------------------------------------------------------------------------
# c2_k: slab width sweep on the headline products
# ------------------------------------------------------------------------------------

def section_c2_k(ctx, data, reps=5):
    torch, gfq = ctx.torch, ctx.gfq
    out = {}
    for q in FIELDS:
        d = data[q]
        ref = d["Cp"]
        nb = gfq.packed_bytes(q, M, N)
        Ck = gfq.empty_packed(q, M, N)
        rows = []
        for k in range(4, 11):
            gfq.matmul(q, d["Ap"], d["Bp"], M, L, N, out=Ck, k=k)
            torch.cuda.synchronize()
            same = bool(torch.equal(Ck[:nb], ref[:nb]))
            warm(torch, lambda: gfq.matmul(q, d["Ap"], d["Bp"], M, L, N, out=Ck, k=k))
            gfq.set_timing(True)
            gfq.timing_read()
            for _ in range(reps):
                gfq.matmul(q, d["Ap"], d["Bp"], M, L, N, out=Ck, k=k)
            torch.cuda.synchronize()
            t = gfq.timing_read()
            gfq.set_timing(False)
            pm = t["product_ms"] / t["product_launches"]
            rm = (t["reduce_ms"] / t["reduce_launches"]) if t["reduce_launches"] else 0.0
            rows.append({"k": k, "product_ms": round(pm, 4), "partial_sum_ms": round(rm, 4),
                         "field_ops_per_s": 2.0 * M * L * N / ((pm + rm) * 1e-3),
                         **rooflines(q, M, L, N, {"k": k, "variant": 0}, pm, getattr(ctx, "peaks", None)),
                         "bit_exact": same})
        out[f"F_{q}"] = rows
    return out


# ------------------------------------------------------------------------------------
# mfma: comparison only -- the headline products as int8 matrix-core GEMMs
# ------------------------------------------------------------------------------------

def int8_product(torch, q, A8, B8):
    """C = A B over F_q from int8 GEMMs with int32 accumulation (exact while l (q-1)^2 <
    2^31): one GEMM and a reduction mod p for F_p; for GF(4) = F_2[x]/(x^2+x+1) the
    coefficient planes by Karatsuba, three GEMMs reduced mod 2; for GF(8) =
    F_2[x]/(x^3+x+1) the trinomial formula of Section 4.3, six GEMMs reduced mod 2; for
    F_9 = F_3[i]/(i^2+1) Karatsuba over F_3, three GEMMs reduced mod 3."""
    if q == 9:
        a0, a1 = torch.remainder(A8, 3), torch.div(A8, 3, rounding_mode="floor")
        b0, b1 = torch.remainder(B8, 3), torch.div(B8, 3, rounding_mode="floor")
        p00, p11 = torch._int_mm(a0, b0), torch._int_mm(a1, b1)
        pss = torch._int_mm(a0 + a1, b0 + b1)
        re, im = torch.remainder(p00 - p11, 3), torch.remainder(pss - p00 - p11, 3)
        return (re + 3 * im).to(torch.uint8)
    if q == 8:
        a = [(A8 >> d) & 1 for d in range(3)]
        b = [(B8 >> d) & 1 for d in range(3)]
        p00, p11, p22 = (torch._int_mm(a[i], b[i]) for i in range(3))
        p01 = torch._int_mm(a[0] ^ a[1], b[0] ^ b[1])
        p02 = torch._int_mm(a[0] ^ a[2], b[0] ^ b[2])
        p12 = torch._int_mm(a[1] ^ a[2], b[1] ^ b[2])
        # product coefficients c0..c4 mod 2, then x^3 = x + 1 and x^4 = x^2 + x
        c0, c1, c2 = p00, p01 - p00 - p11, p02 - p00 - p22 + p11
        c3, c4 = p12 - p11 - p22, p22
        r0, r1, r2 = (c0 + c3) & 1, (c1 + c3 + c4) & 1, (c2 + c4) & 1
        return (r0 + 2 * r1 + 4 * r2).to(torch.uint8)
    if q != 4:
        return torch.remainder(torch._int_mm(A8, B8), q).to(torch.uint8)
    a0, a1 = A8 & 1, A8 >> 1
    b0, b1 = B8 & 1, B8 >> 1
    p0, p1 = torch._int_mm(a0, b0), torch._int_mm(a1, b1)
    p2 = torch._int_mm(a0 + a1, b0 + b1)
    c0 = (p0 + p1) & 1                     # a0 b0 + a1 b1
    c1 = (p2 - p0) & 1                     # a0 b1 + a1 b0 + a1 b1
    return (c0 + 2 * c1).to(torch.uint8)


def section_mfma(ctx, data, reps=5):
    torch = ctx.torch
    out = {"note": "comparison only; not the method of the paper and not part of the library"}
    for q in FIELDS:
        d = data[q]
        A8, B8 = d["Ad"].view(torch.int8), d["Bd"].view(torch.int8)
        C = int8_product(torch, q, A8, B8)
        torch.cuda.synchronize()
        same = bool(torch.equal(C, d["Cd"]))
        warm(torch, lambda: int8_product(torch, q, A8, B8))
        ev = ctx.events(4)
        ev[0].record()
        for _ in range(reps):
            torch._int_mm(A8, B8)
        ev[1].record()
        for _ in range(reps):
            int8_product(torch, q, A8, B8)
        ev[2].record()
        torch.cuda.synchronize()
        gemm = ev[0].elapsed_time(ev[1]) / reps
        full = ev[1].elapsed_time(ev[2]) / reps
        out[f"F_{q}"] = {"int8_gemm_ms": round(gemm, 4), "with_mod_p_ms": round(full, 4),
                         "field_ops_per_s": 2.0 * M * L * N / (full * 1e-3),
                         "int8_gemm_ops_per_s": 2.0 * M * L * N / (gemm * 1e-3),
                         "equals_bitsliced_product": same}
    return out


# ------------------------------------------------------------------------------------
# c3: F_7 and GF(4), 16384 x 2048 times 2048 x 16384, dense and 10% density
# ------------------------------------------------------------------------------------

def section_c3(ctx, reps=5, sample_rows=32):
    import numpy as np
    torch, gfq, inputs = ctx.torch, ctx.gfq, ctx.inputs
    m, l, n = 16384, 2048, 16384
    res = {}
    for q in (7, 4):
        for density in (1.0, 0.1):
            A, B = inputs.pair(q, m, l, n, cfg=3, idx=q, density=density)
            Ad, Bd = ctx.up(A), ctx.up(B)
            Ap, Bp, Cp = gfq.empty_packed(q, m, l), gfq.empty_packed(q, l, n), gfq.empty_packed(q, m, n)
            Cd = torch.empty((m, n), dtype=torch.uint8, device=ctx.dev)

            def path():
                gfq.pack(q, Ad, out=Ap)
                gfq.pack(q, Bd, out=Bp)
                gfq.matmul(q, Ap, Bp, m, l, n, out=Cp)
                gfq.unpack(q, Cp, m, n, out=Cd)

            warm(torch, path)
            ev = ctx.events(2)
            ev[0].record()
            for _ in range(reps):
                path()
            ev[1].record()
            torch.cuda.synchronize()
            path_ms = ev[0].elapsed_time(ev[1]) / reps
            warm(torch, lambda: gfq.matmul(q, Ap, Bp, m, l, n, out=Cp))
            gfq.set_timing(True)
            gfq.timing_read()
            for _ in range(reps):
                gfq.matmul(q, Ap, Bp, m, l, n, out=Cp)
            torch.cuda.synchronize()
            t = gfq.timing_read()
            gfq.set_timing(False)
            pm = t["product_ms"] / t["product_launches"]
            rm = (t["reduce_ms"] / t["reduce_launches"]) if t["reduce_launches"] else 0.0
            cfg = gfq.choose_config(q, m, l, n)
            rows = np.sort(inputs.rng(3, q, 3).choice(m, size=sample_rows, replace=False))
            got = Cd[torch.from_numpy(rows).to(ctx.dev)].cpu().numpy()
            t0 = time.perf_counter()
            want = ctx.oracle.matmul(q, A[rows], B)
            oracle_s = time.perf_counter() - t0
            ok = bool(np.array_equal(got, want))
            # comparison only: the same product as int8 matrix-core GEMMs
            A8, B8 = Ad.view(torch.int8), Bd.view(torch.int8)
            C8 = int8_product(torch, q, A8, B8)
            torch.cuda.synchronize()
            same8 = bool(torch.equal(C8, Cd))
            del C8
            warm(torch, lambda: int8_product(torch, q, A8, B8))
            ev = ctx.events(2)
            ev[0].record()
            for _ in range(reps):
                int8_product(torch, q, A8, B8)
            ev[1].record()
            torch.cuda.synchronize()
            mfma_ms = ev[0].elapsed_time(ev[1]) / reps
            kara = None
            if q == 4:
                # the paper's own route for GF(4): matrix-level Karatsuba over F_2 (best of k)
                Ck = gfq.empty_packed(q, m, n)
                nb = gfq.packed_bytes(q, m, n)
                best = None
                for kk in (6, 7, 8):
                    gfq.matmul(q, Ap, Bp, m, l, n, out=Ck, k=kk, rows=2048, split=1, variant=gfq.VARIANT_KARATSUBA)
                    torch.cuda.synchronize()
                    same_k = bool(torch.equal(Ck[:nb], Cp[:nb]))
                    warm(torch, lambda: gfq.matmul(q, Ap, Bp, m, l, n, out=Ck, k=kk, rows=2048, split=1,
                                                   variant=gfq.VARIANT_KARATSUBA))
                    gfq.set_timing(True)
                    gfq.timing_read()
                    for _ in range(reps):
                        gfq.matmul(q, Ap, Bp, m, l, n, out=Ck, k=kk, rows=2048, split=1,
                                   variant=gfq.VARIANT_KARATSUBA)
                    torch.cuda.synchronize()
                    tk = gfq.timing_read()
                    gfq.set_timing(False)
                    msk = tk["product_ms"] / tk["product_launches"]
                    if best is None or msk < best["product_ms"]:
                        best = {"k": kk, "product_ms": round(msk, 4), "equals_rowwise": same_k}
                kara = best
                del Ck
            name = ("GF4" if q == 4 else f"F_{q}") + ("" if density == 1.0 else "_density0.1")
            res[name] = {"path_ms": round(path_ms, 4), "product_ms": round(pm, 4), "partial_sum_ms": round(rm, 4),
                         "field_ops_per_s_path": 2.0 * m * l * n / (path_ms * 1e-3),
                         "field_ops_per_s_product": 2.0 * m * l * n / ((pm + rm) * 1e-3),
                         **rooflines(q, m, l, n, cfg, pm, getattr(ctx, "peaks", None)),
                         # GF(4)'s accumulate is three XORs per unit against 16 bytes of table
                         # reads: its bound is the LDS port, F_7's the VALU
                         "bound": "lds" if q == 4 else "alu", "config": cfg,
                         "sampled_rows_bit_exact": ok, "sampled_rows": sample_rows,
                         "oracle_field_ops_per_s": 2.0 * sample_rows * l * n / oracle_s,
                         "oracle_threads": ctx.oracle.max_threads(),
                         "int8_mfma_comparison_ms": round(mfma_ms, 4), "int8_mfma_equals": same8}
            if kara is not None:
                res[name]["karatsuba_variant"] = kara
            del Ad, Bd, Ap, Bp, Cp, Cd
    return {"workload": "A 16384x2048, B 2048x16384; uniform and 10% density", **res}


# ------------------------------------------------------------------------------------
# ext: the extension fields GF(8) = F_2[x]/(x^3 + x + 1) (basis {1, x, x^2}) and
# F_9 = F_3[i]/(i^2 + 1) (basis {1, -1, i, -i}), row-wise
# ------------------------------------------------------------------------------------

def section_ext(ctx, reps=5, sample_rows=32):
    import numpy as np
    torch, gfq, inputs = ctx.torch, ctx.gfq, ctx.inputs
    res = {}
    cases = [(8, (16384, 2048, 16384), 1.0), (8, (16384, 2048, 16384), 0.1), (8, (M, L, N), 1.0),
             (9, (16384, 2048, 16384), 1.0), (9, (M, L, N), 1.0)]
    for q, (m, l, n), density in cases:
        A, B = inputs.pair(q, m, l, n, cfg=6, idx=q * 100000 + m + l, density=density)
        Ad, Bd = ctx.up(A), ctx.up(B)
        Ap, Bp, Cp = gfq.pack(q, Ad), gfq.pack(q, Bd), gfq.empty_packed(q, m, n)
        gfq.matmul(q, Ap, Bp, m, l, n, out=Cp)
        Cd = gfq.unpack(q, Cp, m, n)
        warm(torch, lambda: gfq.matmul(q, Ap, Bp, m, l, n, out=Cp))
        gfq.set_timing(True)
        gfq.timing_read()
        for _ in range(reps):
            gfq.matmul(q, Ap, Bp, m, l, n, out=Cp)
        torch.cuda.synchronize()
        t = gfq.timing_read()
        gfq.set_timing(False)
        pm = t["product_ms"] / t["product_launches"]
        rm = (t["reduce_ms"] / t["reduce_launches"]) if t["reduce_launches"] else 0.0
        cfg = gfq.choose_config(q, m, l, n)
        rows = np.sort(inputs.rng(6, m, 3).choice(m, size=sample_rows, replace=False))
        got = Cd[torch.from_numpy(rows).to(ctx.dev)].cpu().numpy()
        ok = bool(np.array_equal(got, ctx.oracle.matmul(q, A[rows], B)))
        A8, B8 = Ad.view(torch.int8), Bd.view(torch.int8)
        same8 = bool(torch.equal(int8_product(torch, q, A8, B8), Cd))
        warm(torch, lambda: int8_product(torch, q, A8, B8))
        ev = ctx.events(2)
        ev[0].record()
        for _ in range(reps):
            int8_product(torch, q, A8, B8)
        ev[1].record()
        torch.cuda.synchronize()
        mfma_ms = ev[0].elapsed_time(ev[1]) / reps
        # the matrix-level route (GF(8): trinomial formula over F_2; F_9: Karatsuba over F_3),
        # best of three slab widths, against the row-wise product
        best = None
        Ck = gfq.empty_packed(q, m, n)
        for kk in (5, 6, 7):
            gfq.matmul(q, Ap, Bp, m, l, n, out=Ck, k=kk, variant=gfq.VARIANT_KARATSUBA)
            torch.cuda.synchronize()
            same_k = bool(torch.equal(Ck, Cp))
            warm(torch, lambda: gfq.matmul(q, Ap, Bp, m, l, n, out=Ck, k=kk, variant=gfq.VARIANT_KARATSUBA))
            gfq.set_timing(True)
            gfq.timing_read()
            for _ in range(reps):
                gfq.matmul(q, Ap, Bp, m, l, n, out=Ck, k=kk, variant=gfq.VARIANT_KARATSUBA)
            torch.cuda.synchronize()
            tk = gfq.timing_read()
            gfq.set_timing(False)
            msk = (tk["product_ms"] + tk["reduce_ms"]) / tk["product_launches"]
            if best is None or msk < best["ms"]:
                best = {"k": kk, "ms": round(msk, 4), "equals_rowwise": same_k}
        del Ck
        name = ("GF8_" if q == 8 else "F9_") + f"{m}x{l}x{n}" + ("" if density == 1.0 else "_density0.1")
        res[name] = {"product_ms": round(pm, 4), "partial_sum_ms": round(rm, 4),
                     "field_ops_per_s_product": 2.0 * m * l * n / ((pm + rm) * 1e-3),
                     **rooflines(q, m, l, n, cfg, pm, getattr(ctx, "peaks", None)), "config": cfg,
                     "sampled_rows_bit_exact": ok, "sampled_rows": sample_rows,
                     "int8_mfma_comparison_ms": round(mfma_ms, 4), "int8_mfma_equals": same8,
                     "matrix_route": best}
        del Ad, Bd, Ap, Bp, Cp, Cd, A8, B8
        torch.cuda.empty_cache()
    return {"workload": "GF(8) and F_9, A m x l, B l x n uniform (and 10% density)", **res}


# ------------------------------------------------------------------------------------
# sw: Strassen-Winograd levels over the Four-Russians product (effective 2mln/t)
# ------------------------------------------------------------------------------------

def section_sw(ctx, reps=5, sizes=(8192, 16384), fields=(3, 5, 4, 8), max_levels=3):
    torch, gfq, inputs = ctx.torch, ctx.gfq, ctx.inputs
    res = {}
    for N in sizes:
        for q in fields:
            A, B = inputs.pair(q, N, N, N, cfg=7, idx=q * 100 + N % 97)
            Ap, Bp = gfq.pack(q, ctx.up(A)), gfq.pack(q, ctx.up(B))
            del A, B
            ref = gfq.matmul(q, Ap, Bp, N, N, N)
            Cp = gfq.empty_packed(q, N, N)
            row = {}
            for levels in range(0, max_levels + 1):
                gfq.matmul_sw(q, Ap, Bp, N, N, N, levels, out=Cp)
                torch.cuda.synchronize()
                same = bool(torch.equal(Cp, ref))
                warm(torch, lambda: gfq.matmul_sw(q, Ap, Bp, N, N, N, levels, out=Cp))
                ev = ctx.events(2)
                ev[0].record()
                for _ in range(reps):
                    gfq.matmul_sw(q, Ap, Bp, N, N, N, levels, out=Cp)
                ev[1].record()
                torch.cuda.synchronize()
                ms = ev[0].elapsed_time(ev[1]) / reps
                row[f"levels{levels}"] = {"ms": round(ms, 4), "field_ops_per_s": 2.0 * N ** 3 / (ms * 1e-3),
                                          "equals_plain": same}
            # the tuner's choice for this size class (GFQ_SW_AUTO; 0 levels without an entry)
            gfq.matmul_sw(q, Ap, Bp, N, N, N, gfq.SW_AUTO, out=Cp)
            torch.cuda.synchronize()
            same = bool(torch.equal(Cp, ref))
            warm(torch, lambda: gfq.matmul_sw(q, Ap, Bp, N, N, N, gfq.SW_AUTO, out=Cp))
            ev = ctx.events(2)
            ev[0].record()
            for _ in range(reps):
                gfq.matmul_sw(q, Ap, Bp, N, N, N, gfq.SW_AUTO, out=Cp)
            ev[1].record()
            torch.cuda.synchronize()
            ms = ev[0].elapsed_time(ev[1]) / reps
            row["auto"] = {"levels": gfq.tune_sw_lookup(q, N, N, N), "ms": round(ms, 4),
                           "field_ops_per_s": 2.0 * N ** 3 / (ms * 1e-3), "equals_plain": same}
            base = row["levels0"]["ms"]
            for v in row.values():
                v["speedup"] = round(base / v["ms"], 3)
            res[("GF" if q in (4, 8) else "F_") + f"{q}_{N}"] = row
            del Ap, Bp, ref, Cp
            torch.cuda.empty_cache()
    return {"workload": "square N x N products, uniform entries; levels 0 = the plain product; "
                        "rate = classical 2 N^3 / t", **res}


# ------------------------------------------------------------------------------------
# c4: 4096 products of mixed fields and shapes, batched against plain launches
# ------------------------------------------------------------------------------------

def section_c4(ctx, count=4096, reps=5, pool=2048):
    import numpy as np
    torch, gfq, inputs = ctx.torch, ctx.gfq, ctx.inputs
    specs = inputs.batch_specs(count, cfg=4)
    offs = inputs.window_offsets(4, [(m, l, n) for (_, m, l, n) in specs], pool)
    pools_h = {q: (inputs.matrix(q, pool, pool, cfg=4, idx=q, which=0),
                   inputs.matrix(q, pool, pool, cfg=4, idx=q, which=1)) for q in (3, 5, 7)}
    pools = {q: (ctx.up(a), ctx.up(b)) for q, (a, b) in pools_h.items()}
    probs, plain_out = [], []
    for (q, m, l, n), (ra, ca, rb, cb) in zip(specs, offs):
        Pa, Pb = pools[q]
        probs.append((q, m, l, n, gfq.pack(q, Pa[ra:ra + m, ca:ca + l]), gfq.pack(q, Pb[rb:rb + l, cb:cb + n]),
                      gfq.empty_packed(q, m, n)))
        plain_out.append(gfq.empty_packed(q, m, n))
    torch.cuda.synchronize()
    ops = sum(2.0 * m * l * n for (_, m, l, n) in specs)

    b = gfq.Batch(probs)
    b.launch()
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        b.launch()                     # an eager launch on the capture stream first: the
        side.synchronize()             # library's side streams for it exist before capture
        with torch.cuda.graph(graph, stream=side):
            b.launch()
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    graph.replay()
    torch.cuda.synchronize()
    ev = ctx.events(2)
    ev[0].record()
    for _ in range(reps):
        graph.replay()
    ev[1].record()
    torch.cuda.synchronize()
    batched_ms = ev[0].elapsed_time(ev[1]) / reps
    graph.replay()
    torch.cuda.synchronize()
    done_us = sorted(b.times_us())
    want = [C.clone() for (*_, C) in probs]

    # the same items drained by persistent workgroups through a device queue head, captured
    # the same way
    pgraph = torch.cuda.CUDAGraph()
    with torch.cuda.stream(side):
        b.launch_persistent()
        side.synchronize()
        with torch.cuda.graph(pgraph, stream=side):
            b.launch_persistent()
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    for (*_, C) in probs:
        C.zero_()
    warm(torch, pgraph.replay)
    ev[0].record()
    for _ in range(reps):
        pgraph.replay()
    ev[1].record()
    torch.cuda.synchronize()
    persistent_ms = ev[0].elapsed_time(ev[1]) / reps
    persistent_same = all(torch.equal(w, C) for w, (*_, C) in zip(want, probs))
    persistent_done_us = sorted(b.times_us())
    del pgraph

    def plain():
        for (q, m, l, n, A, B, _), C in zip(probs, plain_out):
            gfq.matmul(q, A, B, m, l, n, out=C)

    plain()
    torch.cuda.synchronize()
    ev[0].record()
    for _ in range(reps):
        plain()
    ev[1].record()
    torch.cuda.synchronize()
    plain_ms = ev[0].elapsed_time(ev[1]) / reps
    same = all(torch.equal(C[:gfq.packed_bytes(q, m, n)], C2[:gfq.packed_bytes(q, m, n)])
               for (q, m, l, n, _, _, C), C2 in zip(probs, plain_out))
    # the method's work per product at the slab width the batch gave it: the batch's VALU
    # fraction over the replay time
    ks = b.slab_widths()
    batch_ops = sum(algorithmic_ops(q, m, l, n, k, C_ACC, C_ADD) for (q, m, l, n), k in zip(specs, ks))
    # every product against the oracle (timed: the oracle's rate on this workload)
    ok, oracle_s = True, 0.0
    t_log = time.monotonic() + 10.0
    for i in range(count):
        if time.monotonic() > t_log:
            log(f"c4 check: oracle {i} of {count}")
            t_log += 10.0
        q, m, l, n = specs[i]
        ra, ca, rb, cb = offs[i]
        got = gfq.unpack(q, probs[i][6], m, n).cpu().numpy()
        t0 = time.perf_counter()
        want = ctx.oracle.matmul(q, pools_h[q][0][ra:ra + m, ca:ca + l], pools_h[q][1][rb:rb + l, cb:cb + n])
        oracle_s += time.perf_counter() - t0
        ok = ok and bool(np.array_equal(got, want))
    del graph
    b.destroy()
    return {"workload": f"{count} products, field uniform over F_3/F_5/F_7, m, l, n log-uniform in [64, 2048], "
                        f"operands uniform windows of seeded {pool}x{pool} pools",
            "field_ops": ops,
            "batched_ms": round(persistent_ms, 4), "batched_field_ops_per_s": ops / (persistent_ms * 1e-3),
            "batched_launch": "persistent workgroups draining a device queue per (field, tile height), "
                              "captured in one HIP graph",
            "completion_p50_us": round(percentile(persistent_done_us, 50), 1),
            "completion_p99_us": round(percentile(persistent_done_us, 99), 1),
            "batched_alu_frac": round(batch_ops / (persistent_ms * 1e-3) / PEAK_VALU_OPS, 4),
            "worklist_ms": round(batched_ms, 4), "worklist_field_ops_per_s": ops / (batched_ms * 1e-3),
            "worklist_launch": "one workgroup per item of the same lists, captured in one HIP graph",
            "worklist_completion_p50_us": round(percentile(done_us, 50), 1),
            "worklist_completion_p99_us": round(percentile(done_us, 99), 1),
            "persistent_equals_worklist": persistent_same,
            "plain_ms": round(plain_ms, 4), "plain_field_ops_per_s": ops / (plain_ms * 1e-3),
            "speedup": round(plain_ms / persistent_ms, 2),
            "batched_equals_plain": same, "oracle_all_bit_exact": ok, "oracle_checked": count,
            "oracle_field_ops_per_s": ops / oracle_s, "oracle_threads": ctx.oracle.max_threads(),
            "tuned_classes_used": ctx.tuned}


# ------------------------------------------------------------------------------------
# c4_slices: a batch of products with few tiles and a long inner dimension, whose tiles the
# batch cuts into slab slices (partial products summed by a partial-sum launch)
# ------------------------------------------------------------------------------------

def section_c4_slices(ctx, per_field=16, shape=(512, 16384, 512), reps=10, sample_rows=8):
    import numpy as np
    torch, gfq, inputs = ctx.torch, ctx.gfq, ctx.inputs
    m, l, n = shape
    specs = [(q, m, l, n) for q in (3, 5, 7) for _ in range(per_field)]
    probs, host = [], []
    for i, (q, _, _, _) in enumerate(specs):
        A, B = inputs.pair(q, m, l, n, cfg=8, idx=i)
        probs.append((q, m, l, n, gfq.pack(q, ctx.up(A)), gfq.pack(q, ctx.up(B)), gfq.empty_packed(q, m, n)))
        host.append((A, B))
    b = gfq.Batch(probs)
    slices = b.slices()
    b.launch()
    torch.cuda.synchronize()
    warm(torch, b.launch)
    ev = ctx.events(2)
    ev[0].record()
    for _ in range(reps):
        b.launch()
    ev[1].record()
    torch.cuda.synchronize()
    batched_ms = ev[0].elapsed_time(ev[1]) / reps
    done_us = sorted(b.times_us())
    got = [gfq.unpack(q, C, m, n).cpu().numpy() for (q, _, _, _, _, _, C) in probs]
    want = [C.clone() for (*_, C) in probs]
    warm(torch, b.launch_persistent)
    ev[0].record()
    for _ in range(reps):
        b.launch_persistent()
    ev[1].record()
    torch.cuda.synchronize()
    persistent_ms = ev[0].elapsed_time(ev[1]) / reps
    persistent_same = all(torch.equal(w, C) for w, (*_, C) in zip(want, probs))
    plain_out = [gfq.empty_packed(q, m, n) for (q, _, _, _) in specs]

    def plain():
        for (q, _, _, _, A, B, _), C in zip(probs, plain_out):
            gfq.matmul(q, A, B, m, l, n, out=C)

    warm(torch, plain)
    ev[0].record()
    for _ in range(reps):
        plain()
    ev[1].record()
    torch.cuda.synchronize()
    plain_ms = ev[0].elapsed_time(ev[1]) / reps
    same = all(torch.equal(C[:gfq.packed_bytes(q, m, n)], C2[:gfq.packed_bytes(q, m, n)])
               for (q, _, _, _, _, _, C), C2 in zip(probs, plain_out))
    rows = np.sort(inputs.rng(8, m, 1).choice(m, size=sample_rows, replace=False))
    ok = all(np.array_equal(got[i][rows], ctx.oracle.matmul(specs[i][0], host[i][0][rows], host[i][1]))
             for i in range(len(specs)))
    ops = 2.0 * m * l * n * len(specs)
    b.destroy()
    return {"workload": f"{len(specs)} products {m}x{l}x{n} ({per_field} each over F_3, F_5, F_7), uniform",
            "batched_ms": round(batched_ms, 4), "batched_field_ops_per_s": ops / (batched_ms * 1e-3),
            "plain_ms": round(plain_ms, 4), "plain_field_ops_per_s": ops / (plain_ms * 1e-3),
            "speedup": round(plain_ms / batched_ms, 2), "slices": sorted(set(slices)),
            "persistent_ms": round(persistent_ms, 4), "persistent_equals_worklist": persistent_same,
            "completion_p50_us": round(percentile(done_us, 50), 1),
            "completion_p99_us": round(percentile(done_us, 99), 1),
            "batched_equals_plain": same, "sampled_rows_bit_exact": bool(ok), "sampled_rows": sample_rows}


# ------------------------------------------------------------------------------------
# c5: served requests, continuous batching vs serial plain launches
# ------------------------------------------------------------------------------------

def section_c5(ctx, count=20000, budget=200 * 10 ** 9, pool=4096, load=0.8):
    import numpy as np
    torch, gfq, inputs = ctx.torch, ctx.gfq, ctx.inputs
    trace = inputs.request_trace(count, cfg=5)                 # unit-rate arrivals, rescaled below
    shapes = [(n, n, n) for (_, _, n) in trace]
    offs = inputs.window_offsets(5, shapes, pool)
    qs = sorted({q for (_, q, _) in trace})
    pools_h = {q: (inputs.matrix(q, pool, pool, cfg=5, idx=q, which=0),
                   inputs.matrix(q, pool, pool, cfg=5, idx=q, which=1)) for q in qs}
    pools = {q: (ctx.up(a), ctx.up(b)) for q, (a, b) in pools_h.items()}
    sizes = np.array([n * n for (_, _, n) in trace], dtype=np.int64)
    starts = np.concatenate([[0], np.cumsum(((sizes + 255) // 256) * 256)[:-1]])
    total = int(starts[-1] + sizes[-1] + 256)
    outs = [torch.empty(total, dtype=torch.uint8, device=ctx.dev) for _ in range(2)]
    ops = np.array([2.0 * n ** 3 for (_, _, n) in trace])
    # every result is also copied to host memory before its completion is reported, so the
    # latency runs from arrival to the result on the host: request i's copy goes to a ring of
    # pinned host memory (requests in flight at once are far less than a ring apart)
    ring_bytes = 2 << 30
    ring = torch.empty(ring_bytes, dtype=torch.uint8, pin_memory=True)
    ring_off, pos = [], 0
    for (_, _, n) in trace:
        if pos + n * n > ring_bytes:
            pos = 0
        ring_off.append(pos)
        pos += (n * n + 255) // 256 * 256

    def requests(out, idx, t0_us, us_per_unit):
        rs = []
        base = out.data_ptr()
        for i in idx:
            t, q, n = trace[i]
            ra, ca, rb, cb = offs[i]
            Pa, Pb = pools[q]
            rs.append(gfq.Request(q, n, n, n, Pa.data_ptr() + ra * pool + ca, pool, Pb.data_ptr() + rb * pool + cb,
                                  pool, base + int(starts[i]), n, 0, i, t0_us + t * us_per_unit,
                                  ring.data_ptr() + ring_off[i]))
        return rs

    def run(srv, idx, out, us_per_unit, timeout_s):
        t0 = srv.now_us() + 20000.0
        rs = requests(out, idx, t0 if us_per_unit else 0.0, us_per_unit)
        srv.submit(rs)
        comps, t_end, t_log = [], time.monotonic() + timeout_s, time.monotonic() + 10.0
        while len(comps) < len(rs):
            if time.monotonic() > t_end:
                raise TimeoutError(f"c5: {len(comps)} of {len(rs)} requests done after {timeout_s} s")
            comps += srv.poll(timeout_us=20000.0)
            if time.monotonic() > t_log:
                log(f"c5: {len(comps)} of {len(rs)} requests done")
                t_log += 10.0
        assert all(c["status"] == 0 for c in comps), [c for c in comps if c["status"]][:3]
        return comps

    def summary(comps, srv):
        lat = [(c["done_us"] - c["arrival_us"]) * 1e-3 for c in comps]
        first = min(c["arrival_us"] for c in comps)
        last = max(c["done_us"] for c in comps)
        tot = sum(ops[c["tag"]] for c in comps)
        st = srv.stats()
        return {"requests": len(comps), "span_s": round((last - first) * 1e-6, 4),
                "field_ops_per_s": tot / ((last - first) * 1e-6),
                "requests_per_s": len(comps) / ((last - first) * 1e-6),
                "latency_p50_ms": round(percentile(lat, 50), 3), "latency_p99_ms": round(percentile(lat, 99), 3),
                "latency_max_ms": round(max(lat), 3),
                "batches": st["batches"], "mean_batch": round(st["completed"] / max(1, st["batches"]), 2),
                "max_batch": st["max_batch_seen"], "arena_peak_bytes": st["arena_peak_in_use"]}

    torch.cuda.synchronize()
    srv = gfq.Server(budget_bytes=budget, slots=3, max_batch=256)
    # capacity: a prefix of the trace submitted at once, drained as fast as possible
    cal = list(range(min(2000, count)))
    comps = run(srv, cal, outs[0], 0.0, 300.0)
    span = (max(c["done_us"] for c in comps) - min(c["arrival_us"] for c in comps)) * 1e-6
    mu = len(cal) / span
    lam = load * mu
    us_per_unit = 1e6 / lam
    log(f"c5: capacity {mu:.0f} req/s, offered {lam:.0f} req/s")
    comps_b = run(srv, range(count), outs[0], us_per_unit, 600.0)
    served = summary(comps_b, srv)
    srv.destroy()
    log("c5: continuous batching done; serial plain launches")
    srv = gfq.Server(budget_bytes=budget, serial=True)
    comps_s = run(srv, range(count), outs[1], us_per_unit, 900.0)
    serial = summary(comps_s, srv)
    srv.destroy()
    torch.cuda.synchronize()
    identical = bool(torch.equal(outs[0], outs[1]))
    del outs[1]
    check = c5_check(ctx, trace, offs, pools_h, outs[0], starts)
    del outs, ring
    return {"workload": f"{count} requests, field uniform over {{3,4,5,7}}, square n log-uniform in [128, 4096], "
                        f"Poisson arrivals at {load} x the measured capacity; operands uniform windows of seeded "
                        f"{pool}x{pool} pools; result = unpacked uint8 C in device memory, copied to pinned host "
                        f"memory before the completion (latency = arrival to the result on the host)",
            "budget_bytes": budget, "capacity_req_per_s": round(mu, 1), "offered_req_per_s": round(lam, 1),
            "continuous_batching": served, "serial_plain": serial,
            "p99_ratio_serial_over_batched": round(serial["latency_p99_ms"] / served["latency_p99_ms"], 2),
            "results_identical_batched_vs_serial": identical, **check}


def c5_check(ctx, trace, offs, pools_h, out, starts, vectors=8):
    """The served products against the oracle: every request with n <= 1024 and a seeded 2%
    of the larger ones in full, and every request by Freivalds' check, C X = A (B X) for
    `vectors` random columns X over the field (a wrong C passes with probability at most
    q^-vectors).  C X is formed from the served C in device memory (float64 products of
    exact integers, reduced in the field); A (B X) by the oracle on the host."""
    import numpy as np
    torch, inputs, oracle = ctx.torch, ctx.inputs, ctx.oracle
    big = [i for i, (_, _, n) in enumerate(trace) if n > 1024]
    pick = inputs.rng(5, 2, 2).choice(len(big), size=max(1, len(big) // 50), replace=False) if big else []
    full = sorted([i for i, (_, _, n) in enumerate(trace) if n <= 1024] + [big[j] for j in pick])
    ok_full, full_ops, full_s = True, 0.0, 0.0
    t_log = time.monotonic() + 10.0
    for done, i in enumerate(full):
        if time.monotonic() > t_log:
            log(f"c5 check: oracle {done} of {len(full)}")
            t_log += 10.0
        _, q, n = trace[i]
        ra, ca, rb, cb = offs[i]
        got = out[int(starts[i]):int(starts[i]) + n * n].view(n, n).cpu().numpy()
        t0 = time.perf_counter()
        want = oracle.matmul(q, pools_h[q][0][ra:ra + n, ca:ca + n], pools_h[q][1][rb:rb + n, cb:cb + n])
        full_s += time.perf_counter() - t0
        full_ops += 2.0 * n ** 3
        ok_full = ok_full and bool(np.array_equal(got, want))

    def cx_on_device(q, C, X):
        Xd = torch.from_numpy(X).to(C.device).double()
        if q != 4:
            return torch.remainder(C.double() @ Xd, q).to(torch.uint8).cpu().numpy()
        c0, c1 = (C & 1).double(), (C >> 1).double()
        x0, x1 = torch.remainder(Xd, 2), torch.div(Xd, 2, rounding_mode="floor")
        y0 = torch.remainder(c0 @ x0 + c1 @ x1, 2)                 # x^2 = x + 1
        y1 = torch.remainder(c0 @ x1 + c1 @ x0 + c1 @ x1, 2)
        return (y0 + 2 * y1).to(torch.uint8).cpu().numpy()

    # A (B X) as the transpose of X^T B^T A^T (the fields are commutative): rows as long as
    # the matrices, so the oracle's inner loop runs over n columns, not over the vectors;
    # the operand windows come from the transposed pools
    pools_t = {q: (np.ascontiguousarray(a.T), np.ascontiguousarray(b.T)) for q, (a, b) in pools_h.items()}
    ok_fr = True
    for i, (_, q, n) in enumerate(trace):
        if time.monotonic() > t_log:
            log(f"c5 check: Freivalds {i} of {len(trace)}")
            t_log += 10.0
        ra, ca, rb, cb = offs[i]
        X = inputs.rng(5, 3, i).integers(0, q, size=(n, vectors), dtype=np.uint8)
        C = out[int(starts[i]):int(starts[i]) + n * n].view(n, n)
        lhs = cx_on_device(q, C, X)
        At, Bt = pools_t[q][0][ca:ca + n, ra:ra + n], pools_t[q][1][cb:cb + n, rb:rb + n]
        rhs = oracle.matmul(q, oracle.matmul(q, np.ascontiguousarray(X.T), Bt), At).T
        ok_fr = ok_fr and bool(np.array_equal(lhs, rhs))
    return {"oracle_full_checked": len(full), "oracle_full_bit_exact": ok_full,
            "oracle_full_rule": "every request with n <= 1024 and a seeded 2% of the larger ones",
            "oracle_field_ops_per_s": full_ops / full_s, "oracle_threads": oracle.max_threads(),
            "freivalds_checked": len(trace), "freivalds_vectors": vectors, "freivalds_all_pass": ok_fr}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--only", default=",".join(SECTIONS),
                    help="comma-separated sections after the headline (" + ",".join(SECTIONS) + "; empty = none)")
    ap.add_argument("--c5-requests", type=int, default=20000)
    ap.add_argument("--tune-file", default=os.path.join(ROOT, "paper_0901_1413_amd", "tuning", "gfx950.txt"),
                    help="tuning cache to load (skipped if missing)")
    ap.add_argument("--copy-mb", type=int, default=0,
                    help="first run one device-to-device copy of this many MiB (a kernel of known "
                         "traffic that calibrates hardware memory counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported: the library drives one "
              f"MI355X and reports that GPU's throughput", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_0901_1413_amd import gfq, inputs
    import oracle

    torch.cuda.set_device(0)
    gfq.load()
    ctx = Ctx(torch, gfq, inputs, oracle)
    ctx.tuned = False
    if args.tune_file and os.path.exists(args.tune_file):
        gfq.tune_load(args.tune_file)
        ctx.tuned = True

    if args.copy_mb:
        src = torch.ones(args.copy_mb << 20, dtype=torch.uint8, device=ctx.dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    log("machine peaks")
    ctx.peaks = section_peaks(ctx)
    log("headline")
    out, data = headline(ctx, args)
    out["tuning_cache_loaded"] = ctx.tuned
    out["machine_peaks"] = ctx.peaks
    sections = [s for s in args.only.split(",") if s]
    res = {}
    for s in sections:
        if s not in SECTIONS:
            raise SystemExit(f"unknown section {s}")
    if "c2_k" in sections:
        log("c2_k")
        res["c2_k"] = section_c2_k(ctx, data)
    if "mfma" in sections:
        log("mfma")
        res["mfma"] = section_mfma(ctx, data)
    if not args.no_cpu:
        for q in FIELDS:
            data[q]["C_host"] = data[q]["Cd"].cpu().numpy()
        log("cpu baseline")
        out["cpu_baseline"] = cpu_baseline(ctx, data)
    del data
    torch.cuda.empty_cache()
    if "c1" in sections:
        log("c1")
        res["c1"] = section_c1(ctx)
    if "c3" in sections:
        log("c3")
        res["c3"] = section_c3(ctx)
        torch.cuda.empty_cache()
    if "ext" in sections:
        log("ext")
        res["ext"] = section_ext(ctx)
        torch.cuda.empty_cache()
    if "sw" in sections:
        log("sw")
        res["sw"] = section_sw(ctx)
        torch.cuda.empty_cache()
    if "c4" in sections:
        log("c4")
        res["c4"] = section_c4(ctx)
        torch.cuda.empty_cache()
    if "c4_slices" in sections:
        log("c4_slices")
        res["c4_slices"] = section_c4_slices(ctx)
        torch.cuda.empty_cache()
    if "c5" in sections:
        log("c5")
        res["c5"] = section_c5(ctx, count=args.c5_requests)
        torch.cuda.empty_cache()
    if res:
        out["sections"] = res
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
