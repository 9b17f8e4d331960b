"""Compile libgfq.so (HIP, gfx950) in-tree with hipcc."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libgfq.so")
SOURCES = ["gfq_m4rm_gf4.hip", "gfq_m4rm_gf8.hip", "gfq_m4rm_f9.hip", "gfq_m4rm_f5.hip", "gfq_m4rm_f7.hip",
           "gfq_m4rm_f3.hip", "gfq_m4rm.hip", "gfq_batch.hip", "gfq_pack.hip", "gfq_sw.hip", "gfq_noalloc.hip", "gfq_probe.hip", "gfq_api.cpp", "gfq_batch_host.cpp", "gfq_tune.cpp",
           "gfq_server.cpp"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS_CC = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
            # packed-fp32 forms are kept out of every HIP build
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-Wall", "-Wno-unused-command-line-argument", "-pthread",
            "-I", os.path.join(ROOT, "include"), "-I", CSRC]
FLAGS_LINK = ["--offload-arch=gfx950", "-shared", "-fPIC", "-pthread"]


def _run(cmd):
    res = subprocess.run(cmd, capture_output=True, text=True)
    noise = ("packed-fp32-ops", "is not a recognized feature")
    err = "\n".join(l for l in res.stderr.splitlines() if not any(s in l for s in noise))
    return res.returncode, err


def build(verbose: bool = False) -> str:
    """Compile every source to an object (in parallel) and link libgfq.so."""
    from concurrent.futures import ThreadPoolExecutor
    objdir = os.path.join(HERE, "_build")
    os.makedirs(objdir, exist_ok=True)
    jobs = []
    for s in SOURCES:
        obj = os.path.join(objdir, os.path.splitext(s)[0] + ".o")
        cc = [HIPCC, *FLAGS_CC, "-c", "-o", obj, os.path.join(CSRC, s)]
        jobs.append((obj, cc))
    workers = max(1, min(len(jobs), int(os.environ.get("MAX_JOBS", os.cpu_count() or 4)), 8))
    with ThreadPoolExecutor(max_workers=workers) as ex:
        results = list(ex.map(lambda j: _run(j[1]), jobs))
    failed = False
    for (obj, cc), (rc, err) in zip(jobs, results):
        if verbose:
            print(" ".join(cc), flush=True)
        if err.strip() and (rc != 0 or verbose):
            sys.stderr.write(err + "\n")
        failed = failed or rc != 0
    if failed:
        raise RuntimeError("hipcc failed building libgfq.so")
    tmp = LIB + ".tmp"
    link = [HIPCC, *FLAGS_LINK, "-o", tmp, *[o for o, _ in jobs]]
    rc, err = _run(link)
    if rc != 0:
        sys.stderr.write(err + "\n")
        raise RuntimeError("linking libgfq.so failed")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
