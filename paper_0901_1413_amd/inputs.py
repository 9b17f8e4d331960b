"""Seeded synthetic inputs shared by the tests, the smoke check and the benchmark.

This module holds no field arithmetic: it only draws canonical element values, shapes,
field choices and arrival times from numpy's PCG64, keyed by a SeedSequence of
(config, index, which) so that every consumer regenerates identical data.

Conventions (one per workload family):
  * uniform:  every entry i.i.d. uniform over the canonical values [0, q).
  * density:  entry is 0 with probability 1 - density, else uniform over [1, q).
  * log-uniform integer in [lo, hi]: round(exp(U(ln lo, ln hi))), clamped.
"""
from __future__ import annotations

import numpy as np

A_SIDE, B_SIDE, META = 0, 1, 2


def rng(cfg: int, idx: int = 0, which: int = 0) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence([cfg, idx, which])))


def matrix(q: int, rows: int, cols: int, cfg: int, idx: int = 0, which: int = 0,
           density: float = 1.0) -> np.ndarray:
    """rows x cols canonical uint8 entries for field q (q = 4 is GF(4))."""
    g = rng(cfg, idx, which)
    if density >= 1.0:
        return g.integers(0, q, size=(rows, cols), dtype=np.uint8)
    nz = g.random((rows, cols)) < density
    vals = g.integers(1, q, size=(rows, cols), dtype=np.uint8)
    return np.where(nz, vals, 0).astype(np.uint8)


def pair(q: int, m: int, l: int, n: int, cfg: int, idx: int = 0, density: float = 1.0):
    """(A, B) for one product, A m x l and B l x n."""
    return (matrix(q, m, l, cfg, idx, A_SIDE, density),
            matrix(q, l, n, cfg, idx, B_SIDE, density))


def log_uniform_int(g: np.random.Generator, lo: int, hi: int, size=None):
    v = np.exp(g.uniform(np.log(lo), np.log(hi), size=size))
    return np.clip(np.rint(v), lo, hi).astype(np.int64)


def batch_specs(count: int, cfg: int, fields=(3, 5, 7), lo: int = 64, hi: int = 2048):
    """[(q, m, l, n)] for a batch of independent products (field uniform, sizes log-uniform)."""
    g = rng(cfg, 0, META)
    qs = g.choice(np.asarray(fields), size=count)
    dims = log_uniform_int(g, lo, hi, size=(count, 3))
    return [(int(qs[i]), int(dims[i, 0]), int(dims[i, 1]), int(dims[i, 2])) for i in range(count)]


def request_trace(count: int, cfg: int, fields=(3, 5, 7, 4), lo: int = 128, hi: int = 4096,
                  rate: float = 1.0):
    """[(arrival_s, q, n)] square-product requests with Poisson arrivals at `rate` per s."""
    g = rng(cfg, 0, META)
    qs = g.choice(np.asarray(fields), size=count)
    ns = log_uniform_int(g, lo, hi, size=count)
    gaps = g.exponential(1.0 / rate, size=count)
    t = np.cumsum(gaps)
    return [(float(t[i]), int(qs[i]), int(ns[i])) for i in range(count)]


def window_offsets(cfg: int, shapes, pool: int):
    """Seeded top-left corners for operand windows of pool x pool matrices: for each
    (m, l, n) in shapes, (ra, ca) for an m x l window of the A pool and (rb, cb) for an
    l x n window of the B pool, each uniform over the positions where the window fits.
    Every window of a uniform i.i.d. pool is itself uniform i.i.d."""
    g = rng(cfg, 1, META)
    out = []
    for (m, l, n) in shapes:
        assert max(m, l, n) <= pool
        ra, ca = g.integers(0, pool - m + 1), g.integers(0, pool - l + 1)
        rb, cb = g.integers(0, pool - l + 1), g.integers(0, pool - n + 1)
        out.append((int(ra), int(ca), int(rb), int(cb)))
    return out
