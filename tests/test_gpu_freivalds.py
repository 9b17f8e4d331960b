"""Whole-output checks of the full-size products (every element, probabilistically).

Freivalds: for random X (n x 32 over F_q), C = A B implies C X = A (B X).  The three
products with X are computed by the oracle (32 columns are cheap at any size), C by the HIP
path.  A wrong C passes with probability at most q^-32 per product.  The shapes are the
benchmark's: 8192^3 (F_3, F_5; GF(8), F_9) and 16384 x 2048 x 16384 (F_7, GF(4); dense and
10% density; and every field in the shipped table's configuration), plus a two-level
Strassen-Winograd product."""
import numpy as np
import pytest

import oracle
from paper_0901_1413_amd import inputs

pytestmark = pytest.mark.gpu
VECTORS = 32


def freivalds(q, A, B, C, seed):
    n = B.shape[1]
    X = inputs.matrix(q, n, VECTORS, cfg=240, idx=seed)
    BX = oracle.matmul(q, B, X)
    ABX = oracle.matmul(q, A, BX)
    CX = oracle.matmul(q, C, X)
    return np.array_equal(ABX, CX)


def product(g, q, A, B, levels=0):
    import torch
    m, l = A.shape
    n = B.shape[1]
    Ap = g.pack(q, torch.from_numpy(A).cuda())
    Bp = g.pack(q, torch.from_numpy(B).cuda())
    Cp = g.matmul_sw(q, Ap, Bp, m, l, n, levels) if levels else g.matmul(q, Ap, Bp, m, l, n)
    return g.unpack(q, Cp, m, n).cpu().numpy()


@pytest.mark.parametrize("q,shape", [(3, (8192, 8192, 8192)), (5, (8192, 8192, 8192)),
                                     (7, (16384, 2048, 16384)), (4, (16384, 2048, 16384)),
                                     (8, (8192, 8192, 8192)), (9, (8192, 8192, 8192))])
def test_full_size_freivalds(gfq_gpu, q, shape):
    m, l, n = shape
    A, B = inputs.pair(q, m, l, n, cfg=241, idx=q)
    C = product(gfq_gpu, q, A, B)
    assert freivalds(q, A, B, C, seed=q)
    # the check catches one wrong element (a planted error, on the CPU copy)
    C[m // 3, n // 2] = (C[m // 3, n // 2] + 1) % q
    assert not freivalds(q, A, B, C, seed=q)


@pytest.mark.parametrize("q", [7, 4])
def test_sparse_16384x2048x16384_freivalds(gfq_gpu, q):
    """The 10%-density variant of the rectangular workload (zero with probability 0.9, else
    uniform non-zero), every element."""
    m, l, n = 16384, 2048, 16384
    A, B = inputs.pair(q, m, l, n, cfg=244, idx=q, density=0.1)
    C = product(gfq_gpu, q, A, B)
    assert freivalds(q, A, B, C, seed=300 + q)
    C[m - 1, 7] = (C[m - 1, 7] + 1) % q
    assert not freivalds(q, A, B, C, seed=300 + q)


@pytest.mark.parametrize("q", [3, 5, 7, 4])
def test_tuned_16384x2048x16384_freivalds(gfq_gpu, q):
    """The rectangular workload in the shipped table's configuration for its class."""
    import os
    g = gfq_gpu
    m, l, n = 16384, 2048, 16384
    table = os.path.join(os.path.dirname(g.__file__), "tuning", "gfx950.txt")
    g.tune_clear()
    try:
        g.tune_load(table)
        assert g.tune_lookup(q, m, l, n) is not None
        A, B = inputs.pair(q, m, l, n, cfg=245, idx=q)
        C = product(g, q, A, B)
        assert freivalds(q, A, B, C, seed=400 + q)
    finally:
        g.tune_clear()


@pytest.mark.parametrize("q", [3, 5])
def test_strassen_winograd_8192_freivalds(gfq_gpu, q):
    N = 8192
    A, B = inputs.pair(q, N, N, N, cfg=242, idx=q)
    C = product(gfq_gpu, q, A, B, levels=2)
    assert freivalds(q, A, B, C, seed=100 + q)


@pytest.mark.parametrize("q", [3, 5, 4])
def test_full_size_tuned_configuration(gfq_gpu, q):
    """The benchmark's launches: the shipped tuning table loaded, the 8192^3 product runs in
    the configuration the table holds for its class (the one the benchmark times; GF(4): the
    exchanged-read 32-word tiles at k = 8), and every element passes Freivalds' check."""
    import os
    g = gfq_gpu
    N = 8192
    table = os.path.join(os.path.dirname(g.__file__), "tuning", "gfx950.txt")
    g.tune_clear()
    try:
        g.tune_load(table)
        c = g.tune_lookup(q, N, N, N)
        assert c is not None and g.choose_config(q, N, N, N) == c
        A, B = inputs.pair(q, N, N, N, cfg=243, idx=q)
        C = product(g, q, A, B)
        assert freivalds(q, A, B, C, seed=200 + q)
    finally:
        g.tune_clear()
