"""The Strassen-Winograd schedule of gfq_sw.h (host build), checked on the CPU.

The tables are read from a host program that includes the library's header; the test
computes the seven products and the merge with numpy over small prime fields, on ragged
shapes with the header's split rule (zero-padded second halves), and compares the result
with the definition of the matrix product.  Two levels are checked by recursion.
"""
import os
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def sched(tmp_path_factory):
    exe = str(tmp_path_factory.mktemp("sw") / "sw_host_check")
    subprocess.check_call(["g++", "-O1", "-std=c++14", "-Wall", "-I",
                           os.path.join(ROOT, "paper_0901_1413_amd", "csrc"),
                           os.path.join(ROOT, "tests", "sw_host_check.cpp"), "-o", exe])
    rows = [l.split() for l in subprocess.check_output([exe], text=True).splitlines()]
    A = np.array([[int(x) for x in r[2:]] for r in rows if r[0] == "A"])
    B = np.array([[int(x) for x in r[2:]] for r in rows if r[0] == "B"])
    C = np.array([[int(x) for x in r[2:]] for r in rows if r[0] == "C"])
    half = {int(r[1]): (int(r[2]), int(r[3])) for r in rows if r[0] == "half"}
    return A, B, C, half


def quadrants(X, hr, hc):
    """X split at (hr, hc), second halves zero-padded to (hr, hc)."""
    P = np.zeros((2 * hr, 2 * hc), dtype=np.int64)
    P[:X.shape[0], :X.shape[1]] = X
    return [P[:hr, :hc], P[:hr, hc:], P[hr:, :hc], P[hr:, hc:]]


def sw_product(sched, X, Y, p, levels):
    SA, SB, SC, half = sched
    if levels == 0:
        return (X @ Y) % p
    m, l = X.shape
    n = Y.shape[1]
    hm, hl, hn = half[m][0], half[l][1], half[n][1]
    QA, QB = quadrants(X, hm, hl), quadrants(Y, hl, hn)
    prods = []
    for c in range(7):
        a = sum(SA[c][j] * QA[j] for j in range(4)) % p
        b = sum(SB[c][j] * QB[j] for j in range(4)) % p
        prods.append(sw_product(sched, a, b, p, levels - 1))
    Cq = [sum(SC[j][c] * prods[c] for c in range(7)) % p for j in range(4)]
    full = np.block([[Cq[0], Cq[1]], [Cq[2], Cq[3]]])
    return full[:m, :n]


def test_half_rule(sched):
    half = sched[3]
    for d, (hr, hc) in half.items():
        assert hr == (d + 1) // 2
        assert hc % 32 == 0 and 2 * hc >= d and hc - 32 < (d + 1) // 2


@pytest.mark.parametrize("p", [2, 3, 5, 7])
@pytest.mark.parametrize("shape", [(2, 2, 2), (1, 1, 1), (5, 7, 3), (33, 65, 40), (64, 64, 64), (70, 100, 129)])
def test_one_level(sched, p, shape):
    m, l, n = shape
    rng = np.random.default_rng(m * 1000 + l * 10 + n + p)
    X, Y = rng.integers(0, p, (m, l)), rng.integers(0, p, (l, n))
    assert np.array_equal(sw_product(sched, X, Y, p, 1), (X @ Y) % p)


@pytest.mark.parametrize("p", [3, 5])
def test_two_levels(sched, p):
    rng = np.random.default_rng(p)
    X, Y = rng.integers(0, p, (90, 130)), rng.integers(0, p, (130, 70))
    assert np.array_equal(sw_product(sched, X, Y, p, 2), (X @ Y) % p)


def test_seven_products(sched):
    SA, SB, SC, _ = sched
    assert SA.shape == (7, 4) and SB.shape == (7, 4) and SC.shape == (4, 7)
    # every product is used, and each coefficient is -1, 0 or 1
    assert (np.abs(SC).sum(axis=0) > 0).all()
    assert set(np.unique(np.concatenate([SA.ravel(), SB.ravel(), SC.ravel()]))) <= {-1, 0, 1}
