"""Pins for the CPU oracle, each independent of the oracle's own loop.

* F_p products against numpy's int64 matrix product reduced mod p (a library routine).
* GF(4) products against the paper's matrix-level Karatsuba identity (Section 4.3) built
  from numpy products over F_2, and against the hand-derived multiplication table.
* GF(8) products against the paper's six-product trinomial formula (Section 4.3) built
  from numpy products over F_2 and reduced by x^3 + x + 1, and against a multiplication
  table derived by hand from the powers of x; field axioms on that table.
* F_9 = F_3[i]/(i^2 + 1) products against matrix-level Karatsuba over F_3 (Section 4.3:
  three numpy products mod 3), against a hand-derived table, and on the subfield F_3.
* Exhaustive tiny inputs: every 2x2 by 2x2 pair over F_3, every 1x2 by 2x1 pair over
  F_5, F_7, GF(4), GF(8) and F_9.
* Invariants of matrix multiplication: identity, zero, associativity, both distributive
  laws, transpose, scalars, and the additive-basis split of Section 2.
* Packed encodings against the paper's printed element codes (Sections 4.1-4.3).
"""
import itertools
import os

import numpy as np
import pytest

import oracle
from paper_0901_1413_amd import inputs

GOLD = os.path.join(os.path.dirname(__file__), "golden")
FIELDS = (3, 4, 5, 7, 8, 9)


def np_fp(q, A, B):
    return ((A.astype(np.int64) @ B.astype(np.int64)) % q).astype(np.uint8)


def gf4_karatsuba(A, B):
    """AB = (A0B0 + A1B1) + x((A0+A1)(B0+B1) + A0B0) over F_2 (Section 4.3)."""
    A0, A1 = (A & 1).astype(np.int64), (A >> 1).astype(np.int64)
    B0, B1 = (B & 1).astype(np.int64), (B >> 1).astype(np.int64)
    P00 = (A0 @ B0) % 2
    P11 = (A1 @ B1) % 2
    Pss = (((A0 + A1) % 2) @ ((B0 + B1) % 2)) % 2
    c0 = (P00 + P11) % 2
    c1 = (Pss + P00) % 2
    return (c0 + 2 * c1).astype(np.uint8)


def gf8_trinomial(A, B):
    """Six F_2 products by the trinomial formula of Section 4.3, then reduction.

    With a = a0 + a1 x + a2 x^2 (and b alike) the product coefficients are
    c0 = a0b0, c1 = (a0+a1)(b0+b1) - a0b0 - a1b1, c2 = (a0+a2)(b0+b2) - a0b0 - a2b2 + a1b1,
    c3 = (a1+a2)(b1+b2) - a1b1 - a2b2, c4 = a2b2; modulo x^3 + x + 1, x^3 = x + 1 and
    x^4 = x^2 + x fold c3 into c0 and c1 and c4 into c1 and c2."""
    a = [((A >> d) & 1).astype(np.int64) for d in range(3)]
    b = [((B >> d) & 1).astype(np.int64) for d in range(3)]
    mul = lambda X, Y: (X @ Y) % 2
    P = {(i, i): mul(a[i], b[i]) for i in range(3)}
    for i, j in ((0, 1), (0, 2), (1, 2)):
        P[i, j] = mul((a[i] + a[j]) % 2, (b[i] + b[j]) % 2)
    c0 = P[0, 0]
    c1 = P[0, 1] - P[0, 0] - P[1, 1]
    c2 = P[0, 2] - P[0, 0] - P[2, 2] + P[1, 1]
    c3 = P[1, 2] - P[1, 1] - P[2, 2]
    c4 = P[2, 2]
    r0, r1, r2 = (c0 + c3) % 2, (c1 + c3 + c4) % 2, (c2 + c4) % 2
    return (r0 + 2 * r1 + 4 * r2).astype(np.uint8)


def f9_karatsuba(A, B):
    """A = A0 + i A1, B = B0 + i B1 over F_3 with i^2 = -1 (Section 4.3, matrix-level):
    AB = (A0B0 - A1B1) + i((A0+A1)(B0+B1) - A0B0 - A1B1), three F_3 products."""
    A0, A1 = (A % 3).astype(np.int64), (A // 3).astype(np.int64)
    B0, B1 = (B % 3).astype(np.int64), (B // 3).astype(np.int64)
    P00, P11 = A0 @ B0, A1 @ B1
    Pss = (A0 + A1) @ (B0 + B1)
    re, im = (P00 - P11) % 3, (Pss - P00 - P11) % 3
    return (re + 3 * im).astype(np.uint8)


def reference(q, A, B):
    if q == 4:
        return gf4_karatsuba(A, B)
    if q == 8:
        return gf8_trinomial(A, B)
    if q == 9:
        return f9_karatsuba(A, B)
    return np_fp(q, A, B)


def f9_add(X, Y):
    X, Y = np.asarray(X, dtype=np.int64), np.asarray(Y, dtype=np.int64)
    return ((X % 3 + Y % 3) % 3 + 3 * ((X // 3 + Y // 3) % 3)).astype(np.uint8)


def field_add(q):
    if q in (4, 8):
        return lambda X, Y: X ^ Y
    if q == 9:
        return f9_add
    return lambda X, Y: ((X.astype(int) + Y) % q).astype(np.uint8)


def read_table(name):
    rows = [l.split() for l in open(os.path.join(GOLD, name)) if l.strip() and not l.startswith("#")]
    return np.array(rows, dtype=np.uint8)


def gf4_table():
    return read_table("gf4_mul.txt")


def gf8_table():
    return read_table("gf8_mul.txt")


def table_of(q):
    return {4: gf4_table, 8: gf8_table, 9: lambda: read_table("f9_mul.txt")}[q]()


@pytest.mark.parametrize("q", FIELDS)
@pytest.mark.parametrize("shape", [(1, 1, 1), (3, 5, 7), (17, 33, 65), (64, 129, 31), (100, 250, 90)])
def test_random_against_library_route(q, shape):
    m, l, n = shape
    A, B = inputs.pair(q, m, l, n, cfg=101, idx=hash(shape) % 1000)
    assert np.array_equal(oracle.matmul(q, A, B), reference(q, A, B))


@pytest.mark.parametrize("q", FIELDS)
def test_sparse_against_library_route(q):
    A, B = inputs.pair(q, 80, 300, 70, cfg=102, density=0.1)
    assert np.array_equal(oracle.matmul(q, A, B), reference(q, A, B))


def test_gf4_multiplication_table():
    T = gf4_table()
    for a in range(4):
        for b in range(4):
            A = np.array([[a]], np.uint8)
            B = np.array([[b]], np.uint8)
            assert oracle.matmul(4, A, B)[0, 0] == T[a, b], (a, b)
    # the Karatsuba route agrees with the table too, so the two pins pin each other
    for a in range(4):
        for b in range(4):
            assert gf4_karatsuba(np.array([[a]], np.uint8), np.array([[b]], np.uint8))[0, 0] == T[a, b]


def test_gf8_multiplication_table():
    T = gf8_table()
    for a in range(8):
        for b in range(8):
            A = np.array([[a]], np.uint8)
            B = np.array([[b]], np.uint8)
            assert oracle.matmul(8, A, B)[0, 0] == T[a, b], (a, b)
            assert gf8_trinomial(A, B)[0, 0] == T[a, b], (a, b)


@pytest.mark.parametrize("q,gen", [(4, 2), (8, 2), (9, 4)])
def test_extension_field_axioms(q, gen):
    """The golden tables describe a field: commutative, associative, distributive over the
    field's addition, 1 is the identity and every nonzero element has an inverse (rows are
    permutations); the multiplicative group is cyclic of order q - 1 (generator x for
    GF(4), GF(8); 1 + i for F_9, as i alone has order 4)."""
    T = table_of(q).astype(int)
    add = field_add(q)
    r = range(q)
    assert (T == T.T).all()
    assert list(T[1]) == list(r) and not T[0].any()
    for a, b, c in itertools.product(r, repeat=3):
        assert T[T[a, b], c] == T[a, T[b, c]]
        assert T[a, int(add(b, c))] == int(add(T[a, b], T[a, c]))
    for a in range(1, q):
        assert sorted(T[a, 1:]) == list(range(1, q))
    p, seen = 1, []
    for _ in range(q - 1):
        seen.append(p)
        p = T[p, gen]
    assert p == 1 and sorted(seen) == list(range(1, q))


def test_f9_table_and_subfield():
    T = table_of(9)
    for a in range(9):
        for b in range(9):
            A, B = np.array([[a]], np.uint8), np.array([[b]], np.uint8)
            assert oracle.matmul(9, A, B)[0, 0] == T[a, b], (a, b)
            assert f9_karatsuba(A, B)[0, 0] == T[a, b], (a, b)
    # i^2 = -1, and on F_3 (a1 = 0) the product is the F_3 product
    assert T[3, 3] == 2
    A, B = inputs.pair(3, 31, 70, 45, cfg=106)
    assert np.array_equal(oracle.matmul(9, A, B), oracle.matmul(3, A, B))
    # on i F_3 x i F_3 the product is minus the F_3 product of the coefficients
    C3 = oracle.matmul(3, A, B)
    assert np.array_equal(oracle.matmul(9, 3 * A, 3 * B), (3 - C3) % 3)


def test_exhaustive_f3_2x2():
    vals = np.array(list(itertools.product(range(3), repeat=4)), dtype=np.uint8).reshape(-1, 2, 2)
    Aall = np.repeat(vals, len(vals), axis=0)
    Ball = np.tile(vals, (len(vals), 1, 1))
    # stack all 6561 products block-diagonally: row block i of A times column block i of B
    N = len(Aall)
    got = np.empty((N, 2, 2), np.uint8)
    # one oracle call per left matrix with all right matrices side by side
    Bcat = np.concatenate(list(vals), axis=1)              # 2 x (81*2)
    for i, a in enumerate(vals):
        C = oracle.matmul(3, a, Bcat)                        # 2 x 162
        got[i * 81:(i + 1) * 81] = C.reshape(2, 81, 2).transpose(1, 0, 2)
    want = (np.einsum("nij,njk->nik", Aall.astype(np.int64), Ball.astype(np.int64)) % 3).astype(np.uint8)
    assert np.array_equal(got, want)


@pytest.mark.parametrize("q", [4, 5, 7, 8, 9])
def test_exhaustive_1x2_by_2x1(q):
    T = table_of(q) if q in (4, 8, 9) else None
    add = field_add(q)
    for a0, a1, b0, b1 in itertools.product(range(q), repeat=4):
        A = np.array([[a0, a1]], np.uint8)
        B = np.array([[b0], [b1]], np.uint8)
        got = oracle.matmul(q, A, B)[0, 0]
        if q in (4, 8, 9):
            want = add(T[a0, b0], T[a1, b1])
        else:
            want = (a0 * b0 + a1 * b1) % q
        assert got == want, (a0, a1, b0, b1)


@pytest.mark.parametrize("q", FIELDS)
def test_invariants(q):
    m, l, n, p = 37, 45, 29, 21
    A = inputs.matrix(q, m, l, 103, q, 0)
    B = inputs.matrix(q, l, n, 103, q, 1)
    B2 = inputs.matrix(q, l, n, 103, q, 3)
    D = inputs.matrix(q, n, p, 103, q, 4)
    add = field_add(q)
    I_l = np.eye(l, dtype=np.uint8)
    mm = lambda X, Y: oracle.matmul(q, X, Y)
    assert np.array_equal(mm(A, I_l), A)
    assert np.array_equal(mm(I_l, B), B)
    assert not mm(np.zeros((m, l), np.uint8), B).any()
    assert np.array_equal(mm(mm(A, B), D), mm(A, mm(B, D)))
    assert np.array_equal(mm(A, add(B, B2)), add(mm(A, B), mm(A, B2)))
    A2 = inputs.matrix(q, m, l, 103, q, 5)
    assert np.array_equal(mm(add(A, A2), B), add(mm(A, B), mm(A2, B)))
    assert np.array_equal(mm(A, B).T, mm(B.T.copy(), A.T.copy()))
    for c in range(1, q):
        cI = (c * np.eye(m)).astype(np.uint8)
        assert np.array_equal(mm(mm(cI, A), B), mm(cI, mm(A, B)))


@pytest.mark.parametrize("q", FIELDS)
def test_additive_basis_split(q):
    """Section 2: a = sum_d alpha_d phi_d(a) gives AB = sum_d alpha_d (Phi_d(A) B) with
    Phi_d(A) the 0/1 matrix of phi_d.  F_3 uses {1, -1} with phi_0 = [a = 1],
    phi_1 = [a = -1]; F_5, F_7 use {1, 2, 4} with binary digits; GF(4) uses {1, x} and
    GF(8) {1, x, x^2} (the integers 1, 2, 4 encode those elements); F_9 uses the products
    of {1, i} with the F_3 basis, {1, -1, i, -i} (codes 1, 2, 3, 6), phi = [a0 = 1],
    [a0 = -1], [a1 = 1], [a1 = -1]."""
    A, B = inputs.pair(q, 23, 61, 19, cfg=104)
    if q == 3:
        alphas, phis = [1, 2], [(A == 1), (A == 2)]
    elif q == 4:
        alphas, phis = [1, 2], [(A & 1), (A >> 1) & 1]
    elif q == 9:
        alphas, phis = [1, 2, 3, 6], [(A % 3 == 1), (A % 3 == 2), (A // 3 == 1), (A // 3 == 2)]
    else:
        alphas, phis = [1, 2, 4], [(A >> d) & 1 for d in range(3)]
    acc = np.zeros((23, 19), np.uint8)
    for alpha, phi in zip(alphas, phis):
        part = oracle.matmul(q, phi.astype(np.uint8), B)
        scaled = oracle.matmul(q, part, (alpha * np.eye(19)).astype(np.uint8))   # part * alpha
        acc = field_add(q)(acc, scaled)
    assert np.array_equal(acc, oracle.matmul(q, A, B))


def test_degenerate_shapes():
    for q in FIELDS:
        assert oracle.matmul(q, np.zeros((0, 5), np.uint8), np.zeros((5, 4), np.uint8)).shape == (0, 4)
        assert oracle.matmul(q, np.zeros((3, 5), np.uint8), np.zeros((5, 0), np.uint8)).shape == (3, 0)
        C = oracle.matmul(q, np.zeros((3, 0), np.uint8), np.zeros((0, 4), np.uint8))
        assert C.shape == (3, 4) and not C.any()


def test_rejects_bad_field_and_shape():
    with pytest.raises(ValueError):
        oracle.matmul(11, np.zeros((2, 2), np.uint8), np.zeros((2, 2), np.uint8))
    with pytest.raises(ValueError):
        oracle.matmul(3, np.zeros((2, 3), np.uint8), np.zeros((2, 2), np.uint8))


def test_encodings_golden():
    for line in open(os.path.join(GOLD, "encodings.txt")):
        if not line.strip() or line.startswith("#"):
            continue
        q, v, *bits = map(int, line.split())
        planes = oracle.encode_planes(q, np.array([[v]], np.uint8))
        assert [int(p[0, 0]) for p in planes] == bits, (q, v)
        assert oracle.decode_planes(q, planes)[0, 0] == v


def test_packed_layout_by_hand():
    # F_7, one row of 200 elements: W = ceil(200/128)*4 = 8 words per plane, 3 planes.
    X = np.zeros((1, 200), np.uint8)
    X[0, 33] = 5          # binary 101: plane 0 and plane 2 carry bit 1 of word 1
    X[0, 199] = 2         # binary 010: plane 1, word 6, bit 7
    w = oracle.pack(7, X)
    assert w.shape == (1, 24)
    expect = np.zeros(24, np.uint32)
    expect[0 * 8 + 1] = 1 << 1
    expect[2 * 8 + 1] = 1 << 1
    expect[1 * 8 + 6] = 1 << 7
    assert np.array_equal(w[0], expect)
    # F_3: -1 sets both the unit plane and the sign plane; 1 only the unit plane
    Y = np.array([[2, 1, 0]], np.uint8)
    w3 = oracle.pack(3, Y)
    assert w3.shape == (1, 8) and w3[0, 0] == 0b11 and w3[0, 4] == 0b01
    assert oracle.packed_words(3, 128) == 8 and oracle.packed_words(5, 129) == 24


@pytest.mark.parametrize("q", FIELDS)
@pytest.mark.parametrize("cols", [1, 31, 32, 33, 127, 128, 129, 1000])
def test_pack_roundtrip_and_pad(q, cols):
    X = inputs.matrix(q, 3, cols, 105, cols, q)
    w = oracle.pack(q, X)
    assert np.array_equal(oracle.unpack(q, w, 3, cols), X)
    W = -(-cols // 128) * 4
    bits = np.unpackbits(w.reshape(3, oracle.planes(q), W).view(np.uint8), axis=2, bitorder="little")
    assert not bits[:, :, cols:].any()
