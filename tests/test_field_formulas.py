"""Truth tables of the library's bitsliced field formulas (host build of gfq_field.h).

Every formula is run on every input representative and checked against the value it
must have: the residue of the integer it encodes (F_5, F_7: any 3-bit representative;
F_3: the three codes of Section 4.1), or the GF(4) rule x^2 = x + 1.
"""
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
F3_VAL = {(0, 0): 0, (1, 0): 1, (1, 1): 2}


@pytest.fixture(scope="module")
def table(tmp_path_factory):
    exe = str(tmp_path_factory.mktemp("field") / "field_host_check")
    subprocess.check_call(["g++", "-O2", "-std=c++14", "-Wall", "-I",
                           os.path.join(ROOT, "paper_0901_1413_amd", "csrc"),
                           os.path.join(ROOT, "tests", "field_host_check.cpp"), "-o", exe])
    out = subprocess.check_output([exe], text=True)
    return [l.split() for l in out.splitlines()]


def test_f3(table):
    rows = [r for r in table if r[0] == "f3"]
    assert len(rows) == 9
    for r in rows:
        xu, xs, yu, ys = map(int, r[1:5])
        add = (int(r[6]), int(r[7]))
        x, y = F3_VAL[(xu, xs)], F3_VAL[(yu, ys)]
        assert add in F3_VAL and F3_VAL[add] == (x + y) % 3, r
    for r in (r for r in table if r[0] == "f3neg"):
        x = F3_VAL[(int(r[1]), int(r[2]))]
        assert F3_VAL[(int(r[3]), int(r[4]))] == (-x) % 3


def test_f5_f7_binary(table):
    rows = [r for r in table if r[0] == "p3"]
    assert len(rows) == 64
    for r in rows:
        a, b, f7, f7s = int(r[1]), int(r[2]), int(r[4]), int(r[6])
        assert f7 % 7 == (a + b) % 7, r
        assert f7s % 7 == (a - b) % 7, r
    for r in (r for r in table if r[0] == "p1"):
        a = int(r[1])
        f7dbl, f7neg, f7red, f5neg, f5red = (int(r[i]) for i in (3, 5, 7, 9, 11))
        assert f7dbl % 7 == (2 * a) % 7
        assert f7neg % 7 == (-a) % 7
        assert f7red == a % 7                      # canonical in [0, 7)
        assert f5neg % 5 == (-a) % 5
        assert f5red == a % 5                      # canonical in [0, 5)


def test_gf4(table):
    mul = [[0, 0, 0, 0], [0, 1, 2, 3], [0, 2, 3, 1], [0, 3, 1, 2]]
    for r in (r for r in table if r[0] == "g4"):
        a, b, s, mx = map(int, (r[1], r[2], r[4], r[6]))
        assert s == a ^ b
        assert mx == mul[2][a]


def gf8_table():
    path = os.path.join(ROOT, "tests", "golden", "gf8_mul.txt")
    rows = [l.split() for l in open(path) if l.strip() and not l.startswith("#")]
    return [[int(x) for x in r] for r in rows]


def test_gf8(table):
    mul = gf8_table()
    rows = [r for r in table if r[0] == "g8"]
    assert len(rows) == 64
    for r in rows:
        a, b, s, m1, m2 = map(int, (r[1], r[2], r[4], r[6], r[8]))
        assert s == a ^ b
        assert m1 == mul[2][a] and m2 == mul[4][a]


def test_gf8_accumulate_step(table):
    mul = gf8_table()
    rows = [r for r in table if r[0] == "g8acc"]
    assert len(rows) == 8 ** 4
    for r in rows:
        c, t, u, v, out = map(int, r[1:])
        assert out == c ^ t ^ mul[2][u] ^ mul[4][v], r


def test_f3_binary_working_form(table):
    for r in (r for r in table if r[0] == "f3b"):
        a, b, add, sub, c0, c1 = int(r[1]), int(r[2]), int(r[4]), int(r[6]), int(r[8]), int(r[9])
        assert add % 3 == (a + b) % 3 and add < 4
        assert sub % 3 == (a - b) % 3 and sub < 4
        assert F3_VAL[(c0, c1)] == a % 3
    for r in (r for r in table if r[0] == "f3tobin"):
        assert int(r[3]) == F3_VAL[(int(r[1]), int(r[2]))]


def test_carry_save_steps(table):
    rows = [r for r in table if r[0] == "csa"]
    assert len(rows) == 16 ** 3
    for r in rows:
        S, K, X, s4, k4, s3, k3, s2, k2, n2, m2 = map(int, r[1:])
        assert (s4 + k4) % 15 == (S + K + X) % 15
        assert (s3 + k3) % 7 == ((S & 7) + (K & 7) + (X & 7)) % 7
        assert (s2 + k2) % 3 == ((S & 3) + (K & 3) + (X & 3)) % 3
        assert (n2 + m2) % 3 == ((S & 3) + (K & 3) - (X & 3)) % 3


def test_f3_slab_step(table):
    """One F_3 slab as the product kernel accumulates it (binary residues modulo 3): acc + t
    - v for every residue code acc, t, v in 0..3.  And the exchange of a lane's planes: a
    lane that reads t and v with their planes exchanged, starting from the exchanged
    accumulator, ends at the exchange of the true result (exchanging b0 and b1 of b0 + 2 b1
    multiplies it by 2 = -1 mod 3), which is what lets one row of each read pass gather
    from the opposite half of the banks and be turned back at the store."""
    rows = {tuple(map(int, r[1:4])): int(r[4]) for r in table if r[0] == "f3acc"}
    assert len(rows) == 4 * 4 * 4
    sw = lambda x: (x >> 1) | ((x & 1) << 1)
    for x in range(4):
        assert sw(x) % 3 == (-x) % 3
    for (a, t, v), r in rows.items():
        assert r % 3 == (a + t - v) % 3, (a, t, v, r)
        assert sw(rows[(sw(a), sw(t), sw(v))]) % 3 == r % 3, (a, t, v)


def test_f5_eight_instruction_add_sub(table):
    """The F_5 table addition and subtraction of eight three-input instructions give a + b and
    a - b (mod 5) for every pair of 3-bit representatives."""
    rows = [r for r in table if r[0] == "f5add8"]
    assert len(rows) == 64
    for r in rows:
        a, b, s, d = map(int, r[1:])
        assert s % 5 == (a + b) % 5 and d % 5 == (a - b) % 5, r


def test_f5_slab_step(table):
    """One slab of the F_5 accumulator (value a + b + 2c modulo 5): the new value is
    a + b + 2c + t + 2v + 4w + 2 (mod 5) for every state and every 3-bit representative of
    the three table rows; the starting value cancels the constant 2 per slab:
    init(n) + 2n = 0 (mod 5); and the final value a + b + 2c is its own canonical code."""
    rows = [r for r in table if r[0] == "f5slab"]
    assert len(rows) == 8 * 8 * 8 * 8
    for r in rows:
        a, b, c, t, v, w, out, _ = map(int, r[1:])
        a2, b2, c2 = out & 1, (out >> 1) & 1, out >> 2
        assert (a2 + b2 + 2 * c2) % 5 == (a + b + 2 * c + t + 2 * v + 4 * w + 2) % 5, r
    inits = [r for r in table if r[0] == "f5init"]
    assert len(inits) == 40
    for r in inits:
        n, a, b, c, full = map(int, r[1:])
        assert (a + b + 2 * c + 2 * n) % 5 == 0 and full == 1, r
    vals = [r for r in table if r[0] == "f5val"]
    assert len(vals) == 8
    for r in vals:
        st, z = map(int, r[1:])
        assert z == (st & 1) + ((st >> 1) & 1) + 2 * (st >> 2), r


def test_f3_binary_add_is_shortest(tmp_path):
    """The F_3 table addition (f3b_add) takes four three-input instructions; the committed
    exhaustive search shows that no program of three or fewer exists and checks the
    four-gate program."""
    exe = str(tmp_path / "f3b_add_search")
    subprocess.check_call(["g++", "-O2", "-std=c++17",
                           os.path.join(ROOT, "paper_0901_1413_amd", "search", "f3b_add_search.cpp"), "-o", exe])
    out = subprocess.run([exe], capture_output=True, text=True, timeout=300)
    assert out.returncode == 0, out.stdout + out.stderr
    lines = out.stdout.splitlines()
    for L in (1, 2, 3):
        assert f"length {L}: 0 programs" in lines, out.stdout
    assert "four-gate program: correct" in lines


def test_column_schedule_search():
    """The column-count model behind the accumulator states and the F_5 table addition:
    F_3's slab step needs 8 instructions and fits a 3-bit state, F_7's 18 and a 4-bit state
    (three bits cannot close the cycle), F_5's 20 and a 3-bit state, and the F_5 table addition
    and subtraction 8 each."""
    import importlib.util
    path = os.path.join(ROOT, "paper_0901_1413_amd", "search", "column_schedules.py")
    spec = importlib.util.spec_from_file_location("column_schedules", path)
    cs = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(cs)
    acc = cs.accumulate()
    assert acc["F_3"][:2] == (8, 3) and acc["F_7"][:2] == (18, 4)
    assert cs.f5_accumulate()[:2] == (20, 3)          # nine full adders and a half adder
    assert cs.f5add() == {"add": 8, "sub": 8}


def test_gf4_exchanged_reads_identity():
    """The GF(4) kernel's exchanged reads, checked with the oracle's GF(4) arithmetic (elements
    c0 + c1 x as the integers c0 + 2 c1, products by 1 x 1 oracle products): exchanging the two
    planes of t is x t^2; a row that reads both table rows exchanged and in exchanged order adds
    swap(T1) + x swap(T0) = L(T0 + x T1) with L(a) = x^2 a^2; L is additive and its own inverse,
    and L(c0 + c1 x) = c0 + (c0 + c1) x, the one masked XOR applied before the store."""
    import numpy as np

    import oracle

    def mul(a, b):
        return int(oracle.matmul(4, np.array([[a]], dtype=np.uint8), np.array([[b]], dtype=np.uint8))[0, 0])

    X = 2
    swap = lambda a: (a >> 1) | ((a & 1) << 1)
    L = lambda a: mul(mul(X, X), mul(a, a))
    for a in range(4):
        assert swap(a) == mul(X, mul(a, a))
        assert L(L(a)) == a
        c0, c1 = a & 1, a >> 1
        assert L(a) == c0 | ((c0 ^ c1) << 1)
        for b in range(4):
            assert L(a ^ b) == L(a) ^ L(b)                  # additive (addition is XOR)
    for t0 in range(4):
        for t1 in range(4):
            assert swap(t1) ^ mul(X, swap(t0)) == L(t0 ^ mul(X, t1))


def test_f7_doubled_copy_reads():
    """F_7's doubled-copy table layout: an entry t = (t0, t1, t2) is stored as the slots
    (t2, t0, t1, t2); the first row of a read pass reads slots 1, 2, 3 (t itself), the second
    slots 0, 1, 2, which is 2t (mod 7) for every 3-bit representative, so that row accumulates
    2C; its canonical result times 4 is the rotation (c0, c1, c2) -> (c1, c2, c0), which keeps
    canonical values canonical."""
    val = lambda b: b[0] + 2 * b[1] + 4 * b[2]
    for v in range(8):
        t = (v & 1, (v >> 1) & 1, v >> 2)
        slots = (t[2], t[0], t[1], t[2])
        assert slots[1:4] == t
        assert val(slots[0:3]) % 7 == (2 * val(t)) % 7
    for C in range(7):                       # the second row finishes with 2C, canonical
        c = (2 * C) % 7
        b = (c & 1, (c >> 1) & 1, c >> 2)
        r = (b[1], b[2], b[0])
        assert val(r) == C


def test_gf8_front_slot_reads():
    """GF(8)'s front-slot table layout, checked with the oracle's GF(8) arithmetic (elements
    c0 + c1 x + c2 x^2 as the integers c0 + 2 c1 + 4 c2): an entry t is stored as the slots
    (t0 + t2, t1, t2, t0); the first row of a read pass reads planes 0, 1, 2 from slots 3, 1, 2
    (t itself), the second from slots 2, 0, 1, which is x t; that row finishes with x C, and
    (c0, c1, c2) -> (c0 + c1, c2, c0) is multiplication by x^6 = x^-1, which gives C back."""
    import numpy as np

    import oracle

    def mul(a, b):
        return int(oracle.matmul(8, np.array([[a]], dtype=np.uint8), np.array([[b]], dtype=np.uint8))[0, 0])

    X = 2
    bits = lambda v: (v & 1, (v >> 1) & 1, v >> 2)
    num = lambda b: b[0] | (b[1] << 1) | (b[2] << 2)
    for v in range(8):
        t = bits(v)
        slots = (t[0] ^ t[2], t[1], t[2], t[0])
        assert num((slots[3], slots[1], slots[2])) == v
        assert num((slots[2], slots[0], slots[1])) == mul(X, v)
    for C in range(8):
        c = bits(mul(X, C))
        assert num((c[0] ^ c[1], c[2], c[0])) == C
