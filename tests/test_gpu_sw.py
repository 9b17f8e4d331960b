"""GPU parity of Strassen-Winograd products over the Four-Russians product (gfq_matmul_sw):
bit-exact against the oracle, and packed products byte-identical to gfq_matmul's."""
import numpy as np
import pytest

import oracle
from paper_0901_1413_amd import inputs

pytestmark = pytest.mark.gpu
FIELDS = (3, 4, 5, 7, 8, 9)


def dev(x):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def check_sw(g, q, A, B, levels, **kw):
    m, l = A.shape
    n = B.shape[1]
    Ap, Bp = g.pack(q, dev(A)), g.pack(q, dev(B))
    Cp = g.empty_packed(q, m, n)
    Cp.fill_(0xA5)
    g.matmul_sw(q, Ap, Bp, m, l, n, levels, out=Cp, **kw)
    C = g.unpack(q, Cp, m, n).cpu().numpy()
    want = oracle.matmul(q, A, B)
    assert np.array_equal(C, want), f"q={q} shape={A.shape}x{B.shape} levels={levels} kw={kw}"
    want_p = oracle.pack(q, want).view(np.uint8).reshape(-1)
    assert np.array_equal(Cp.cpu().numpy()[:want_p.size], want_p), "packed product differs from the oracle's encoding"


@pytest.mark.parametrize("q", FIELDS)
@pytest.mark.parametrize("levels", [1, 2])
@pytest.mark.parametrize("shape", [(1, 1, 1), (2, 2, 2), (5, 7, 3), (33, 65, 129), (300, 257, 131), (256, 512, 384)])
def test_sw_shapes(gfq_gpu, q, levels, shape):
    m, l, n = shape
    A, B = inputs.pair(q, m, l, n, cfg=230, idx=m + 3 * l + 7 * n + levels)
    check_sw(gfq_gpu, q, A, B, levels)


@pytest.mark.parametrize("q", [3, 5, 9])
@pytest.mark.parametrize("levels", [3, 4])
def test_sw_deep(gfq_gpu, q, levels):
    A, B = inputs.pair(q, 600, 700, 500, cfg=231, idx=levels)
    check_sw(gfq_gpu, q, A, B, levels)


@pytest.mark.parametrize("q", [5, 8])
@pytest.mark.parametrize("k", list(range(1, 11)))
def test_sw_leaf_every_k(gfq_gpu, q, k):
    A, B = inputs.pair(q, 200, 520, 300, cfg=232, idx=k)
    check_sw(gfq_gpu, q, A, B, 1, k=k)


@pytest.mark.parametrize("q", [3, 7])
@pytest.mark.parametrize("rows", [256, 512, 1024, 2048])
def test_sw_leaf_tiles(gfq_gpu, q, rows):
    A, B = inputs.pair(q, 1100, 300, 700, cfg=233, idx=rows)
    check_sw(gfq_gpu, q, A, B, 2, rows=rows)


def test_sw_gf4_karatsuba_leaves(gfq_gpu):
    g = gfq_gpu
    A, B = inputs.pair(4, 500, 400, 300, cfg=234)
    check_sw(g, 4, A, B, 2, variant=g.VARIANT_KARATSUBA)


def test_sw_sparse_and_identity(gfq_gpu):
    for q in FIELDS:
        A, B = inputs.pair(q, 300, 400, 200, cfg=235, idx=q, density=0.1)
        check_sw(gfq_gpu, q, A, B, 2)
        check_sw(gfq_gpu, q, np.eye(300, dtype=np.uint8), A, 1)


@pytest.mark.parametrize("q", [3, 5])
def test_sw_4096_equals_plain(gfq_gpu, q):
    """4096^3, two levels: the packed product equals the plain Four-Russians product byte for
    byte, and sampled rows equal the oracle."""
    import torch
    g = gfq_gpu
    N = 4096
    A, B = inputs.pair(q, N, N, N, cfg=236, idx=q)
    Ap, Bp = g.pack(q, dev(A)), g.pack(q, dev(B))
    plain = g.matmul(q, Ap, Bp, N, N, N)
    sw = g.matmul_sw(q, Ap, Bp, N, N, N, 2)
    assert torch.equal(plain, sw)
    C = g.unpack(q, sw, N, N)
    rows = np.arange(0, N, 127)
    assert np.array_equal(C[torch.from_numpy(rows).cuda()].cpu().numpy(), oracle.matmul(q, A[rows], B))


def test_sw_degenerate_and_validation(gfq_gpu):
    import torch
    g = gfq_gpu
    for q in FIELDS:
        C = g.empty_packed(q, 5, 40)
        C.fill_(0xAB)
        g.matmul_sw(q, g.empty_packed(q, 5, 0), g.empty_packed(q, 0, 40), 5, 0, 40, 2, out=C)
        g.sync()
        assert not C.cpu().numpy()[:g.packed_bytes(q, 5, 40)].any()
        g.matmul_sw(q, g.empty_packed(q, 0, 3), g.empty_packed(q, 3, 4), 0, 3, 4, 1)
    A = g.empty_packed(3, 64, 64)
    for bad in (-2, g.SW_MAX_LEVELS + 1):                   # -1 is SW_AUTO
        with pytest.raises(g.GfqError) as e:
            g.matmul_sw(3, A, A, 64, 64, 64, bad, out=g.empty_packed(3, 64, 64))
        assert e.value.status == -1
    with pytest.raises(g.GfqError) as e:
        g.matmul_sw(11, A, A, 64, 64, 64, 1, out=g.empty_packed(3, 64, 64))
    assert e.value.status == -2
    torch.cuda.synchronize()


def test_sw_levels_zero_is_plain(gfq_gpu):
    import torch
    g = gfq_gpu
    A, B = inputs.pair(7, 300, 200, 100, cfg=237)
    Ap, Bp = g.pack(7, dev(A)), g.pack(7, dev(B))
    assert torch.equal(g.matmul_sw(7, Ap, Bp, 300, 200, 100, 0), g.matmul(7, Ap, Bp, 300, 200, 100))


def test_sw_concurrent_streams(gfq_gpu):
    """The recursion's operand sums and products live in a workspace per (device, stream):
    products in flight on different streams must not share it."""
    import torch
    g = gfq_gpu
    q, m, l, n = 5, 900, 1000, 700
    pairs = [inputs.pair(q, m, l, n, cfg=238, idx=i) for i in range(4)]
    ops = [(g.pack(q, dev(A)), g.pack(q, dev(B))) for A, B in pairs]
    outs = [g.empty_packed(q, m, n) for _ in pairs]
    torch.cuda.synchronize()
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    for rep in range(3):
        for i, (Ap, Bp) in enumerate(ops):
            with torch.cuda.stream(streams[i % 2]):
                g.matmul_sw(q, Ap, Bp, m, l, n, 1 + (i + rep) % 2, out=outs[i])
    torch.cuda.synchronize()
    for i, (A, B) in enumerate(pairs):
        assert np.array_equal(g.unpack(q, outs[i], m, n).cpu().numpy(), oracle.matmul(q, A, B)), i


def test_sw_four_levels_with_slices(gfq_gpu):
    """Four levels give 2401 leaves; a leaf configuration with 64 slices of the inner
    dimension is cut down so that leaves x slices fit one grid (65535)."""
    g = gfq_gpu
    A, B = inputs.pair(3, 300, 9000, 200, cfg=239)
    check_sw(g, 3, A, B, 4, k=4)
    check_sw(g, 3, A, B, 4, k=4, rows=256, split=64)


def test_sw_ignores_pad_bits_of_inputs(gfq_gpu):
    """Every pad bit of packed A and B set: the recursion's quadrant splits read those words
    (A's pad columns only ever meet zero rows of B, B's land in C's masked columns)."""
    g = gfq_gpu
    for q in (3, 7, 9):
        m, l, n = 300, 333, 270
        A, B = inputs.pair(q, m, l, n, cfg=243, idx=q)
        Ap, Bp = oracle.pack(q, A), oracle.pack(q, B)

        def dirty(w, cols):
            w = w.copy().reshape(w.shape[0], oracle.planes(q), -1)
            bits = np.unpackbits(w.view(np.uint8), axis=2, bitorder="little")
            bits[:, :, cols:] = 1
            return np.packbits(bits, axis=2, bitorder="little").view("<u4").reshape(w.shape[0], -1)

        Ad, Bd = dirty(Ap, l), dirty(Bp, n)
        for levels in (1, 2):
            Cp = g.matmul_sw(q, dev(Ad.view(np.uint8).reshape(-1)), dev(Bd.view(np.uint8).reshape(-1)), m, l, n, levels)
            C = g.unpack(q, Cp, m, n).cpu().numpy()
            assert np.array_equal(C, oracle.matmul(q, A, B)), (q, levels)
            got = Cp.cpu().numpy()[:g.packed_bytes(q, m, n)]
            assert np.array_equal(got, oracle.pack(q, C).view(np.uint8).reshape(-1)), (q, levels)


def test_sw_auto_levels_from_the_tuner(gfq_gpu):
    """GFQ_SW_AUTO: levels from the tuner's cache for the size class (0 without an entry);
    the product is the same at every level."""
    import torch
    g = gfq_gpu
    q, N = 5, 2048
    A, B = inputs.pair(q, N, N, N, cfg=244)
    Ap, Bp = g.pack(q, dev(A)), g.pack(q, dev(B))
    plain = g.matmul(q, Ap, Bp, N, N, N)
    g.tune_clear()
    assert g.tune_sw_lookup(q, N, N, N) is None
    assert torch.equal(g.matmul_sw(q, Ap, Bp, N, N, N, g.SW_AUTO), plain)     # no entry: plain
    lev = g.tune_sw(q, N, N, N)
    assert 0 <= lev < g.SW_MAX_LEVELS and g.tune_sw_lookup(q, N, N, N) == lev
    assert torch.equal(g.matmul_sw(q, Ap, Bp, N, N, N, g.SW_AUTO), plain)
    g.tune_clear()
