"""GPU parity: the HIP library, called through its C ABI, against the CPU oracle.

All comparisons are bit-exact (integer and boolean arithmetic only): unpacked products
element by element, packed products byte by byte against the oracle's encoding of its
own product, and packed operands against the oracle's encoder.
"""
import numpy as np
import pytest

import oracle
from paper_0901_1413_amd import inputs

pytestmark = pytest.mark.gpu
FIELDS = (3, 4, 5, 7, 8, 9)


def dev(x):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def run(g, q, A, B, **kw):
    m, l = A.shape
    n = B.shape[1]
    Ap, Bp = g.pack(q, dev(A)), g.pack(q, dev(B))
    Cp = g.matmul(q, Ap, Bp, m, l, n, **kw)
    C = g.unpack(q, Cp, m, n)
    g.sync()
    return C.cpu().numpy(), Cp.cpu().numpy()


def check(g, q, A, B, **kw):
    C, Cp = run(g, q, A, B, **kw)
    want = oracle.matmul(q, A, B)
    assert np.array_equal(C, want), f"q={q} shape={A.shape}x{B.shape} kw={kw}"
    want_p = oracle.pack(q, want).view(np.uint8).reshape(-1)
    assert np.array_equal(Cp[:want_p.size], want_p), "packed product differs from the oracle's encoding"


@pytest.mark.parametrize("q", FIELDS)
@pytest.mark.parametrize("cols", [1, 31, 32, 33, 63, 64, 65, 127, 128, 129, 1000])
def test_pack_matches_oracle_encoding(gfq_gpu, q, cols):
    X = inputs.matrix(q, 7, cols, 201, cols, q)
    P = gfq_gpu.pack(q, dev(X))
    got = P.cpu().numpy()[:gfq_gpu.packed_bytes(q, 7, cols)]
    assert np.array_equal(got, oracle.pack(q, X).view(np.uint8).reshape(-1))
    back = gfq_gpu.unpack(q, P, 7, cols).cpu().numpy()
    assert np.array_equal(back, X)


@pytest.mark.parametrize("q", FIELDS)
def test_pack_reduces_integers(gfq_gpu, q):
    X = np.arange(256, dtype=np.uint8).reshape(2, 128)
    got = gfq_gpu.unpack(q, gfq_gpu.pack(q, dev(X)), 2, 128).cpu().numpy()
    want = {4: X & 3, 8: X & 7}.get(q, X % q)      # GF(4), GF(8): the low coefficient bits
    assert np.array_equal(got, want.astype(np.uint8))


@pytest.mark.parametrize("q", FIELDS)
@pytest.mark.parametrize("shape", [(1, 1, 1), (1, 300, 1), (5, 7, 3), (33, 65, 129), (130, 259, 1057),
                                   (300, 1000, 70), (64, 128, 2048), (257, 33, 4099)])
def test_matmul_default_config(gfq_gpu, q, shape):
    m, l, n = shape
    A, B = inputs.pair(q, m, l, n, cfg=202, idx=m * 7 + n)
    check(gfq_gpu, q, A, B)


@pytest.mark.parametrize("q", FIELDS)
@pytest.mark.parametrize("k", list(range(1, 11)))
def test_matmul_every_k(gfq_gpu, q, k):
    A, B = inputs.pair(q, 97, 301, 1100, cfg=203, idx=k)
    check(gfq_gpu, q, A, B, k=k)


@pytest.mark.parametrize("q", FIELDS)
@pytest.mark.parametrize("rows,split", [(256, 1), (512, 1), (1024, 1), (2048, 1), (256, 3), (512, 7), (1024, 64)])
def test_matmul_tiles_and_splits(gfq_gpu, q, rows, split):
    A, B = inputs.pair(q, 600, 700, 300, cfg=204, idx=rows + split)
    check(gfq_gpu, q, A, B, rows=rows, split=split)


@pytest.mark.parametrize("q", FIELDS)
def test_matmul_sparse(gfq_gpu, q):
    A, B = inputs.pair(q, 200, 500, 400, cfg=205, density=0.1)
    check(gfq_gpu, q, A, B)


@pytest.mark.parametrize("q", FIELDS)
def test_degenerate(gfq_gpu, q):
    import torch
    g = gfq_gpu
    # l == 0 gives a zero product; m == 0 / n == 0 are no-ops
    C = g.empty_packed(q, 5, 40)
    C.fill_(0xAB)
    g.matmul(q, g.empty_packed(q, 5, 0), g.empty_packed(q, 0, 40), 5, 0, 40, out=C)
    g.sync()
    assert not C.cpu().numpy()[:g.packed_bytes(q, 5, 40)].any()
    g.matmul(q, g.empty_packed(q, 0, 3), g.empty_packed(q, 3, 4), 0, 3, 4)
    g.sync()
    # all-zero and identity operands
    I = np.eye(70, dtype=np.uint8)
    A = inputs.matrix(q, 70, 70, 206, q)
    check(g, q, A, I)
    check(g, q, I, A)
    check(g, q, np.zeros((10, 70), np.uint8), A)
    assert torch.cuda.is_available()


def test_pad_bits_of_inputs_are_ignored(gfq_gpu):
    """Set every pad bit of packed A and B; the product must not change."""
    g = gfq_gpu
    for q in FIELDS:
        m, l, n = 40, 45, 50
        A, B = inputs.pair(q, m, l, n, cfg=207, idx=q)
        Ap, Bp = oracle.pack(q, A), oracle.pack(q, B)
        def dirty(w, cols):
            w = w.copy().reshape(w.shape[0], oracle.planes(q), -1)
            bits = np.unpackbits(w.view(np.uint8), axis=2, bitorder="little")
            bits[:, :, cols:] = 1          # for F_3 every pad element becomes the code of -1
            return np.packbits(bits, axis=2, bitorder="little").view("<u4").reshape(w.shape[0], -1)
        Ad, Bd = dirty(Ap, l), dirty(Bp, n)
        Cp = g.matmul(q, dev(Ad.view(np.uint8).reshape(-1)), dev(Bd.view(np.uint8).reshape(-1)), m, l, n)
        C = g.unpack(q, Cp, m, n).cpu().numpy()
        assert np.array_equal(C, oracle.matmul(q, A, B)), q
        got = Cp.cpu().numpy()[:g.packed_bytes(q, m, n)]
        assert np.array_equal(got, oracle.pack(q, C).view(np.uint8).reshape(-1)), q


def test_validation_errors(gfq_gpu):
    g = gfq_gpu
    import torch
    A = g.empty_packed(3, 8, 8)
    with pytest.raises(g.GfqError) as e:
        g.matmul(11, A, A, 8, 8, 8)
    assert e.value.status == -2
    with pytest.raises(g.GfqError) as e:
        g.matmul(3, A, A, 8, 8, 8, out=A)          # output aliases the inputs
    assert e.value.status == -6
    buf = torch.zeros(4096, dtype=torch.uint8, device="cuda")
    with pytest.raises(g.GfqError) as e:
        g.matmul(3, buf[1:], buf[1:], 8, 8, 8, out=torch.zeros(4096, dtype=torch.uint8, device="cuda")[4:])
    assert e.value.status == -5
    with pytest.raises(g.GfqError) as e:
        g.matmul(3, A, A, 8, 8, 8, k=11)
    assert e.value.status == -1


def test_c1_f3_512(gfq_gpu):
    """F_3, A and B 512 x 512 uniform: the whole product against the oracle."""
    A, B = inputs.pair(3, 512, 512, 512, cfg=1)
    check(gfq_gpu, 3, A, B)


@pytest.mark.parametrize("q", FIELDS)
def test_pack_unpack_strided_and_offset(gfq_gpu, q):
    """Leading dimensions above the column count and sources/destinations that are not
    16-byte aligned take the byte-wise path; aligned ones take the 128-bit path."""
    import torch
    g = gfq_gpu
    big = inputs.matrix(q, 37, 300, 208, q)
    for c0, cols in ((0, 256), (1, 255), (3, 129), (16, 64), (5, 33)):
        X = dev(big)[:, c0:c0 + cols]                 # ld = 300, offset c0
        P = g.pack(q, X)
        want = oracle.pack(q, big[:, c0:c0 + cols]).view(np.uint8).reshape(-1)
        assert np.array_equal(P.cpu().numpy()[:want.size], want), (c0, cols)
        out = torch.full((37, 320), 0xEE, dtype=torch.uint8, device="cuda")
        g.unpack(q, P, 37, cols, out=out[:, 7:7 + cols])
        o = out.cpu().numpy()
        assert np.array_equal(o[:, 7:7 + cols], big[:, c0:c0 + cols]), (c0, cols)
        assert (o[:, :7] == 0xEE).all() and (o[:, 7 + cols:] == 0xEE).all()   # nothing outside


def test_split_products_on_concurrent_streams(gfq_gpu):
    """Products whose inner dimension is split write partial sums to a workspace; products in
    flight on different streams must not share it."""
    import torch
    g = gfq_gpu
    q, m, l, n = 5, 700, 2000, 900
    pairs = [inputs.pair(q, m, l, n, cfg=0, idx=70 + i) for i in range(4)]
    dev = [(g.pack(q, torch.from_numpy(A).cuda()), g.pack(q, torch.from_numpy(B).cuda())) for A, B in pairs]
    outs = [g.empty_packed(q, m, n) for _ in pairs]
    torch.cuda.synchronize()
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    for rep in range(3):
        for i, (Ap, Bp) in enumerate(dev):
            with torch.cuda.stream(streams[i % 2]):
                g.matmul(q, Ap, Bp, m, l, n, out=outs[i], k=6, rows=256, split=8)
    torch.cuda.synchronize()
    for i, (A, B) in enumerate(pairs):
        assert np.array_equal(g.unpack(q, outs[i], m, n).cpu().numpy(), oracle.matmul(q, A, B)), i


def test_more_row_tiles_than_one_grid_holds(gfq_gpu):
    """A grid holds at most 65535 row tiles; a taller product is launched in pieces.  F_3 with
    256-row tiles and m = 65535 * 256 + 300 rows, checked on rows around the piece boundary."""
    import torch
    g = gfq_gpu
    q, l, n = 3, 32, 64
    m = 65535 * 256 + 300
    A, B = inputs.pair(q, m, l, n, cfg=0, idx=80)
    Ap, Bp = g.pack(q, torch.from_numpy(A).cuda()), g.pack(q, torch.from_numpy(B).cuda())
    Cp = g.empty_packed(q, m, n)
    g.matmul(q, Ap, Bp, m, l, n, out=Cp, k=6, rows=256, split=1)
    C = g.unpack(q, Cp, m, n)
    edge = 65535 * 256
    rows = np.concatenate([np.arange(0, 64), np.arange(edge - 300, edge + 300), np.arange(m - 64, m)])
    got = C[torch.from_numpy(rows).cuda()].cpu().numpy()
    assert np.array_equal(got, oracle.matmul(q, A[rows], B))


# The matrix-level routes (gfq_config.variant = VARIANT_KARATSUBA): GF(4) by Karatsuba over
# F_2, GF(8) by the trinomial formula over F_2, F_9 by Karatsuba over F_3.  Every
# configuration gives the oracle's product, byte for byte in packed form.
MATRIX_ROUTE_FIELDS = (4, 8, 9)


@pytest.mark.parametrize("q", MATRIX_ROUTE_FIELDS)
@pytest.mark.parametrize("shape", [(1, 1, 1), (5, 7, 3), (33, 65, 129), (130, 259, 1057), (257, 33, 4099),
                                   (600, 1000, 70)])
def test_matrix_route_shapes(gfq_gpu, q, shape):
    m, l, n = shape
    A, B = inputs.pair(q, m, l, n, cfg=210, idx=m * 7 + n)
    check(gfq_gpu, q, A, B, variant=gfq_gpu.VARIANT_KARATSUBA)


@pytest.mark.parametrize("q", MATRIX_ROUTE_FIELDS)
@pytest.mark.parametrize("k", list(range(1, 11)))
def test_matrix_route_every_k(gfq_gpu, q, k):
    A, B = inputs.pair(q, 97, 301, 1100, cfg=211, idx=k)
    if q in (8, 9) and k == 10:
        # six-plane tables: two of 2^10 entries do not fit LDS even at 16-byte super-rows
        with pytest.raises(gfq_gpu.GfqError) as e:
            check(gfq_gpu, q, A, B, k=k, variant=gfq_gpu.VARIANT_KARATSUBA)
        assert e.value.status == -1
        return
    check(gfq_gpu, q, A, B, k=k, variant=gfq_gpu.VARIANT_KARATSUBA)


@pytest.mark.parametrize("q", MATRIX_ROUTE_FIELDS)
@pytest.mark.parametrize("rows,split", [(256, 1), (512, 1), (1024, 1), (2048, 1), (256, 3), (2048, 7), (1024, 64)])
def test_matrix_route_tiles_and_splits(gfq_gpu, q, rows, split):
    A, B = inputs.pair(q, 600, 700, 300, cfg=212, idx=rows + split)
    check(gfq_gpu, q, A, B, rows=rows, split=split, variant=gfq_gpu.VARIANT_KARATSUBA)


@pytest.mark.parametrize("q", MATRIX_ROUTE_FIELDS)
def test_matrix_route_sparse_and_identity(gfq_gpu, q):
    A, B = inputs.pair(q, 300, 513, 257, cfg=213, idx=0, density=0.1)
    check(gfq_gpu, q, A, B, variant=gfq_gpu.VARIANT_KARATSUBA)
    eye = np.eye(513, dtype=np.uint8)
    check(gfq_gpu, q, eye, B, variant=gfq_gpu.VARIANT_KARATSUBA)


@pytest.mark.parametrize("q", MATRIX_ROUTE_FIELDS)
def test_matrix_route_equals_rowwise_2048(gfq_gpu, q):
    """2048^3: the two routes give the same packed product byte for byte."""
    import torch
    g = gfq_gpu
    N = 2048
    A, B = inputs.pair(q, N, N, N, cfg=214, idx=q)
    Ap, Bp = g.pack(q, dev(A)), g.pack(q, dev(B))
    rw = g.matmul(q, Ap, Bp, N, N, N, variant=g.VARIANT_ROWWISE)
    mr = g.matmul(q, Ap, Bp, N, N, N, variant=g.VARIANT_KARATSUBA)
    assert torch.equal(rw, mr)


def test_variant_validation(gfq_gpu):
    import torch
    g = gfq_gpu
    Ap, Bp = g.pack(3, dev(np.zeros((64, 64), np.uint8))), g.pack(3, dev(np.zeros((64, 64), np.uint8)))
    for q, var in ((3, g.VARIANT_KARATSUBA), (5, g.VARIANT_KARATSUBA), (7, g.VARIANT_KARATSUBA), (4, 2), (4, -1),
                   (8, 2), (9, -1)):
        with pytest.raises(g.GfqError) as e:
            g.matmul(q, Ap, Bp, 64, 64, 64, variant=var)
        assert e.value.status == -1, (q, var)
    torch.cuda.synchronize()


@pytest.mark.parametrize("rows,k", [(2048, 8), (1024, 7), (256, 10)])
def test_gf8_4096_sampled(gfq_gpu, rows, k):
    """GF(8), A and B 4096 x 4096 uniform, in three launch configurations (eight rows per
    lane, four, and narrow tiles at k = 10): sampled rows, spread over every row tile and
    covering the last one, against the oracle."""
    import torch
    g = gfq_gpu
    q, N = 8, 4096
    A, B = inputs.pair(q, N, N, N, cfg=220, idx=rows)
    Ap, Bp = g.pack(q, dev(A)), g.pack(q, dev(B))
    C = g.unpack(q, g.matmul(q, Ap, Bp, N, N, N, rows=rows, k=k), N, N)
    sample = np.unique(np.concatenate([np.arange(0, N, 97), np.arange(N - 5, N)]))
    got = C[torch.from_numpy(sample).cuda()].cpu().numpy()
    assert np.array_equal(got, oracle.matmul(q, A[sample], B))


@pytest.mark.parametrize("k", [6, 8, 10])
def test_f9_2048_sampled(gfq_gpu, k):
    """F_9, A and B 2048 x 2048 uniform, at the widest tables (k = 6) and at narrowed ones
    (k = 8, 10): sampled rows, spread over every row tile and covering the last one,
    against the oracle."""
    import torch
    g = gfq_gpu
    q, N = 9, 2048
    A, B = inputs.pair(q, N, N, N, cfg=221, idx=k)
    Ap, Bp = g.pack(q, dev(A)), g.pack(q, dev(B))
    C = g.unpack(q, g.matmul(q, Ap, Bp, N, N, N, k=k), N, N)
    sample = np.unique(np.concatenate([np.arange(0, N, 61), np.arange(N - 5, N)]))
    got = C[torch.from_numpy(sample).cuda()].cpu().numpy()
    assert np.array_equal(got, oracle.matmul(q, A[sample], B))


@pytest.mark.parametrize("q", [5, 9])
def test_longest_inner_dimension(gfq_gpu, q):
    """l = 2^24 - 1, the largest inner dimension the library accepts (m = 3, n = 40: B is
    the large operand), against the oracle; l = 2^24 is rejected before any launch."""
    import torch
    g = gfq_gpu
    m, l, n = 3, (1 << 24) - 1, 40
    A, B = inputs.pair(q, m, l, n, cfg=250, idx=q)
    check(g, q, A, B)
    Ap = g.empty_packed(q, m, 1 << 24)
    Bp = g.empty_packed(q, 1 << 24, n)
    with pytest.raises(g.GfqError) as e:
        g.matmul(q, Ap, Bp, m, 1 << 24, n)
    assert e.value.status == -3
    torch.cuda.synchronize()


# the slab width at which each field's table takes 128-byte super-rows, i.e. one 32-word tile
# row per entry plane (planes swapped on odd entries for the even plane counts of F_3, GF(4), F_9)
WIDE_K = {3: 8, 4: 8, 5: 7, 7: 7, 8: 7, 9: 7}


@pytest.mark.parametrize("q", FIELDS)
@pytest.mark.parametrize("rows,split", [(512, 1), (512, 3), (256, 2), (1024, 1), (1024, 3), (2048, 2)])
def test_wide_tiles(gfq_gpu, q, rows, split):
    """32-word tiles: three column tiles with a ragged last one (n = 2300 is 72 words), a ragged
    last row tile and a ragged last slab, at the tile heights and splits the layout runs with;
    every element and every packed byte against the oracle."""
    A, B = inputs.pair(q, 1100, 701, 2300, cfg=230, idx=rows + split)
    check(gfq_gpu, q, A, B, k=WIDE_K[q], rows=rows, split=split)


@pytest.mark.parametrize("q,rows", [(3, 512), (3, 1024), (3, 256), (9, 0), (4, 1024), (4, 512), (4, 256),
                                    (7, 256), (7, 512), (8, 512), (8, 256)])
def test_wide_tiles_entry_parity(gfq_gpu, q, rows):
    """B = identity rows in a fixed order and A one-hot, so that every table entry of both
    parities is gathered and each product row equals one row of B: a plane swap left undone on
    odd entries, or on the rows that read their planes exchanged (F_3, F_9: the second row of
    every 16-lane read pass, which accumulates the negated row; GF(4): that row also takes its
    two table rows in exchanged order and accumulates x^2 C^2), or through a front slot (F_7,
    GF(8): that row reads 2t or x t), would show as wrong planes."""
    k = WIDE_K[q]
    l, n = 2 * k, 1500
    rng = np.random.default_rng(231)
    B = rng.integers(0, q, size=(l, n), dtype=np.uint8)
    m = 1 << k
    A = np.zeros((m, l), dtype=np.uint8)
    for e in range(m):                       # row e selects slab-0 rows by the bits of e
        for t in range(k):
            A[e, t] = (e >> t) & 1
        A[e, k + (e % k)] = 1                # and one row of slab 1
    check(gfq_gpu, q, A, B, k=k, rows=rows)
    if q in (4, 7, 8):
        # coefficients of every basis element (x, x^2; 2, 4): every gather of a slab selects
        # entries of both parities
        X = A.copy()
        X[:, 1::3] *= 2
        if q != 4:
            X[:, 2::3] *= 4
        X[:, k:] = A[:, k:] * np.uint8(3)
        check(gfq_gpu, q, X, B, k=k, rows=rows)


FIT_M = (1, 40, 65, 100, 129, 200, 257, 300, 513, 700, 1025, 1100, 1600, 2049, 2100)


@pytest.mark.parametrize("q", FIELDS)
@pytest.mark.parametrize("k,rows", [(0, 2048), (0, 1024), (0, 512), (4, 256), (10, 2048)])
def test_ragged_last_row_tile(gfq_gpu, q, k, rows):
    """Products whose last row tile holds 1 .. 2100 rows, at each tile height (k = 0: the
    wide-tile slab width), with ragged slabs and column tiles; every element and packed byte
    against the oracle."""
    k = k or WIDE_K[q]
    for i, m in enumerate(FIT_M):
        A, B = inputs.pair(q, m, 3 * k + 1, 1500, cfg=232, idx=1000 * k + i)
        check(gfq_gpu, q, A, B, k=k, rows=rows)


@pytest.mark.parametrize("q", MATRIX_ROUTE_FIELDS)
@pytest.mark.parametrize("rows", [2048, 512])
def test_matrix_route_ragged_last_row_tile(gfq_gpu, q, rows):
    """The matrix-level routes' products with last row tiles of 1 .. 2100 rows against the
    oracle."""
    for i, m in enumerate(FIT_M):
        A, B = inputs.pair(q, m, 45, 700, cfg=233, idx=rows + i)
        check(gfq_gpu, q, A, B, rows=rows, variant=gfq_gpu.VARIANT_KARATSUBA)
