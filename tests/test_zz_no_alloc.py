"""gfq_matmul_noalloc (the product with no device allocation) against gfq_matmul_config, the
entry point it is a variant of: packed products byte for byte on two calls in a row, the
second smaller, so the second reads the library's fixed partial-product array after the
first has filled it; the split lowered to fit that array; and the explicit configuration
whose partial products do not fit it refused before any launch."""
import numpy as np
import pytest

import oracle
from paper_0901_1413_amd import inputs

pytestmark = pytest.mark.gpu


def dev(x):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def packed_pair(g, q, m, l, n, cfg, idx):
    A, B = inputs.pair(q, m, l, n, cfg=cfg, idx=idx)
    return A, B, g.pack(q, dev(A)), g.pack(q, dev(B))


@pytest.mark.parametrize("q", [3, 5, 7, 4])
def test_noalloc_equals_matmul_config_two_calls(gfq_gpu, q):
    g = gfq_gpu
    # a split product that fills several partial products, then a smaller one
    for (m, l, n, k, rows, split, idx) in ((2100, 3000, 1500, 7, 512, 8, 1), (300, 450, 200, 6, 256, 3, 2)):
        A, B, Ap, Bp = packed_pair(g, q, m, l, n, 240, idx)
        C_ref = g.empty_packed(q, m, n)
        C_na = g.empty_packed(q, m, n)
        C_na.fill_(0x5A)                                # stale bytes the call must overwrite
        g.matmul(q, Ap, Bp, m, l, n, out=C_ref, k=k, rows=rows, split=split)
        g.matmul_noalloc(q, Ap, Bp, m, l, n, C_na, k=k, rows=rows, split=split)
        g.sync()
        assert bool((C_na == C_ref).all()), f"q={q} {m}x{l}x{n} split={split}"
        if idx == 2:                                    # the small one also against the oracle
            C = g.unpack(q, C_na, m, n).cpu().numpy()
            assert np.array_equal(C, oracle.matmul(q, A, B))


def test_noalloc_chosen_config_and_degenerate(gfq_gpu):
    g = gfq_gpu
    q, m, l, n = 3, 513, 2000, 700
    A, B, Ap, Bp = packed_pair(g, q, m, l, n, 241, 0)
    C_ref, C_na = g.empty_packed(q, m, n), g.empty_packed(q, m, n)
    g.matmul(q, Ap, Bp, m, l, n, out=C_ref)
    g.matmul_noalloc(q, Ap, Bp, m, l, n, C_na)
    g.sync()
    assert bool((C_na == C_ref).all())
    # l = 0 writes a zero product; m = 0 is a no-op
    Z = g.empty_packed(q, m, n)
    Z.fill_(0x33)
    g.matmul_noalloc(q, Ap, Bp, m, 0, n, Z)
    g.matmul_noalloc(q, Ap, Bp, 0, l, n, Z)
    g.sync()
    assert int(Z.count_nonzero()) == 0


def test_noalloc_split_fitted_to_the_array(gfq_gpu, tmp_path):
    """A tuned configuration whose four partial products (4 x 24 MiB for F_5, 8192 x 8192)
    exceed the 64 MiB array: with no explicit configuration the split is lowered (to two) and
    the product equals gfq_matmul's; the same configuration given explicitly is refused."""
    g = gfq_gpu
    q, m, l, n = 5, 8192, 512, 8192
    assert 4 * g.packed_bytes(q, m, n) > g.NOALLOC_SCRATCH_BYTES >= 2 * g.packed_bytes(q, m, n)
    f = tmp_path / "tune.txt"
    f.write_text("gfx950 0 5 13 9 13 7 512 4 0 8192 8192\n")
    g.tune_clear()
    try:
        g.tune_load(str(f))
        assert g.choose_config(q, m, l, n)["split"] == 4
        A, B, Ap, Bp = packed_pair(g, q, m, l, n, 242, 0)
        C_ref, C_na = g.empty_packed(q, m, n), g.empty_packed(q, m, n)
        g.matmul(q, Ap, Bp, m, l, n, out=C_ref)          # four slices in the workspace
        g.matmul_noalloc(q, Ap, Bp, m, l, n, C_na)       # two slices in the array
        g.sync()
        assert bool((C_na == C_ref).all())
        rows = np.array([0, 1, 777, 4095, 4096, 8191])
        C = g.unpack(q, C_na, m, n)[dev(rows).long()].cpu().numpy()
        assert np.array_equal(C, oracle.matmul(q, A[rows], B))
        with pytest.raises(g.GfqError) as e:
            g.matmul_noalloc(q, Ap, Bp, m, l, n, C_na, k=7, rows=512, split=4)
        assert e.value.status == -9                      # GFQ_EBUDGET
        g.sync()
    finally:
        g.tune_clear()
