"""Autotuner: the tuned configuration is cached per size class, used by gfq_choose_config /
gfq_matmul and by batches, survives a save / load round trip, and the products computed
with it still equal the oracle's bit for bit."""
import numpy as np
import pytest

import oracle
from paper_0901_1413_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.fixture
def tuned(gfq_gpu):
    gfq_gpu.tune_clear()
    yield gfq_gpu
    gfq_gpu.tune_clear()


def dev(x):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


@pytest.mark.parametrize("q", [3, 5])
def test_tune_plain_is_used_and_exact(tuned, q, tmp_path):
    g = tuned
    m, l, n = 1000, 1500, 900
    assert g.tune_lookup(q, m, l, n) is None
    c = g.tune(q, m, l, n)
    assert 3 <= c["k"] <= 10 and c["rows"] in (256, 512, 1024, 2048) and c["split"] >= 1
    assert g.tune_lookup(q, m, l, n) == c
    assert g.choose_config(q, m, l, n) == c
    # a shape of the same class shares the entry (split clamped to its slab count)
    assert g.tune_lookup(q, m - 100, l - 200, n + 20)["k"] == c["k"]
    A, B = inputs.pair(q, m, l, n, cfg=0, idx=50 + q)
    got = g.matmul_unpacked(q, dev(A), dev(B)).cpu().numpy()
    assert np.array_equal(got, oracle.matmul(q, A, B))
    f = tmp_path / "tune.txt"
    g.tune_save(str(f))
    g.tune_clear()
    assert g.tune_lookup(q, m, l, n) is None
    g.tune_load(str(f))
    assert g.tune_lookup(q, m, l, n) == c


def test_tune_batch_class_used_by_batches(tuned):
    g = tuned
    c = g.tune(7, 300, 400, 256, batch=True)
    # the batch layouts hold k <= 6 at two rows per lane and k <= 8 at four (one-copy rows)
    assert c["split"] == 1 and c["k"] <= (8 if c["rows"] > 256 else 6)
    assert g.tune_lookup(7, 300, 400, 10, batch=True) == c        # n does not enter a batch class
    specs = [(7, 300, 400, 256), (7, 290, 390, 77), (3, 300, 400, 100)]
    probs, host = [], []
    for i, (q, m, l, n) in enumerate(specs):
        A, B = inputs.pair(q, m, l, n, cfg=0, idx=60 + i)
        probs.append((q, m, l, n, g.pack(q, dev(A)), g.pack(q, dev(B)), g.empty_packed(q, m, n)))
        host.append((A, B))
    g.matmul_batched(probs)
    g.sync()
    for (q, m, l, n, _, _, C), (A, B) in zip(probs, host):
        assert np.array_equal(g.unpack(q, C, m, n).cpu().numpy(), oracle.matmul(q, A, B))


def test_tune_rejects_bad_arguments(tuned):
    g = tuned
    for args in [(2, 64, 64, 64), (3, 0, 64, 64), (3, 64, 0, 64), (3, 64, 64, 1 << 17)]:
        with pytest.raises(g.GfqError):
            g.tune(*args)


def test_lookup_splits_smaller_products_again(tuned, tmp_path):
    """An entry of the class 2049..4096 timed at 4096^3 (F_9, k = 7, 512-row tiles of 32 words,
    split 4): a 4096^3 product keeps it; a 2500^3 product of the same class has 15 tiles (3
    column tiles by 5 row tiles) instead of 32, so its split is chosen again for its own shape
    (the cost model gives 16: 240 workgroups, one round), never below the cached split; an entry
    timed at 2500^3 itself keeps its split there.  The re-split product is checked against the
    oracle on sampled rows."""
    import torch
    g = tuned
    f = tmp_path / "t.txt"
    f.write_text("gfx950 0 9 12 12 12 7 512 4 0\n")
    g.tune_load(str(f))
    assert g.choose_config(9, 4096, 4096, 4096) == {"k": 7, "rows": 512, "split": 4, "variant": 0}
    assert g.choose_config(9, 2500, 2500, 2500) == {"k": 7, "rows": 512, "split": 16, "variant": 0}
    q, N = 9, 2500
    A, B = inputs.pair(q, N, N, N, cfg=222, idx=0)
    C = g.matmul_unpacked(q, dev(A), dev(B))
    sample = np.unique(np.concatenate([np.arange(0, N, 97), np.arange(N - 3, N)]))
    got = C[torch.from_numpy(sample).cuda()].cpu().numpy()
    assert np.array_equal(got, oracle.matmul(q, A[sample], B))
    g.tune_clear()
    f.write_text("gfx950 0 9 12 12 12 7 512 4 0 2500 2500\n")
    g.tune_load(str(f))
    assert g.choose_config(9, 2500, 2500, 2500)["split"] == 4
    # the split chosen again is never below the cached one (the model alone would give 16)
    g.tune_clear()
    f.write_text("gfx950 0 9 12 12 12 7 512 32 0\n")
    g.tune_load(str(f))
    assert g.choose_config(9, 2500, 2500, 2500)["split"] == 32
