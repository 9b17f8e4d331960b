"""Batched products (one work-list launch per field and tile shape, workgroups taking
(product, row tile, column tile, slab slice) items longest first, and a partial-sum launch for
sliced products): every product of a mixed batch against the oracle and against the same
product launched alone (bit-exact), graph replays, degenerate products, slab slices."""
import numpy as np
import pytest

import oracle
from paper_0901_1413_amd import inputs

pytestmark = pytest.mark.gpu


def dev(x):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def make_batch(g, specs, cfg):
    probs, host = [], []
    for idx, (q, m, l, n) in enumerate(specs):
        A, B = inputs.pair(q, m, l, n, cfg=cfg, idx=idx)
        Ap, Bp = g.pack(q, dev(A)), g.pack(q, dev(B))
        C = g.empty_packed(q, m, n)
        C.fill_(0x5A)
        probs.append((q, m, l, n, Ap, Bp, C))
        host.append((A, B))
    return probs, host


def check_against_oracle_and_alone(g, probs, host, which):
    for i in which:
        q, m, l, n, Ap, Bp, C = probs[i]
        A, B = host[i]
        got = g.unpack(q, C, m, n).cpu().numpy()
        assert np.array_equal(got, oracle.matmul(q, A, B)), (i, q, m, l, n)
        alone = g.matmul(q, Ap, Bp, m, l, n)
        nb = g.packed_bytes(q, m, n)
        assert np.array_equal(alone.cpu().numpy()[:nb], C.cpu().numpy()[:nb]), ("alone differs", i)


def test_mixed_batch(gfq_gpu):
    g = gfq_gpu
    rng = np.random.default_rng(301)
    specs = []
    for i in range(60):
        q = int(rng.choice([3, 4, 5, 7, 8, 9]))
        m, l, n = (int(x) for x in rng.integers(1, 700, size=3))
        specs.append((q, m, l, n))
    specs += [(3, 1, 1, 1), (5, 1025, 33, 7), (7, 64, 2048, 64), (4, 2048, 64, 1000), (8, 1500, 700, 1200),
              (9, 900, 500, 1300)]
    probs, host = make_batch(g, specs, 302)
    g.matmul_batched(probs)
    g.sync()
    check_against_oracle_and_alone(g, probs, host, range(len(specs)))


def test_batch_replay_and_times(gfq_gpu):
    g = gfq_gpu
    specs = [(3, 300, 200, 100), (5, 64, 64, 64), (7, 1000, 900, 130), (4, 513, 127, 511), (3, 2048, 2048, 2048),
             (8, 777, 300, 555), (9, 300, 400, 500)]
    probs, host = make_batch(g, specs, 303)
    b = g.Batch(probs)
    for rep in range(3):
        for (_, _, _, _, _, _, C) in probs:
            C.fill_(0x11)
        b.launch()
        g.sync()
        t = b.times_us()
        assert all(x > 0 for x in t) and max(t) < 1e7, t
        check_against_oracle_and_alone(g, probs, host, range(len(specs)))
    b.destroy()


def test_batch_degenerate_and_rejection(gfq_gpu):
    g = gfq_gpu
    specs = [(3, 5, 0, 7), (5, 0, 4, 4), (7, 4, 4, 0), (4, 9, 3, 9), (8, 6, 0, 6), (9, 0, 3, 3)]
    probs, host = make_batch(g, specs, 304)
    g.matmul_batched(probs)
    g.sync()
    q, m, l, n, _, _, C = probs[0]
    assert not C.cpu().numpy()[:g.packed_bytes(q, m, n)].any()          # l = 0: zero product
    check_against_oracle_and_alone(g, probs, host, [3])
    bad = list(probs) + [(11, 4, 4, 4, probs[3][4], probs[3][5], probs[3][6])]
    with pytest.raises(g.GfqError) as e:
        g.matmul_batched(bad)
    assert e.value.status == -2


def test_c4_shaped_batch_sampled(gfq_gpu):
    """512 products shaped like the batched workload (fields F_3/F_5/F_7, m, l, n
    log-uniform in [64, 2048]); every product equals its single launch, a sample equals
    the oracle."""
    g = gfq_gpu
    specs = inputs.batch_specs(512, cfg=4)
    probs, host = make_batch(g, specs, 4)
    g.matmul_batched(probs)
    g.sync()
    for i, (q, m, l, n, Ap, Bp, C) in enumerate(probs):
        alone = g.matmul(q, Ap, Bp, m, l, n)
        nb = g.packed_bytes(q, m, n)
        assert np.array_equal(alone.cpu().numpy()[:nb], C.cpu().numpy()[:nb]), i
    check_against_oracle_and_alone(g, probs, host, range(0, 512, 37))


@pytest.mark.parametrize("forked", [False, True])
def test_batch_graph_capture_replays(gfq_gpu, forked):
    """gfq_batch_launch allocates nothing and makes no synchronising call, so it can be
    captured into a HIP graph; every replay (with eager work in between) equals the eager
    launch bit for bit.  forked: the capture stream launched the batch eagerly before, so its
    side streams exist and the capture holds the groups as parallel branches; otherwise the
    capture launches the groups one after another."""
    import torch
    g = gfq_gpu
    specs = [(3, 300, 200, 100), (5, 64, 64, 64), (7, 1000, 900, 130), (4, 513, 127, 511), (5, 700, 1500, 900)]
    probs, host = make_batch(g, specs, 311)
    b = g.Batch(probs)
    b.launch()
    g.sync()
    want = [C.clone() for (*_, C) in probs]
    for i, (q, m, l, n, _, _, C) in enumerate(probs):
        assert np.array_equal(g.unpack(q, C, m, n).cpu().numpy(), oracle.matmul(q, *host[i])), i
    graph = torch.cuda.CUDAGraph()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        if forked:
            b.launch()
            side.synchronize()
        with torch.cuda.graph(graph, stream=side):
            b.launch()
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    Ao, Bo = inputs.pair(3, 64, 64, 64, cfg=311, idx=99)
    Aop, Bop = g.pack(3, dev(Ao)), g.pack(3, dev(Bo))
    other = g.empty_packed(3, 64, 64)
    for rep in range(4):
        for (*_, C) in probs:
            C.zero_()
        g.matmul(3, Aop, Bop, 64, 64, 64, out=other)            # eager work between replays
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        for i, (w, (*_, C)) in enumerate(zip(want, probs)):
            assert torch.equal(w, C), (rep, i)
        times = b.times_us()
        assert all(t > 0 for t in times), (rep, times)
    del graph


def test_batch_narrow_tiles(gfq_gpu):
    """Products taller than 256 rows and at most 256 (128) columns wide run as one column of
    8-word (4-word) tiles; every field, ragged edges, against the oracle and the plain launch."""
    g = gfq_gpu
    specs = []
    for q in (3, 4, 5, 7, 8, 9):
        specs += [(q, 1500, 300, 100), (q, 700, 200, 250), (q, 257, 65, 128), (q, 2049, 129, 129), (q, 300, 33, 1)]
    probs, host = make_batch(g, specs, 320)
    g.matmul_batched(probs)
    g.sync()
    check_against_oracle_and_alone(g, probs, host, range(len(specs)))


def test_batch_slab_slices(gfq_gpu):
    """Products with few tiles and a long inner dimension (300 x 20000 x 700, every field) are
    cut into slab slices whose partial products a partial-sum launch adds; the small products
    beside them stay whole.  Every product against the oracle and its single launch, on two
    launches of the batch, with completion times."""
    g = gfq_gpu
    specs = [(q, 300, 20000, 700) for q in (3, 4, 5, 7, 8, 9)]
    specs += [(3 + (i % 2) * 2, 64 + i, 100 + 7 * i, 33 + 5 * i) for i in range(40)]
    probs, host = make_batch(g, specs, 330)
    b = g.Batch(probs)
    slices = b.slices()
    assert all(s > 1 for s in slices[:6]), slices[:6]
    assert all(s == 1 for s in slices[6:]), slices[6:]
    for rep in range(2):
        for (*_, C) in probs:
            C.fill_(0x33)
        b.launch()
        g.sync()
        t = b.times_us()
        assert all(x > 0 for x in t), t
        check_against_oracle_and_alone(g, probs, host, range(len(specs)))
    b.destroy()


def test_batch_persistent_matches_worklist(gfq_gpu):
    """The same batch drained by persistent workgroups through a device queue head: every
    product equals the work-list launch's byte for byte and the oracle, on three launches in a
    row (the head is reset by each launch), including sliced products and their partial sums."""
    import torch
    g = gfq_gpu
    rng = np.random.default_rng(340)
    specs = [(int(rng.choice([3, 4, 5, 7, 8, 9])),) + tuple(int(x) for x in rng.integers(1, 600, size=3))
             for _ in range(40)]
    specs += [(3, 300, 9000, 700), (7, 200, 9000, 300), (4, 2048, 64, 1000), (5, 1025, 33, 7)]
    probs, host = make_batch(g, specs, 341)
    b = g.Batch(probs)
    b.launch()
    g.sync()
    want = [C.clone() for (*_, C) in probs]
    for rep in range(3):
        for (*_, C) in probs:
            C.fill_(0x77)
        b.launch_persistent()
        g.sync()
        for i, (w, (*_, C)) in enumerate(zip(want, probs)):
            assert torch.equal(w, C), (rep, i, specs[i])
        t = b.times_us()
        assert all(x > 0 for x in t), (rep, t)
    check_against_oracle_and_alone(g, probs, host, range(0, len(specs), 3))
    b.destroy()


def test_batch_persistent_graph_capture(gfq_gpu):
    """A persistent launch captured into a graph (the lists as parallel branches): every replay,
    with eager work in between, equals the work-list launch."""
    import torch
    g = gfq_gpu
    specs = [(3, 300, 200, 100), (5, 64, 64, 64), (7, 1000, 900, 130), (4, 513, 127, 511), (5, 700, 1500, 900)]
    probs, host = make_batch(g, specs, 342)
    b = g.Batch(probs)
    b.launch()
    g.sync()
    want = [C.clone() for (*_, C) in probs]
    graph = torch.cuda.CUDAGraph()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        b.launch_persistent()
        side.synchronize()
        with torch.cuda.graph(graph, stream=side):
            b.launch_persistent()
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    Ao, Bo = inputs.pair(3, 64, 64, 64, cfg=342, idx=99)
    Aop, Bop = g.pack(3, dev(Ao)), g.pack(3, dev(Bo))
    other = g.empty_packed(3, 64, 64)
    for rep in range(3):
        for (*_, C) in probs:
            C.zero_()
        g.matmul(3, Aop, Bop, 64, 64, 64, out=other)
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        for i, (w, (*_, C)) in enumerate(zip(want, probs)):
            assert torch.equal(w, C), (rep, i)
    del graph
    b.destroy()


def test_batch_persistent_narrow_and_degenerate(gfq_gpu):
    """Persistent drains of narrow-tile lists (8- and 4-word tiles of tall, thin products),
    two launches back to back on one stream (the second launch's head reset is ordered after
    the first launch's drain), and of a batch of degenerate products (an l = 0 product, whose
    tiles write zeros, and products without tiles)."""
    g = gfq_gpu
    specs = []
    for q in (3, 4, 5, 7, 8, 9):
        specs += [(q, 1500, 300, 100), (q, 700, 200, 250), (q, 2049, 129, 129)]
    probs, host = make_batch(g, specs, 350)
    b = g.Batch(probs)
    b.launch_persistent()
    b.launch_persistent()
    g.sync()
    check_against_oracle_and_alone(g, probs, host, range(len(specs)))
    b.destroy()
    empty, _ = make_batch(g, [(3, 5, 0, 7), (5, 0, 4, 4), (7, 4, 4, 0)], 351)
    e = g.Batch(empty)
    e.launch_persistent()
    g.sync()
    C = empty[0][6]
    assert not bool((C[:g.packed_bytes(3, 5, 7)] != 0).any())          # l = 0: the zero product
    e.destroy()


FIT_M = (1, 40, 65, 100, 129, 200, 257, 300, 513, 700, 1025, 1100, 1600, 2049, 2100)


@pytest.mark.parametrize("tall", [False, True])
def test_batch_tile_fit_rows(gfq_gpu, tmp_path, tall):
    """Batch items cut by a product's edges run the tile body at the fewest rows per lane
    that cover their rows (R, R / 2, ..., 1; F_9: 2), and at half the tile width when they
    hold at most half its words.  Products whose last row tile holds 1 .. 2100 rows, in every
    field, 100, 200, 1100 and 1500 columns wide (narrow tiles; 16-word tiles of 4, 7 and 3
    words in the last column tile; 15 words), with the tile heights the library chooses (two
    rows per lane) and with batch tuning entries of 2048-row tiles (the field's most rows per
    lane); the work-list and the persistent launches, each product against the oracle and
    against its plain launch."""
    import torch
    g = gfq_gpu
    if tall:
        arch = torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]
        table = tmp_path / "tall_tiles.txt"
        table.write_text("".join(f"{arch} 1 {q} {bm} 6 0 6 2048 1 0\n"
                                 for q in (3, 4, 5, 7, 8, 9) for bm in range(6, 15)))
        g.tune_clear()
        g.tune_load(str(table))
    try:
        specs = [(q, m, 40, n) for q in (3, 4, 5, 7, 8, 9) for m in FIT_M for n in (100, 200, 1100, 1500)]
        probs, host = make_batch(g, specs, 360 + int(tall))
        b = g.Batch(probs)
        b.launch()
        g.sync()
        check_against_oracle_and_alone(g, probs, host, range(len(specs)))
        for (*_, C) in probs:
            C.fill_(0x5A)
        b.launch_persistent()
        g.sync()
        check_against_oracle_and_alone(g, probs, host, range(len(specs)))
        b.destroy()
    finally:
        if tall:
            g.tune_clear()
