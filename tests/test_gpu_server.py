"""Product server (continuous batching): every result equals the oracle's and the same
product computed alone with the plain calls, bit for bit, whatever it was batched with;
arrival order, the memory budget, resident packed operands, serial mode, degenerate
requests and validation."""
import numpy as np
import pytest

import oracle
from paper_0901_1413_amd import inputs

pytestmark = pytest.mark.gpu


def dev(x):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def make(g, specs, cfg, t0=0.0, gaps_us=None):
    import torch
    reqs, keep, host = [], [], []
    t = t0
    for i, (q, m, l, n) in enumerate(specs):
        A, B = inputs.pair(q, m, l, n, cfg=cfg, idx=i)
        Ad, Bd = dev(A), dev(B)
        Cd = torch.full((m, n), 0xAB, dtype=torch.uint8, device="cuda")
        if gaps_us is not None:
            t += gaps_us[i]
        reqs.append(g.Server.request(q, m, l, n, Ad, Bd, Cd, tag=i, not_before_us=t if gaps_us is not None else 0.0))
        keep.append((Ad, Bd, Cd))
        host.append((A, B))
    return reqs, keep, host


def check(g, specs, keep, host, comps):
    assert sorted(c["tag"] for c in comps) == list(range(len(specs)))
    for c in comps:
        assert c["status"] == 0, c
        assert c["arrival_us"] <= c["launch_us"] <= c["done_us"], c
    for i, (q, m, l, n) in enumerate(specs):
        Ad, Bd, Cd = keep[i]
        got = Cd.cpu().numpy()
        A, B = host[i]
        assert np.array_equal(got, oracle.matmul(q, A, B)), ("oracle", i, q, m, l, n)
        alone = g.matmul_unpacked(q, Ad, Bd).cpu().numpy() if m and n else got
        assert np.array_equal(got, alone), ("alone", i, q, m, l, n)


def mixed_specs(seed, count, lo=16, hi=700):
    rng = np.random.default_rng(seed)
    specs = []
    for _ in range(count):
        q = int(rng.choice([3, 4, 5, 7, 8, 9]))
        if rng.random() < 0.5:
            n = int(round(np.exp(rng.uniform(np.log(lo), np.log(hi)))))
            specs.append((q, n, n, n))
        else:
            m, l, n = (int(x) for x in rng.integers(1, hi, size=3))
            specs.append((q, m, l, n))
    return specs


def test_server_poisson_mix_equals_alone_and_oracle(gfq_gpu):
    g = gfq_gpu
    specs = mixed_specs(401, 240)
    rng = np.random.default_rng(402)
    gaps = rng.exponential(150.0, size=len(specs))            # about 6700 requests/s
    # the last 40 arrive 150 ms after the others, so that the trace is served in more than one
    # batch however long the host takes to submit it (a fresh process loads the kernels first)
    gaps[200] += 150000.0
    srv = g.Server(budget_bytes=256 << 20, slots=3)
    try:
        reqs, keep, host = make(g, specs, 403, t0=0.0, gaps_us=gaps)
        t0 = srv.now_us() + 5000.0                             # arrivals start 5 ms after setup
        for r in reqs:
            r.not_before_us += t0
        srv.submit(reqs, keep)
        comps = srv.wait_all(len(specs))
        check(g, specs, keep, host, comps)
        by_tag = {c["tag"]: c for c in comps}
        for i, r in enumerate(reqs):
            assert by_tag[i]["arrival_us"] >= r.not_before_us - 1e-6
        st = srv.stats()
        assert st["completed"] == len(specs) and st["queued"] == 0 and st["arena_in_use"] == 0
        assert st["batches"] >= 2
    finally:
        srv.destroy()


def test_server_burst_forms_large_batches(gfq_gpu):
    g = gfq_gpu
    specs = mixed_specs(404, 300, lo=32, hi=400)
    srv = g.Server(budget_bytes=1 << 30, slots=2, max_batch=128)
    try:
        reqs, keep, host = make(g, specs, 405)
        srv.submit(reqs, keep)
        comps = srv.wait_all(len(specs))
        check(g, specs, keep, host, comps)
        st = srv.stats()
        assert 1 < st["max_batch_seen"] <= 128
        assert st["batches"] < len(specs)
    finally:
        srv.destroy()


def test_server_budget_limits_admission(gfq_gpu):
    g = gfq_gpu
    budget = 1 << 20
    specs = [(5, 300, 300, 300)] * 30 + [(3, 257, 129, 300)] * 10
    srv = g.Server(budget_bytes=budget, slots=3)
    try:
        reqs, keep, host = make(g, specs, 406)
        srv.submit(reqs, keep)
        comps = srv.wait_all(len(specs))
        check(g, specs, keep, host, comps)
        st = srv.stats()
        assert 0 < st["arena_peak_in_use"] <= budget and st["arena_held"] <= budget
        assert st["max_batch_seen"] < len(specs)
        # a request whose packed operands alone exceed the budget is refused at submission
        big_reqs, big_keep, _ = make(g, [(7, 2000, 2000, 64)], 407)
        with pytest.raises(g.GfqError) as e:
            srv.submit(big_reqs, big_keep)
        assert e.value.status == -9
    finally:
        srv.destroy()


def test_server_resident_packed_operands(gfq_gpu):
    import torch
    g = gfq_gpu
    q, l, n = 7, 333, 500
    rng_specs = [(q, m, l, n) for m in (1, 64, 257, 600)]
    Bh = inputs.matrix(q, l, n, cfg=0, idx=900, which=1)
    Bp = g.pack(q, dev(Bh))                                     # kept packed on the device
    srv = g.Server()
    try:
        reqs, keep, host = [], [], []
        for i, (_, m, _, _) in enumerate(rng_specs):
            Ah = inputs.matrix(q, m, l, cfg=0, idx=910 + i, which=0)
            Ad = dev(Ah)
            if i % 2 == 0:                                      # packed product
                Cd = g.empty_packed(q, m, n)
                flags = g.REQ_B_PACKED | g.REQ_C_PACKED
            else:
                Cd = torch.full((m, n), 0xAB, dtype=torch.uint8, device="cuda")
                flags = g.REQ_B_PACKED
            reqs.append(g.Server.request(q, m, l, n, Ad, Bp, Cd, tag=i, flags=flags))
            keep.append((Ad, Bp, Cd))
            host.append(Ah)
        Ap = g.pack(q, dev(host[0]))                           # packed A as well
        Cp = g.empty_packed(q, 1, n)
        reqs.append(g.Server.request(q, 1, l, n, Ap, Bp, Cp, tag=len(reqs),
                                     flags=g.REQ_A_PACKED | g.REQ_B_PACKED | g.REQ_C_PACKED))
        keep.append((Ap, Bp, Cp))
        host.append(host[0])
        srv.submit(reqs, keep)
        comps = srv.wait_all(len(reqs))
        assert all(c["status"] == 0 for c in comps)
        for i, r in enumerate(reqs):
            m = r.m
            want = oracle.matmul(q, host[i], Bh)
            C = keep[i][2]
            got = g.unpack(q, C, m, n).cpu().numpy() if r.flags & g.REQ_C_PACKED else C.cpu().numpy()
            assert np.array_equal(got, want), i
    finally:
        srv.destroy()


def test_server_serial_mode_matches(gfq_gpu):
    g = gfq_gpu
    specs = mixed_specs(408, 40, lo=16, hi=300)
    srv = g.Server(serial=True)
    try:
        reqs, keep, host = make(g, specs, 409)
        srv.submit(reqs, keep)
        comps = srv.wait_all(len(specs))
        check(g, specs, keep, host, comps)
        assert all(c["batch_size"] == 1 for c in comps)
        assert srv.stats()["max_batch_seen"] == 1
    finally:
        srv.destroy()


def test_server_pool_slices(gfq_gpu):
    """Operands that are windows of larger device matrices (leading dimension > columns)."""
    import torch
    g = gfq_gpu
    P = 1000
    srv = g.Server()
    try:
        reqs, keep, host = [], [], []
        rng = np.random.default_rng(410)
        for i, q in enumerate([3, 4, 5, 7, 8, 9]):
            pa = inputs.matrix(q, P, P, cfg=0, idx=920 + i, which=0)
            pb = inputs.matrix(q, P, P, cfg=0, idx=920 + i, which=1)
            m, l, n = (int(x) for x in rng.integers(1, 400, size=3))
            r0, c0, r1, c1 = (int(x) for x in rng.integers(0, 500, size=4))
            Ad, Bd = dev(pa)[r0:r0 + m, c0:c0 + l], dev(pb)[r1:r1 + l, c1:c1 + n]
            Cbig = torch.full((m, n + 37), 0xAB, dtype=torch.uint8, device="cuda")
            Cd = Cbig[:, 5:5 + n]
            reqs.append(g.Server.request(q, m, l, n, Ad, Bd, Cd, tag=i))
            keep.append((Ad, Bd, Cd, Cbig))
            host.append((pa[r0:r0 + m, c0:c0 + l], pb[r1:r1 + l, c1:c1 + n], q))
        srv.submit(reqs, keep)
        comps = srv.wait_all(len(reqs))
        assert all(c["status"] == 0 for c in comps)
        for i, (A, B, q) in enumerate(host):
            Cbig = keep[i][3].cpu().numpy()
            n = B.shape[1]
            assert np.array_equal(Cbig[:, 5:5 + n], oracle.matmul(q, A, B)), i
            assert (Cbig[:, :5] == 0xAB).all() and (Cbig[:, 5 + n:] == 0xAB).all(), i
    finally:
        srv.destroy()


def test_server_degenerate_requests(gfq_gpu):
    import torch
    g = gfq_gpu
    srv = g.Server()
    try:
        C = torch.full((5, 7), 0xAB, dtype=torch.uint8, device="cuda")
        A = torch.zeros((5, 1), dtype=torch.uint8, device="cuda")
        B = torch.zeros((1, 7), dtype=torch.uint8, device="cuda")
        reqs = [
            g.Request(3, 0, 5, 5, None, 5, None, 5, None, 5, 0, 0, 0.0),           # m = 0
            g.Request(5, 5, 0, 7, None, 0, None, 7, C.data_ptr(), 7, 0, 1, 0.0),   # l = 0: C = 0
            g.Request(7, 5, 5, 0, None, 5, None, 0, None, 0, 0, 2, 0.0),           # n = 0
            g.Server.request(4, 5, 1, 7, A, B, torch.empty((5, 7), dtype=torch.uint8, device="cuda"), tag=3),
        ]
        srv.submit(reqs, [None, C, None, (A, B)])
        comps = srv.wait_all(4)
        assert all(c["status"] == 0 for c in comps)
        assert (C.cpu().numpy() == 0).all()
    finally:
        srv.destroy()


def test_server_validation(gfq_gpu):
    import torch
    g = gfq_gpu
    srv = g.Server(budget_bytes=1 << 20)
    try:
        A = torch.zeros((64, 64), dtype=torch.uint8, device="cuda")
        B = torch.zeros((64, 64), dtype=torch.uint8, device="cuda")
        C = torch.zeros((64, 64), dtype=torch.uint8, device="cuda")
        P = g.empty_packed(3, 64, 64)
        good = g.Server.request(3, 64, 64, 64, A, B, C, tag=7)
        cases = [
            (g.Request(2, 64, 64, 64, A.data_ptr(), 64, B.data_ptr(), 64, C.data_ptr(), 64, 0, 1, 0.0), -2),
            (g.Request(3, 70000, 64, 64, A.data_ptr(), 64, B.data_ptr(), 64, C.data_ptr(), 64, 0, 1, 0.0), -3),
            (g.Request(3, 64, 64, 64, A.data_ptr(), 63, B.data_ptr(), 64, C.data_ptr(), 64, 0, 1, 0.0), -3),
            (g.Request(3, 64, 64, 64, A.data_ptr(), 64, B.data_ptr(), 64, C.data_ptr(), 32, 0, 1, 0.0), -3),
            (g.Request(3, 64, 64, 64, None, 64, B.data_ptr(), 64, C.data_ptr(), 64, 0, 1, 0.0), -4),
            (g.Request(3, 64, 64, 64, A.data_ptr(), 64, B.data_ptr(), 64, None, 64, 0, 1, 0.0), -4),
            (g.Request(3, 64, 64, 64, P.data_ptr() + 4, 0, B.data_ptr(), 64, C.data_ptr(), 64, 1, 1, 0.0), -5),
            (g.Request(3, 64, 64, 64, A.data_ptr(), 64, B.data_ptr(), 64, A.data_ptr() + 64, 64, 0, 1, 0.0), -6),
            (g.Request(3, 64, 64, 64, A.data_ptr(), 64, B.data_ptr(), 64, C.data_ptr(), 64, 8, 1, 0.0), -1),
        ]
        for bad, status in cases:
            with pytest.raises(g.GfqError) as e:
                srv.submit([good, bad], [(A, B, C)])
            assert e.value.status == status, (status, e.value)
        assert srv.stats()["submitted"] == 0                   # a rejected call queues nothing
        srv.submit([good], [(A, B, C)])
        comps = srv.wait_all(1)
        assert comps[0]["status"] == 0 and comps[0]["tag"] == 7
    finally:
        srv.destroy()


@pytest.mark.parametrize("serial", [False, True])
def test_results_copied_to_host(gfq_gpu, serial):
    """Requests with a host destination: the completion reports the product already in
    host memory (pinned), equal to the device result and to the oracle's."""
    import torch
    g = gfq_gpu
    specs = mixed_specs(421, 24, lo=16, hi=400)
    srv = g.Server(budget_bytes=128 << 20, serial=serial)
    try:
        reqs, keep, host = make(g, specs, 422)
        hosts = []
        for i, (q, m, l, n) in enumerate(specs):
            h = torch.full((m * n + 16,), 0xCD, dtype=torch.uint8, pin_memory=True)
            hosts.append(h)
            reqs[i].C_host = h.data_ptr()
        srv.submit(reqs, [k + (h,) for k, h in zip(keep, hosts)])
        comps = srv.wait_all(len(specs))
        # read the host copies before anything else touches the device results
        got_host = [hosts[i][:m * n].numpy().reshape(m, n).copy() for i, (q, m, l, n) in enumerate(specs)]
        check(g, specs, keep, host, comps)
        for i, (q, m, l, n) in enumerate(specs):
            assert np.array_equal(got_host[i], keep[i][2].cpu().numpy()), ("host copy", i)
            assert bool((hosts[i][m * n:] == 0xCD).all()), ("past the span", i)
    finally:
        srv.destroy()


def test_watchdog_fails_overdue_batches(gfq_gpu):
    """The watchdog forced from the host: with a limit far below any batch's run time every
    batch is overdue at its first poll, so its requests complete with GFQ_EHIP, the server
    is marked failed and refuses later submissions.  The device work itself runs to its end
    normally; the test waits for it before the operands go away."""
    import torch
    g = gfq_gpu
    specs = [(3, 256, 256, 256), (5, 200, 300, 100), (4, 128, 128, 128)]
    srv = g.Server(budget_bytes=64 << 20, slots=1, watchdog_s=1e-9)
    reqs, keep, host = make(g, specs, 431)
    try:
        srv.submit(reqs, keep)
        comps = srv.wait_all(len(specs))
        assert sorted(c["tag"] for c in comps) == list(range(len(specs)))
        assert all(c["status"] == -8 for c in comps), comps
        with pytest.raises(g.GfqError) as e:
            srv.submit([g.Server.request(3, 256, 256, 256, keep[0][0], keep[0][1], keep[0][2], tag=99)])
        assert e.value.status == -8
    finally:
        torch.cuda.synchronize()                  # the abandoned batch's device work
        srv.destroy()
    torch.cuda.synchronize()
