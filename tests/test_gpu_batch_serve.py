"""Batched and served forms: every cell's / request's result must equal the
single-cell path bit for bit, whatever else runs with it (also on the FP64
LDS path with several cells per launch); graph replays must
equal eager execution at every replay; admission must queue (not fail) what
fits later and fail what can never fit.
"""
import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def bzq():
    import torch  # noqa: F401
    from paper_2004_11239_amd import bzq as b
    return b


def _dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def _host(t):
    import torch
    torch.cuda.synchronize()
    return t.cpu().numpy()


def _f(N, L, seed):
    return workloads.to_spectral(workloads.random_mixture(seed).sample(N, L))


def _cells(bzq):
    pa = bzq.Plan(16, 8.0, 4.0, 0.0, 0.5, 16, 38, precision="fp32")
    pb = bzq.Plan(24, 8.0, 4.0, -1.0, 0.25, 8, 26, precision="fp32")
    pc = bzq.Plan(8, 8.0, 4.0, 0.0, 0.75, 8, 14, precision="fp64")
    plans = [pa, pb, pa, pc, pa, pb, pa]
    fs = [_f(p.N, 8.0, 100 + i) for i, p in enumerate(plans)]
    return plans, fs


@pytest.mark.parametrize("cpl", [0, 2, 64])
def test_batch_collision_bitwise_equals_solo(bzq, cpl):
    import torch
    plans, fs = _cells(bzq)
    solo = [_host(p.collision(_dev(f))) for p, f in zip(plans, fs)]
    fd = [_dev(f) for f in fs]
    batch = bzq.Batch(plans, fd, cells_per_launch=cpl)
    groups = batch.groups()
    assert sum(g["cells"] for g in groups) == len(plans) and len(groups) == 3
    outs = [torch.empty_like(f) for f in fd]
    batch.collision(outs)
    for a, b in zip(solo, outs):
        assert np.array_equal(a, _host(b))
    batch.destroy()


def test_batch_step_graph_replays_equal_eager(bzq):
    plans, fs = _cells(bzq)
    dt = 0.01
    # reference: single-cell Heun steps, one replay at a time
    ref = [_dev(f) for f in fs]
    eager = [_dev(f) for f in fs]
    graph = [_dev(f) for f in fs]
    be = bzq.Batch(plans, eager, cells_per_launch=4)
    bg = bzq.Batch(plans, graph, cells_per_launch=4)
    for rep in range(3):
        for p, r in zip(plans, ref):
            p.step(r, dt, 1)
        be.step(dt, 1, use_graph=False)
        bg.step(dt, 1, use_graph=True)
        R = [_host(x) for x in ref]
        for a, b, c in zip(R, eager, graph):
            assert np.array_equal(a, _host(b)), rep
            assert np.array_equal(a, _host(c)), rep
    be.destroy()
    bg.destroy()


def test_batch_fp64_lds_path_bitwise_equals_solo(bzq):
    """FP64 at N = 48 (P = 72): the pencils do not fit the register file, so the
    evaluation takes the separate ingest and the LDS z-inverse, here with three
    cells in one launch; Q and two Heun steps (the update inside finalize), eager
    and graph-replayed, bitwise equal to the single-cell path."""
    import torch
    plan = bzq.Plan(48, 9.0, 4.5, 0.0, 0.5, 4, 6, precision="fp64")
    plans = [plan, plan, plan]
    fs = [_f(48, 9.0, 300 + i) for i in range(3)]
    solo = [_host(plan.collision(_dev(f))) for f in fs]
    fd = [_dev(f) for f in fs]
    batch = bzq.Batch(plans, fd, cells_per_launch=3)
    outs = [torch.empty_like(f) for f in fd]
    batch.collision(outs)
    for a, b in zip(solo, outs):
        assert np.array_equal(a, _host(b))
    batch.destroy()
    dt = 0.01
    ref = [_dev(f) for f in fs]
    eager = [_dev(f) for f in fs]
    graph = [_dev(f) for f in fs]
    be = bzq.Batch(plans, eager, cells_per_launch=3)
    bg = bzq.Batch(plans, graph, cells_per_launch=3)
    for rep in range(2):
        for r in ref:
            plan.step(r, dt, 1)
        be.step(dt, 1, use_graph=False)
        bg.step(dt, 1, use_graph=True)
        R = [_host(x) for x in ref]
        for a, b, c in zip(R, eager, graph):
            assert np.array_equal(a, _host(b)), rep
            assert np.array_equal(a, _host(c)), rep
    be.destroy()
    bg.destroy()


def test_workspaces_on_two_streams(bzq):
    import torch
    plan = bzq.Plan(16, 8.0, 4.0, 0.0, 0.5, 16, 38, precision="fp32")
    f1, f2 = _dev(_f(16, 8.0, 1)), _dev(_f(16, 8.0, 2))
    r1, r2 = _host(plan.collision(f1)), _host(plan.collision(f2))
    w1, w2 = bzq.Workspace(plan), bzq.Workspace(plan)
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    torch.cuda.synchronize()
    o1, o2 = torch.empty_like(f1), torch.empty_like(f2)
    for _ in range(3):
        w1.collision(f1, o1, stream=s1)
        w2.collision(f2, o2, stream=s2)
    torch.cuda.synchronize()
    assert np.array_equal(_host(o1), r1) and np.array_equal(_host(o2), r2)


REQS = [(16, -1.0, 0.25, 11), (24, 0.0, 0.75, 12), (16, 0.0, 0.75, 13), (32, -1.0, 0.25, 14),
        (24, -1.0, 0.25, 15), (16, 0.0, 0.25, 16)]


def _submit(srv, N, g, s, seed, n_steps=3, N_rho=8, M=14):
    return srv.submit(_f(N, 8.0, seed), N, 8.0, 4.0, g, s, N_rho, M, "fp32", 0.01, n_steps)


def test_server_result_alone_equals_in_mix(bzq):
    srv = bzq.Server(16 << 30, slots=4)
    alone = []
    for (N, g, s, seed) in REQS:
        rid = _submit(srv, N, g, s, seed)
        srv.wait(rid)
        out, (ta, ts, td) = srv.poll(rid, N)
        assert ta <= ts <= td
        alone.append(out)
    ids = [_submit(srv, N, g, s, seed) for (N, g, s, seed) in REQS]
    for rid, (N, *_), a in zip(ids, REQS, alone):
        srv.wait(rid)
        out, _ = srv.poll(rid, N)
        assert np.array_equal(out, a)
    st = srv.stats()
    assert st["completed"] == 2 * len(REQS) and st["failed"] == 0
    srv.destroy()
    # the same request through the single-cell path
    p = bzq.Plan(16, 8.0, 4.0, -1.0, 0.25, 8, 14, precision="fp32")
    f = _dev(_f(16, 8.0, 11))
    p.step(f, 0.01, 3)
    assert np.array_equal(_host(f), alone[0])


def test_server_admission_queues_and_fails_what_cannot_fit(bzq):
    # the N = 32 plan alone takes most of the budget, so the N = 16 plans
    # must be evicted and rebuilt around it
    need16 = bzq.plan_bytes_estimate(16, 16, 110, "fp32") + 16 ** 3 * 16
    need32 = bzq.plan_bytes_estimate(32, 32, 110, "fp32") + 32 ** 3 * 16
    budget = need32 + need16 + need16 // 2
    assert budget > (64 << 20)
    srv = bzq.Server(budget, slots=4)
    ids = [(_submit(srv, N, g, s, seed, 1, N, 110), N) for (N, g, s, seed) in REQS if N in (16, 32)]
    for rid, N in ids:
        srv.wait(rid, 300)
        out, _ = srv.poll(rid, N)
        assert np.isfinite(out).all()
    st = srv.stats()
    assert st["failed"] == 0 and st["peak_device_bytes"] <= budget
    assert st["evictions"] >= 1
    srv.destroy()
    # a request larger than the whole budget fails instead of waiting forever
    small = bzq.Server(64 << 20, slots=1)
    rid = small.submit(_f(64, 8.0, 3), 64, 8.0, 4.0, 0.0, 0.5, 64, 110, "fp32", 0.01, 1)
    small.wait(rid, 60)
    with pytest.raises(bzq.BzqError):
        small.poll(rid, 64)
    small.destroy()


def test_serve_driver_reports_latency(bzq):
    from paper_2004_11239_amd import serve
    r = serve.run(50.0, 1.0, seed=3, budget_gb=8, slots=4, n_steps=2, sizes=(16, 24), M=14, max_queued=0)
    assert r["completed"] == r["requests"] > 10
    assert 0 < r["p50_s"] <= r["p99_s"]


def test_server_collision_requests_alone_and_in_mix(bzq):
    """A Q(f) request (BZQ_REQ_COLLISION) returns bzq_collision's result bitwise,
    alone and in a mix with step requests of other sizes and gammas."""
    N, g, s, seed = 16, -1.0, 0.25, 31
    srv = bzq.Server(16 << 30, slots=4)
    rid = srv.submit(_f(N, 8.0, seed), N, 8.0, 4.0, g, s, 8, 14, "fp32", kind="collision")
    srv.wait(rid)
    alone, _ = srv.poll(rid, N)
    ids = []
    for i, (Nm, gm, sm, sd) in enumerate(REQS):
        ids.append((_submit(srv, Nm, gm, sm, sd), Nm))
        if i == 2:
            qid = srv.submit(_f(N, 8.0, seed), N, 8.0, 4.0, g, s, 8, 14, "fp32", kind="collision")
    srv.wait(qid)
    mixed, _ = srv.poll(qid, N)
    for rid, Nm in ids:
        srv.wait(rid)
        srv.poll(rid, Nm)
    srv.destroy()
    p = bzq.Plan(N, 8.0, 4.0, g, s, 8, 14, precision="fp32")
    ref = _host(p.collision(_dev(_f(N, 8.0, seed))))
    assert np.array_equal(alone, ref)
    assert np.array_equal(mixed, ref)


def test_server_bounded_queue_rejects(bzq):
    """With one slot and at most two waiting requests, a burst of submissions is
    partly refused with BZQ_EBUSY (nothing queued); every accepted request
    completes and the refusals are counted."""
    srv = bzq.Server(16 << 30, slots=1, max_queued=2)
    f = _f(32, 8.0, 5)
    accepted, refused = [], 0
    for _ in range(12):
        try:
            accepted.append(srv.submit(f, 32, 8.0, 4.0, 0.0, 0.5, 16, 38, "fp32", 0.01, 4))
        except bzq.BzqError as e:
            assert e.code == 6
            refused += 1
    # the first two fill the queue before the worker takes any of them
    assert refused > 0 and len(accepted) >= 2
    for rid in accepted:
        srv.wait(rid, 120)
        out, _ = srv.poll(rid, 32)
        assert np.isfinite(out).all()
    st = srv.stats()
    assert st["rejected"] == refused and st["completed"] == len(accepted) and st["failed"] == 0
    srv.destroy()


def test_server_gamma_sibling_without_room_for_both(bzq):
    """A budget that holds one plan with its state but not the cached plan
    beside a plan derived from it for another gamma: the second request evicts
    the idle first plan and builds its own instead of waiting forever."""
    N, N_rho, M = 32, 16, 38
    full = bzq.plan_bytes_estimate(N, N_rho, M, "fp32") + N ** 3 * 16
    budget = full + full // 3
    srv = bzq.Server(budget, slots=2)
    a = _submit(srv, N, 0.0, 0.5, 41, 1, N_rho, M)
    srv.wait(a, 120)
    qa, _ = srv.poll(a, N)
    b = _submit(srv, N, -1.0, 0.5, 42, 1, N_rho, M)
    assert srv.wait(b, 120) is None
    qb, _ = srv.poll(b, N)
    assert np.isfinite(qa).all() and np.isfinite(qb).all()
    st = srv.stats()
    assert st["failed"] == 0 and st["completed"] == 2 and st["evictions"] >= 1
    assert st["peak_device_bytes"] <= budget
    srv.destroy()
    # the gamma = -1 result equals the single-cell path
    p = bzq.Plan(N, 8.0, 4.0, -1.0, 0.5, N_rho, M, precision="fp32")
    f = _dev(_f(N, 8.0, 42))
    p.step(f, 0.01, 1)
    assert np.array_equal(_host(f), qb)


def test_mixed_size_launches_are_refused(bzq):
    """While the mixed-size launches are switched off, a batch that demands
    them (cells_per_launch = -1) is refused with BZQ_EUNSUPPORTED before any
    of their kernels runs, and the default (0) takes grouped launches."""
    p16 = bzq.Plan(16, 8.0, 4.0, 0.0, 0.5, 8, 14, precision="fp32")
    p24 = bzq.Plan(24, 8.0, 4.0, -1.0, 0.25, 6, 14, precision="fp32")
    fd = [_dev(_f(16, 8.0, 1)), _dev(_f(24, 8.0, 2))]
    with pytest.raises(bzq.BzqError) as e:
        bzq.Batch([p16, p24], fd, cells_per_launch=-1)
    assert e.value.code == 4
    b = bzq.Batch([p16, p24], fd, cells_per_launch=1)
    assert b.rounds() == 0 and len(b.groups()) == 2
    b.destroy()


@pytest.mark.skip(reason="mixed-size launches are switched off: their first device run ended in a GPU memory "
                         "fault whose cause is not known (a CPU build of the kernel bodies finds every access "
                         "in bounds and every result bitwise equal)")
@pytest.mark.parametrize("budget_mb", [8192, 48])
def test_mixed_size_launches_bitwise_equal_solo(bzq, budget_mb, monkeypatch):
    """Cells of N = 16, 24 and 32 (FP32 bulk, different gammas and s) in the
    mixed-size launches: one launch per pipeline stage over a device table of
    work items of every size, in one round (8 GB of workspace) or in several
    (48 MB).  Q of every cell, and two Heun steps (eager and graph-replayed),
    equal the single-cell path bit for bit."""
    import torch
    monkeypatch.setenv("BZQ_BATCH_WS_MB", str(budget_mb))
    p16 = bzq.Plan(16, 8.0, 4.0, 0.0, 0.5, 8, 14, precision="fp32")
    p24 = bzq.Plan(24, 8.0, 4.0, -1.0, 0.25, 6, 14, precision="fp32")
    p32 = bzq.Plan(32, 8.0, 4.0, 0.0, 0.75, 4, 14, precision="fp32")
    plans = [p16, p24, p32, p16, p16, p24, p32, p16, p24]
    fs = [_f(p.N, 8.0, 300 + i) for i, p in enumerate(plans)]
    solo_q = [_host(p.collision(_dev(f))) for p, f in zip(plans, fs)]
    fd = [_dev(f) for f in fs]
    batch = bzq.Batch(plans, fd, cells_per_launch=-1)
    rounds = batch.rounds()
    assert rounds >= 1 and (rounds > 1) == (budget_mb < 100), rounds
    outs = [torch.empty_like(f) for f in fd]
    batch.collision(outs)
    for a, b in zip(solo_q, outs):
        assert np.array_equal(a, _host(b))
    # two Heun steps: solo, batched eager, batched graph
    ref = [_dev(f) for f in fs]
    for p, r in zip(plans, ref):
        p.step(r, 0.01, 2)
    batch.step(0.01, 2, use_graph=False)
    for a, b in zip(ref, fd):
        assert np.array_equal(_host(a), _host(b))
    fg = [_dev(f) for f in fs]
    bg = bzq.Batch(plans, fg, cells_per_launch=-1)
    for rep in range(2):
        bg.step(0.01, 1, use_graph=True)
        torch.cuda.synchronize()
    for a, b in zip(ref, fg):
        assert np.array_equal(_host(a), _host(b))
    batch.destroy()
    bg.destroy()
    # a plan the mixed launches do not take is refused when they are demanded
    p8 = bzq.Plan(8, 8.0, 4.0, 0.0, 0.5, 4, 14, precision="fp32")
    with pytest.raises(bzq.BzqError):
        bzq.Batch([p16, p8], [_dev(_f(16, 8.0, 1)), _dev(_f(8, 8.0, 2))], cells_per_launch=-1)
