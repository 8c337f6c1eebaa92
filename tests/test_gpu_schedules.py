"""Every kernel schedule against the oracle, and the schedule autotuner.

A plan's schedule picks, per pipeline stage, one whole pencil per lane or two
waves per pencil (the pipelined kernel for the last stage), and the last
stage's workgroup count.  All schedules evaluate eq. realQ and must meet the
same parity bar against the stored oracle samples (32^3 and 64^3) and against
the oracle evaluated live on a 48^3 sample (ragged radix-3 lengths).
Tolerances as in test_gpu_parity.py.
"""
import functools
import itertools
import os

import numpy as np
import pytest

import oracle
import workloads

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
TOL = {"fp64": 1e-11, "fp32": 1e-5}


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


def _golden(name):
    data = np.load(os.path.join(GOLDEN, name + ".npz"), allow_pickle=False)
    N, L, R, gamma, s, N_rho, M, seed = data["params"]
    N, N_rho, M, seed = int(N), int(N_rho), int(M), int(seed)
    mix = workloads.two_maxwellians(seed) if int(data["kind"]) == 0 else workloads.random_mixture(seed)
    f = workloads.to_spectral(mix.sample(N, L))
    return (N, L, R, gamma, s, N_rho, M), f, data["modes"], data["Q"]


@pytest.fixture(scope="module")
def case48():
    N, L, R, gamma, s, N_rho, M = 48, 9.0, 4.5, 0.0, 0.5, 6, 14
    f = workloads.to_spectral(workloads.random_mixture(11).sample(N, L))
    d = oracle.Discretization.power(N, L, R, gamma, s, N_rho, M)
    rng = np.random.default_rng(4848)
    ks = np.concatenate([np.array([[0, 0, 0], [23, -23, 23], [1, 0, 0]]), rng.integers(-23, 24, size=(21, 3))])
    return (N, L, R, gamma, s, N_rho, M), f, ks, oracle.collision_direct(f, d, k_out=ks)


SCHEDULES = [c + (1024,) for c in itertools.product((1, 2), repeat=3)] + [(0, 0, 2, 512), (0, 0, 2, 2048),
                                                                          (0, 0, 1, 2048)]


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
@pytest.mark.parametrize("which", ["medium_s050", "large_s050", "n48"])
def test_every_schedule_matches_oracle(bzq, case48, which, prec):
    if which == "n48":
        params, f, ks, ref = case48
    else:
        params, f, ks, ref = _golden(which)
    N = params[0]
    plan = bzq.Plan(*params, precision=prec)
    fd = _dev(f)
    for sched in SCHEDULES:
        got_s = plan.set_schedule(*sched)
        Q = _host(plan.collision(fd))
        got = Q[tuple(np.mod(ks, N).T)]
        err = float(np.linalg.norm(got - ref) / np.linalg.norm(ref))
        print(f"{which} {prec} {sched} -> {got_s}: {err:.3e}", flush=True)
        assert err < TOL[prec], (sched, err)
        assert Q[0, 0, 0] == 0.0
    plan.destroy()


@pytest.mark.parametrize("sched", [(1, 3, 1, 1024), (2, 3, 1, 512), (1, 3, 2, 2048)])
def test_parity_split_plane_fp64_matches_oracle(bzq, sched):
    """FP64 at P = 96: the plane taken by column parity (variant 3), with its
    four-way column pass assembled through LDS and the two parities' row
    transforms combined in registers, against the stored oracle samples at
    64^3."""
    params, f, ks, ref = _golden("large_s050")
    N = params[0]
    plan = bzq.Plan(*params, precision="fp64")
    got_s = plan.set_schedule(*sched)
    assert got_s["plane"] == 3
    Q = _host(plan.collision(_dev(f)))
    got = Q[tuple(np.mod(ks, N).T)]
    err = float(np.linalg.norm(got - ref) / np.linalg.norm(ref))
    print(f"large fp64 {sched}: {err:.3e}", flush=True)
    assert err < TOL["fp64"], (sched, err)
    assert Q[0, 0, 0] == 0.0
    plan.destroy()


def test_parity_split_plane_only_fp64_at_p96(bzq):
    for N, prec in ((64, "fp32"), (32, "fp64"), (48, "fp64")):
        plan = bzq.Plan(N, 8.0, 4.0, 0.0, 0.5, 4, 6, precision=prec)
        with pytest.raises(bzq.BzqError):
            plan.set_schedule(1, 3, 1, 1024)
        plan.destroy()


def test_schedule_rejects_missing_variants(bzq):
    plan = bzq.Plan(16, 8.0, 4.0, 0.0, 0.5, 8, 14, precision="fp32")
    with pytest.raises(bzq.BzqError):
        plan.set_schedule(2, 1, 1, 1024)      # no two-wave kernels at P = 24
    with pytest.raises(bzq.BzqError):
        plan.set_schedule(1, 1, 1, 777)
    assert plan.schedule()["zinv"] == 1


def test_autotune_keeps_parity_and_caches(bzq, tmp_path, monkeypatch):
    monkeypatch.setenv("BZQ_TUNE_CACHE", str(tmp_path / "tune.txt"))
    params, f, ks, ref = _golden("medium_s050")
    N = params[0]
    fd = _dev(f)
    plan = bzq.Plan(*params, precision="fp32")
    sched = plan.autotune(fd, use_cache=False)
    assert sched["zinv"] in (1, 2) and sched["plane"] in (1, 2) and sched["zfwd"] in (1, 2)
    Q = _host(plan.collision(fd))
    got = Q[tuple(np.mod(ks, N).T)]
    assert np.linalg.norm(got - ref) / np.linalg.norm(ref) < TOL["fp32"]
    # one schedule, bitwise reproducible
    assert np.array_equal(Q, _host(plan.collision(fd)))
    assert (tmp_path / "tune.txt").exists()
    plan2 = bzq.Plan(*params, precision="fp32")
    assert plan2.autotune(fd, use_cache=True) == sched


@functools.lru_cache(maxsize=None)
def _small_n_reference(N):
    f = workloads.broadband_spectrum(N, 31 + N)
    d = oracle.Discretization.power(N, 8.0, 4.0, -1.0, 0.5, 4, 14)
    return f, oracle.collision_direct(f, d)


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
@pytest.mark.parametrize("N", [16, 24])
def test_pipelined_last_stage_small_n_matches_oracle(bzq, N, prec):
    """The pipelined z-forward at P = 24 and 36 (one producer wave with whole
    register transforms, one consumer wave): every mode of a broadband input
    against the oracle evaluated live, per mode and in the L2 norm, beside the
    whole-pencil kernel; both s_target values that change the split count."""
    L, R, gamma, s, N_rho, M = 8.0, 4.0, -1.0, 0.5, 4, 14
    f, ref = _small_n_reference(N)
    plan = bzq.Plan(N, L, R, gamma, s, N_rho, M, precision=prec)
    fd = _dev(f)
    for sched in [(1, 1, 2, 512), (1, 1, 2, 2048), (1, 1, 1, 1024)]:
        got_s = plan.set_schedule(*sched)
        assert got_s["zfwd"] == sched[2]
        Q = _host(plan.collision(fd))
        err = float(np.linalg.norm(Q - ref) / np.linalg.norm(ref))
        worst = float(np.max(np.abs(Q - ref)) / np.max(np.abs(ref)))
        print(f"N={N} {prec} {sched} -> {got_s}: rel L2 {err:.3e}, worst {worst:.3e}", flush=True)
        assert err < TOL[prec] and worst < TOL[prec], (sched, err, worst)
    plan.destroy()
