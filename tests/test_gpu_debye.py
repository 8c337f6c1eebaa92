"""The Debye-Yukawa kernel of Section 5.6 and its cutoff (bzq_plan_create_debye)
against the oracle's DebyeKernel.

The weight has a logarithmic singularity (and a kink at theta = pi/3); both
sides integrate it with a composite rule of their own construction (host C++
and scipy/numpy), and the oracle's rule is pinned against a 30-digit theta
quadrature of eq. ApproximatedDebye.  Tolerances as in test_gpu_parity.py.
"""
import math

import numpy as np
import pytest

import oracle
import workloads
from oracle.angular import DebyeKernel

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-11, "fp32": 1e-5}
CUTS = [0.0, math.pi / 10]


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


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.mark.parametrize("cut", CUTS)
def test_debye_weights_match_oracle(bzq, cut):
    """Stored weights of sampled pairs at the BKW geometry (R = 6, a|k| up to ~37)."""
    N, R = 32, 6.0
    L = (3 + math.sqrt(2)) * R / 4
    plan = bzq.Plan.debye(N, L, R, cut, 8, 38, precision="fp64")
    pairs = plan.pairs()
    P = plan.info()["P"]
    n1 = N - 1
    r = np.arange(n1) - (N // 2 - 1)
    K = np.stack(np.meshgrid(r, r, r, indexing="ij"), -1).transpose(1, 0, 2, 3).reshape(n1 * n1, n1, 3)
    nh = (n1 * n1 + 1) // 2
    K = K[:nh].reshape(-1, 3)
    kern = DebyeKernel(cut)
    for j in (0, 9, len(pairs) // 2, len(pairs) - 1):
        rho, sx, sy, sz, wq, _ = pairs[j]
        a = math.pi * rho / (2 * L)
        sig = np.array([sx, sy, sz])
        F = oracle.F_weight(K, a, sig, kern)
        ref = (2 * wq * np.real(np.exp(-1j * a * (K @ sig)) * F) / P ** 3).reshape(nh, n1)
        got = plan.weights(j)
        err = np.max(np.abs(got - ref)) / np.max(np.abs(ref))
        print(cut, j, f"{err:.2e}")
        assert err <= 1e-12, (j, err)
    assert plan.info()["n_jacobi"] == (204 if cut == 0.0 else 120)
    plan.destroy()


@pytest.mark.parametrize("cut", CUTS)
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_debye_collision_matches_oracle(bzq, cut, prec):
    for (N, L, R, N_rho, M, seed) in [(8, 6.0, 3.0, 5, 14, 3), (16, 8.0, 4.0, 8, 38, 4)]:
        d = oracle.Discretization.debye(N, L, R, cut, N_rho, M)
        f = workloads.to_spectral(workloads.random_mixture(seed).sample(N, L))
        ref = oracle.collision_direct(f, d)
        plan = bzq.Plan.debye(N, L, R, cut, N_rho, M, precision=prec)
        Q = _host(plan.collision(_dev(f)))
        err = _rel(Q, ref)
        print(N, cut, prec, f"{err:.3e}")
        assert err < TOL[prec]
        assert Q[0, 0, 0] == 0.0
        plan.destroy()


def test_debye_sampled_32(bzq):
    """32^3, sampled output modes (oracle one mode at a time), FP64 and FP32."""
    N, L, R, N_rho, M = 32, 8.0, 4.0, 12, 50
    d = oracle.Discretization.debye(N, L, R, 0.0, N_rho, M)
    f = workloads.to_spectral(workloads.random_mixture(8).sample(N, L))
    rng = np.random.default_rng(32)
    ks = np.concatenate([np.array([[0, 0, 0], [15, -15, 15], [1, 0, 0]]), rng.integers(-15, 16, size=(21, 3))])
    ref = oracle.collision_direct(f, d, k_out=ks)
    for prec in ("fp64", "fp32"):
        plan = bzq.Plan.debye(N, L, R, 0.0, N_rho, M, precision=prec)
        Q = _host(plan.collision(_dev(f)))
        got = Q[tuple(np.mod(ks, N).T)]
        err = _rel(got, ref)
        print(prec, f"{err:.3e}")
        assert err < TOL[prec]
        plan.destroy()
