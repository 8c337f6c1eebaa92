"""Pins of the oracle's angular weight F (eq. FF) against independent routes.

* eq. cutoff3D: the closed form for constant b;
* the second-order expansion of the proof of Proposition 2.1;
* eq. FF3D1 done as a 2-D (t, azimuth) rule without any Bessel function;
* a 30-digit mpmath quadrature of the theta-form;
* the BKW rate lambda = 1/6 of the paper's kernels b5..b8 (Section 5.3) by
  direct quadrature of its definition;
* the paper's own eps-split precompute (Section 4.1) converging to F.
"""
import math

import numpy as np
import pytest
from scipy.integrate import quad

from oracle.angular import (PAPER_KERNELS, F_eps_split, F_sphere, F_weight, bkw_lambda,
                            cutoff_kernel, power_kernel, psi, psi_cutoff_closed_form,
                            psi_small_argument)

RNG = np.random.default_rng(1234)


def test_cutoff_closed_form():
    C = 1.0 / (4.0 * math.pi)
    x = RNG.uniform(-45, 45, 200)
    y = RNG.uniform(0, 45, 200)
    got = psi(x, y, cutoff_kernel(C))
    ref = psi_cutoff_closed_form(x, y, C)
    assert np.max(np.abs(got - ref)) < 1e-13


@pytest.mark.parametrize("s", [0.0, 0.25, 0.5, 0.75, 0.95])
def test_small_argument_expansion(s):
    k = power_kernel(s)
    for scale in (1e-2, 1e-3):
        x, y = 0.7 * scale, 1.3 * scale
        err = abs(psi(x, y, k) - psi_small_argument(x, y, k))
        # next term is third order in (x, y)
        assert err < 50.0 * k.c * scale ** 3, (s, scale, err)
    # F(0) = 0 exactly (Remark 4.1 rests on it)
    assert psi(0.0, 0.0, k) == 0.0


def test_conjugate_symmetry():
    k = power_kernel(0.5)
    x = RNG.uniform(0, 40, 50)
    y = RNG.uniform(0, 40, 50)
    np.testing.assert_allclose(psi(-x, y, k), np.conj(psi(x, y, k)), rtol=0, atol=1e-14)


@pytest.mark.parametrize("name", ["b5", "b6", "b7", "b8"])
def test_bessel_route_matches_sphere_route(name):
    """F by the exact azimuth (J0) vs F by a product rule over the sphere (eq. FF3D1)."""
    kern = PAPER_KERNELS[name]
    for trial in range(6):
        kv = RNG.integers(-7, 8, size=3)
        q = RNG.normal(size=3)
        q /= np.linalg.norm(q)
        a = RNG.uniform(0.05, 1.4)
        ref = F_sphere(kv, a, q, kern, n_t=96, n_phi=96)
        got = F_weight(kv[None, :], a, q, kern)[0]
        assert abs(got - ref) <= 2e-12 * max(1.0, abs(ref)), (name, kv, a, got, ref)


def test_against_mpmath_reference():
    mp = pytest.importorskip("mpmath")
    mp.mp.dps = 30
    k = power_kernel(0.5)

    def psi_mp(x, y):
        x = mp.mpf(x)
        y = mp.mpf(y)

        def f(t):
            Y = 2 * y * mp.sqrt(t * (1 - t))
            return t ** (-k.s) * (mp.expj(2 * x * t) * mp.besselj(0, Y) - 1) / t

        pts = mp.linspace(0, 1, 9)
        re = mp.quad(lambda t: mp.re(f(t)), pts)
        im = mp.quad(lambda t: mp.im(f(t)), pts)
        return complex(4 * mp.pi * k.c * mp.mpc(re, im))

    for x, y in [(0.3, 0.1), (5.0, 2.0), (9.5, 9.5)]:
        ref = psi_mp(x, y)
        assert abs(psi(x, y, k) - ref) <= 1e-14 * abs(ref) + 1e-16, (x, y)


@pytest.mark.parametrize("name", ["b5", "b6", "b7", "b8"])
def test_paper_kernels_share_lambda(name):
    kern = PAPER_KERNELS[name]
    # lambda = 1/4 \int_{S^2} (1 - cos^2 th) b d sigma = pi/2 \int_0^pi sin^3 th b(th) d th
    paper_b = {
        "b5": lambda th: 1 / (4 * math.pi),
        "b6": lambda th: 1 / (8 * math.pi * math.sin(th) * math.sin(th / 2)),
        "b7": lambda th: 1 / (6 * math.pi ** 2 * math.sin(th) * math.sin(th / 2) ** 2),
        "b8": lambda th: 5 * math.cos(th / 2) / (192 * math.pi * math.sin(th) * math.sin(th / 2) ** 2.5),
    }[name]
    lam_direct = 0.5 * math.pi * quad(lambda th: math.sin(th) ** 3 * paper_b(th), 0, math.pi,
                                      limit=200, epsabs=1e-14, epsrel=1e-13)[0]
    assert abs(lam_direct - 1 / 6) < 1e-10
    assert abs(bkw_lambda(kern) - 1 / 6) < 1e-14
    # the t-form of the kernel equals the paper's formula pointwise
    for th in (0.01, 0.3, 1.0, 2.5, 3.1):
        assert abs(kern.b_of_theta(th) - paper_b(th)) < 1e-12 * paper_b(th)


def test_power_kernel_lambda_and_b8_identity():
    for s in (0.0, 0.25, 0.5, 0.75):
        assert abs(bkw_lambda(power_kernel(s)) - 1 / 6) < 1e-14
    assert abs(power_kernel(0.75).c - PAPER_KERNELS["b8"].c) < 1e-17


def test_paper_eps_split_converges_to_exact_weight():
    """The paper's precompute is an approximation of F; its error shrinks with eps."""
    k = power_kernel(0.75)
    x, y = 5.0, 5.0
    exact = psi(x, y, k)
    errs = [abs(F_eps_split(x, y, k, eps=e, n_outer=600) - exact) / abs(exact)
            for e in (math.pi / 100, math.pi / 1000)]
    assert errs[1] < errs[0]
    assert errs[1] < 1e-6
