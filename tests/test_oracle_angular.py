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


def _psi_mp(x, y, kern, npts=33):
    r"""eq. FF with the azimuth done (J0) in t = sin^2(th/2), by 30-digit mpmath
    quadrature: 4 pi c \int_0^1 t^{-s} (1-t)^{-r} [e^{2ixt} J0(Y) - 1] / t dt,
    Y = 2 y sqrt(t(1-t)).  The bracket over t is formed without cancellation:
    (J0(Y) - 1)/t = -y^2 (1-t) 1F2(1; 2, 2; -y^2 t(1-t)) and expm1(2ixt)/t; the
    two end panels take t = a u^4 and 1 - t = (1-b) u^4, which makes the
    algebraic end singularities smooth in u."""
    import mpmath as mp
    with mp.workdps(30):
        x, y = mp.mpf(x), mp.mpf(y)
        s, r = mp.mpf(kern.s), mp.mpf(kern.r)

        def f(t, omt):
            j0m1_t = -(y * y) * omt * mp.hyp1f2(1, 2, 2, -(y * y) * t * omt)
            j0 = 1 + t * j0m1_t
            return t ** (-s) * omt ** (-r) * (mp.expm1(2j * x * t) / t * j0 + j0m1_t)

        pts = mp.linspace(0, 1, npts)
        a, b = pts[1], pts[-2]
        tot = (mp.quad(lambda u: f(a * u ** 4, 1 - a * u ** 4) * 4 * a * u ** 3, [0, 1])
               + mp.quad(lambda u: f(1 - (1 - b) * u ** 4, (1 - b) * u ** 4) * 4 * (1 - b) * u ** 3, [0, 1])
               + mp.quad(lambda t: f(t, 1 - t), pts[1:-1]))
        return complex(4 * mp.pi * mp.mpf(kern.c) * tot)


@pytest.mark.parametrize("name", ["s025", "s050", "s075", "b6", "b7"])
def test_against_mpmath_reference(name):
    """Psi of the 64-node Gauss-Jacobi rule against a 30-digit quadrature, over
    the whole range of (x, y) = (a k.sigma, a |k x sigma|) the workloads reach:
    a |k| <= pi R/(2L) sqrt(3) (N/2 - 1) = 42.2 at N = 64, L = 10, R = 5."""
    pytest.importorskip("mpmath")
    kern = {"s025": power_kernel(0.25), "s050": power_kernel(0.5), "s075": power_kernel(0.75),
            "b6": PAPER_KERNELS["b6"], "b7": PAPER_KERNELS["b7"]}[name]
    for x, y in [(0.3, 0.1), (5.0, 2.0), (9.5, 9.5), (42.2, 0.0), (0.0, 42.2), (-29.8, 29.8),
                 (17.0, 38.0), (-40.0, 11.0)]:
        ref = _psi_mp(x, y, kern)
        got = complex(psi(x, y, kern))
        assert abs(got - ref) <= 1e-14 * abs(ref) + 1e-16, (name, x, y, got, ref)


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


# ---------------------------------------------------------------- Debye-Yukawa
def _debye_theta_mp(x, y, theta_cut):
    """eq. FF with the azimuth done (J0), in theta, for eq. ApproximatedDebye:
    2 pi \\int_{theta_cut}^pi |log(2 sin(th/2))| / (2 sin(th/2)) [e^{ix(1-cos th)} J0(y sin th) - 1] d th."""
    import mpmath as mp
    with mp.workdps(30):
        def f(th):
            sb = abs(mp.log(2 * mp.sin(th / 2))) / (2 * mp.sin(th / 2))
            return 2 * mp.pi * sb * (mp.expj(x * (1 - mp.cos(th))) * mp.besselj(0, y * mp.sin(th)) - 1)
        pts = [mp.mpf(theta_cut)] + [mp.pi * k / 24 for k in range(1, 25) if mp.pi * k / 24 > theta_cut]
        return complex(mp.quad(f, pts))


@pytest.mark.parametrize("name", ["debye", "debye_cut"])
def test_debye_against_theta_quadrature(name):
    """The composite rule for the logarithmic weight against a 30-digit
    quadrature of the paper's theta-form, up to x, y ~ 70."""
    pytest.importorskip("mpmath")
    from oracle.angular import DEBYE_KERNELS
    kern = DEBYE_KERNELS[name]
    for x, y in [(0.2, 0.1), (3.0, 2.0), (-12.0, 9.0), (30.0, 25.0), (0.0, 60.0), (70.0, 30.0)]:
        ref = _debye_theta_mp(x, y, kern.theta_cut)
        got = complex(psi(x, y, kern))
        assert abs(got - ref) <= 2e-12 * max(1.0, abs(ref)), (name, x, y, got, ref)


def test_debye_structure():
    from oracle.angular import DEBYE_KERNELS, DebyeKernel
    k0, kc = DEBYE_KERNELS["debye"], DEBYE_KERNELS["debye_cut"]
    assert kc.theta_cut == pytest.approx(math.pi / 10)
    assert psi(0.0, 0.0, k0) == 0.0 and psi(0.0, 0.0, kc) == 0.0
    x = RNG.uniform(-40, 40, 20)
    y = RNG.uniform(0, 40, 20)
    np.testing.assert_allclose(psi(-x, y, k0), np.conj(psi(x, y, k0)), rtol=0, atol=1e-13)
    # the cutoff rule has no node below t_c = sin^2(pi/20); b vanishes there
    t, w = kc.rule()
    assert t.min() >= math.sin(math.pi / 20) ** 2 * (1 - 1e-15)
    assert kc.b_of_theta(0.9 * math.pi / 10) == 0.0
    # sin th b is the paper's expression above the cut
    th = 1.1
    assert abs(kc.b_of_theta(th) * math.sin(th) - abs(math.log(2 * math.sin(th / 2))) / (2 * math.sin(th / 2))) < 1e-15
    # the rule integrates the weight exactly on constants: \int_0^1 |log(2 sqrt t)| (1-t)^{-1/2} dt
    from scipy.integrate import quad
    exact = (quad(lambda t: -math.log(2 * math.sqrt(t)) / math.sqrt(1 - t), 0, 0.25, limit=200)[0]
             + quad(lambda t: math.log(2 * math.sqrt(t)) / math.sqrt(1 - t), 0.25, 1, limit=200)[0])
    assert abs(np.sum(k0.rule()[1]) - exact) < 1e-12
    assert DebyeKernel(0.0).prefactor == math.pi
