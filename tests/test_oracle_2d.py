"""Pins of the two-dimensional oracle (d = 2, Section 5.2) against routes that
share none of its arithmetic.

* the angular weight F (eq. FF2D1):
  - for constant b, the closed form of eq. cutoff2D (Bessel J0);
  - for b1-b4, a 50-digit mpmath quadrature in theta of eq. FF2D1 with the
    two halves of the circle folded together (theta and 2 pi - theta), which is
    what makes the integral converge for nu >= 1;
  - F(0) = 0, F(-x, y) = conj F(x, y), F(x, -y) = F(x, y);
  - the paper's own precompute (epsilon split with Taylor ends, Section 4.1)
    converges to it as epsilon shrinks;
* the kernels of Section 5.2 as typed from their theta-forms, and their common
  BKW rate lambda = 1/8 (eq. KK2) by scipy quadrature of its definition;
* a literal loop over eq. sum with G(l, m) of eq. GG and F integrated over the
  circle as in eq. FF (absolute angle, no change of variable) on a 4^2 grid;
* the invariants of the discrete operator: Q_0 = 0 exactly, Q(-k) = conj Q(k),
  momentum and energy to spectral accuracy, Q(M, M) ~ 0 for a Maxwellian, bilinearity;
* the BKW solution (Section 5.1 with d = 2) and the printed Table 1.
"""
import math
import os

import numpy as np
import pytest
from scipy.integrate import quad

import workloads
from oracle import collision2d as o2

HERE = os.path.dirname(os.path.abspath(__file__))
RNG = np.random.default_rng(2020)
KERNELS = ["b1", "b2", "b3", "b4"]
R_BKW = 6.0
L_BKW = (3 + math.sqrt(2)) * R_BKW / 4


# ------------------------------------------------------------ angular weight
def test_cutoff_closed_form():
    C = 1.0 / (2.0 * math.pi)
    kern = o2.PAPER_KERNELS_2D["b1"]
    assert kern.s == -1.0 and kern.r == 0.0 and kern.c == C
    x = RNG.uniform(-62, 62, 300)
    y = RNG.uniform(-62, 62, 300)
    got = o2.psi2d(x, y, kern)
    ref = o2.psi2d_cutoff_closed_form(x, y, C)
    assert np.max(np.abs(got - ref)) < 1e-13


def _F_theta_mp(x, y, kern, dps=50):
    """eq. FF2D1 in theta, the integrand at theta and 2 pi - theta added:
    2 \\int_0^pi b(cos th) [ e^{i x (1 - cos th)} cos(y sin th) - 1 ] d th,
    with b(cos th) = c sin^{-2-2s}(th/2) cos^{-2r}(th/2)."""
    import mpmath as mp
    with mp.workdps(dps):
        c, s, r = mp.mpf(kern.c), mp.mpf(kern.s), mp.mpf(kern.r)
        xm, ym = mp.mpf(x), mp.mpf(y)

        def f(th):
            b = c * mp.sin(th / 2) ** (-2 - 2 * s) * mp.cos(th / 2) ** (-2 * r)
            return 2 * b * (mp.expj(xm * (1 - mp.cos(th))) * mp.cos(ym * mp.sin(th)) - 1)

        return complex(mp.quad(f, [0, mp.pi / 8, mp.pi / 2, mp.pi]))


@pytest.mark.parametrize("name", KERNELS)
def test_theta_quadrature_50_digits(name):
    pytest.importorskip("mpmath")
    kern = o2.PAPER_KERNELS_2D[name]
    pts = [(0.3, 0.0), (0.0, 0.7), (1.7, -2.3), (-4.1, 3.3), (9.5, 0.2), (-13.0, -11.0), (30.0, 21.0)]
    for x, y in pts:
        ref = _F_theta_mp(x, y, kern)
        got = complex(o2.psi2d(x, y, kern))
        assert abs(got - ref) <= 1e-12 * max(1.0, abs(ref)), (name, x, y, got, ref)


@pytest.mark.parametrize("name", KERNELS)
def test_symmetries_and_zero(name):
    kern = o2.PAPER_KERNELS_2D[name]
    x = RNG.uniform(-40, 40, 64)
    y = RNG.uniform(-40, 40, 64)
    F = o2.psi2d(x, y, kern)
    np.testing.assert_allclose(o2.psi2d(-x, y, kern), np.conj(F), rtol=0, atol=1e-13 * np.abs(F).max())
    np.testing.assert_allclose(o2.psi2d(x, -y, kern), F, rtol=0, atol=1e-13 * np.abs(F).max())
    assert o2.psi2d(0.0, 0.0, kern) == 0.0


@pytest.mark.parametrize("name", KERNELS)
def test_paper_eps_split_converges_to_exact_weight(name):
    """Section 4.1's 2-D precompute: the Taylor ends drop the terms of order three
    and up; the odd ones cancel between the two ends, so the first one left is of
    order theta^4, and against b ~ theta^(-2-2s) it costs O(eps^(3-2s)).  A tenfold
    smaller eps must shrink the error by that order (10^5 for b1 .. 316 for b4)."""
    kern = o2.PAPER_KERNELS_2D[name]
    order = 3.0 - 2.0 * kern.s
    for x, y in ((5.0, 3.0), (-2.0, 9.0)):
        exact = complex(o2.psi2d(x, y, kern))
        errs = [abs(o2.F2d_eps_split(x, y, kern, eps=e, n_outer=600) - exact) / abs(exact)
                for e in (math.pi / 100, math.pi / 1000)]
        assert 0.7 * 10 ** order < errs[0] / errs[1] < 1.4 * 10 ** order, (name, x, y, errs)
        assert errs[1] < 1e-5, (name, x, y, errs)


# ------------------------------------------------------------ kernels, lambda
_THETA_FORMS = {
    "b1": lambda th: 1.0 / (2.0 * math.pi),
    "b2": lambda th: 3.0 / (32.0 * math.sin(th / 2)),
    "b3": lambda th: 1.0 / (8.0 * math.pi * math.sin(th / 2) ** 2),
    "b4": lambda th: 5.0 * abs(math.cos(th / 2)) / (256.0 * math.sin(th / 2) ** 2.5),
}


@pytest.mark.parametrize("name", KERNELS)
def test_kernels_and_bkw_rate(name):
    """eq. b1-b4 typed from their theta-forms; lambda = 1/4 \\int (1 - cos^2) b = 1/8 (eq. KK2)."""
    kern = o2.PAPER_KERNELS_2D[name]
    b = _THETA_FORMS[name]
    for th in (0.05, 0.7, 1.9, 3.0, 4.4, 6.1):
        t = math.sin(th / 2) ** 2
        assert abs(kern.c * t ** (-1 - kern.s) * (1 - t) ** (-kern.r) - b(th)) <= 1e-14 * b(th)
    # theta = u^2 near 0 and theta = 2 pi - u^2 near 2 pi take out the endpoint singularity
    half = quad(lambda u: 2 * u * math.sin(u * u) ** 2 * b(u * u), 0, math.sqrt(math.pi),
                epsabs=1e-15, epsrel=1e-13, limit=200)[0]
    other = quad(lambda u: 2 * u * math.sin(2 * math.pi - u * u) ** 2 * b(2 * math.pi - u * u), 0,
                 math.sqrt(math.pi), epsabs=1e-15, epsrel=1e-13, limit=200)[0]
    assert abs(0.25 * (half + other) - 0.125) < 1e-11
    assert abs(o2.bkw_lambda_2d(kern, n=16) - 0.125) < 1e-13


def test_bkw2d_Q_is_lambda_times_dK():
    """eq. QQ (d = 2) equals lambda (1 - K) d f / dK of the BKW profile (eq. BKW with
    eq. KK2), by central differences."""
    K, lam, h = 0.6, 0.125, 1e-5
    for v2 in (0.0, 0.4, 1.0, 2.5, 6.0):
        dfdK = (o2.bkw2d_f(v2, K + h) - o2.bkw2d_f(v2, K - h)) / (2 * h)
        assert abs(o2.bkw2d_Q(v2, K, lam) - lam * (1 - K) * dfdK) < 1e-9
    # K(t) solves K' = lambda (1 - K) with K(0) = 1/2
    t = 3.0
    dK = (o2.bkw2d_K(t + 1e-5) - o2.bkw2d_K(t - 1e-5)) / 2e-5
    assert abs(dK - 0.125 * (1 - o2.bkw2d_K(t))) < 1e-10
    assert o2.bkw2d_K(0.0) == 0.5


# ------------------------------------------------------------ the direct sum
def _F_circle(k, a, qhat, kern):
    """eq. FF: \\int_{S^1} b(sigma.qhat) (e^{i a k.(qhat - sigma)} - 1) d sigma with sigma =
    (cos phi, sin phi), b written through t = (1 - sigma.qhat)/2 = sin^2(th/2)."""
    th0 = math.atan2(qhat[1], qhat[0])

    def integrand(phi, part):
        s = (math.cos(phi), math.sin(phi))
        t = 0.5 * (1.0 - (s[0] * qhat[0] + s[1] * qhat[1]))
        b = kern.c * t ** (-1 - kern.s) * (1 - t) ** (-kern.r)
        z = a * (k[0] * (qhat[0] - s[0]) + k[1] * (qhat[1] - s[1]))
        return b * (math.cos(z) - 1.0) if part == 0 else b * math.sin(z)

    opts = dict(epsabs=1e-14, epsrel=1e-13, limit=400)
    re = quad(integrand, th0, th0 + 2 * math.pi, args=(0,), **opts)[0]
    im = quad(integrand, th0, th0 + 2 * math.pi, args=(1,), **opts)[0]
    return re + 1j * im


@pytest.mark.parametrize("name", ["b1", "b2"])
def test_literal_sum_on_4square(name):
    """eq. sum as a loop over l + m = k, G(l, m) of eq. GG with the radial and
    circle rules, F from eq. FF.  (b3, b4 are not absolutely integrable in the
    unfolded form; their F is pinned by the theta quadrature above.)"""
    N, L, R, gamma = 4, 3.0, 2.0, 0.5
    kern = o2.PAPER_KERNELS_2D[name]
    d = o2.Discretization2D(N, L, R, gamma, kern, 3, 6)
    f = workloads.to_spectral_2d(RNG.uniform(0.5, 1.5, (N, N)))
    Q = o2.collision_direct2d(f, d)
    rho, wr = np.polynomial.legendre.leggauss(3)
    rho, wr = 0.5 * R * (rho + 1), 0.5 * R * wr
    modes = [(a, b) for a in (-1, 0, 1) for b in (-1, 0, 1)]
    Fc = {}
    for k in modes:
        acc = 0.0j
        for m in modes:
            l = (k[0] - m[0], k[1] - m[1])
            if l not in modes:
                continue
            G = 0.0j
            for p in range(3):
                for q in range(6):
                    th = (q + 0.5) * 2 * math.pi / 6
                    qh = (math.cos(th), math.sin(th))
                    key = (k, p, q)
                    if key not in Fc:
                        Fc[key] = _F_circle(k, math.pi * rho[p] / (2 * L), qh, kern)
                    G += (wr[p] * (2 * math.pi / 6) * rho[p] ** (1 + gamma)
                          * np.exp(-1j * math.pi / L * rho[p] * (m[0] * qh[0] + m[1] * qh[1])) * Fc[key])
            acc += G * f[l] * f[m]
        assert abs(acc - Q[k]) <= 1e-11 * np.abs(Q).max(), (k, acc, Q[k])


@pytest.fixture(scope="module")
def q16():
    N, L, R = 16, 8.0, 4.0
    d = o2.Discretization2D(N, L, R, 0.0, o2.PAPER_KERNELS_2D["b3"], 16, 32)
    f = workloads.to_spectral_2d(workloads.random_mixture_2d(5, N, L))
    return d, f, o2.collision_direct2d(f, d)


def _moments_of(g_phys, N, L):
    v = workloads.velocity_grid(N, L)
    h2 = (2 * L / N) ** 2
    v1, v2 = v[:, None], v[None, :]
    return (h2 * np.sum(g_phys), h2 * np.sum(g_phys * v1), h2 * np.sum(g_phys * v2),
            h2 * np.sum(g_phys * (v1 ** 2 + v2 ** 2)))


def test_invariants(q16):
    d, f, Q = q16
    N = d.N
    assert Q[0, 0] == 0.0                                    # mass (Remark 4.1)
    k = np.arange(N)
    mirror = Q[np.ix_((-k) % N, (-k) % N)]
    np.testing.assert_allclose(mirror, np.conj(Q), rtol=0, atol=1e-15 * np.abs(Q).max())
    assert np.all(Q[N // 2, :] == 0) and np.all(Q[:, N // 2] == 0)
    m0, _, _, _ = _moments_of(o2.to_physical2d(Q, d.L), N, d.L)
    assert abs(m0) < 1e-14 * np.abs(Q).max() * (2 * d.L) ** 2


def test_momentum_and_energy_spectrally_conserved():
    """Momentum and energy of Q (trapezoid rule on the grid) vanish to the
    truncation error of the input, which falls spectrally with N (Section 4)."""
    L = 8.0
    out = {}
    for N in (24, 32):
        v = workloads.velocity_grid(N, L)
        f = sum(w * np.exp(-((v[:, None] - u0) ** 2 + (v[None, :] - u1) ** 2) / 2) / (2 * math.pi)
                for w, u0, u1 in [(0.45, 1.2, 0.5), (0.55, -1.2, -0.3)])
        d = o2.Discretization2D(N, L, 4.0, 0.0, o2.PAPER_KERNELS_2D["b3"], N, 32)
        Q = o2.collision_direct2d(workloads.to_spectral_2d(f), d)
        _, m1, m2, en = _moments_of(o2.to_physical2d(Q, L), N, L)
        _, _, _, en_f = _moments_of(f, N, L)
        out[N] = max(abs(m1), abs(m2), abs(en)) / en_f
        if N == 24:
            # a Maxwellian is an equilibrium: Q(M, M) ~ 0 up to the same truncation error
            M = np.exp(-((v[:, None] - 0.4) ** 2 + (v[None, :] + 0.3) ** 2) / 2.6) / (math.pi * 2.6)
            QM = o2.collision_direct2d(workloads.to_spectral_2d(M), d)
            assert np.linalg.norm(QM) < 1e-3 * np.linalg.norm(Q)
    assert out[32] < out[24] / 30
    assert out[32] < 1e-7


def test_bilinear_scaling(q16):
    d, f, Q = q16
    np.testing.assert_allclose(o2.collision_direct2d(2.5 * f, d), 6.25 * Q, rtol=0,
                               atol=1e-13 * np.abs(Q).max())


# ------------------------------------------------------------ Table 1
def table1():
    rows = {}
    for line in open(os.path.join(HERE, "golden", "table1_2d.txt")):
        if line.strip() and not line.startswith("#"):
            parts = line.split()
            rows[int(parts[0])] = dict(zip(KERNELS, map(float, parts[1:])))
    return rows


def bkw_table1_error(Q, N, centred=True):
    """L_inf over the N^2 grid of Q_num(v_j) - Q_exact(v_j) at t = 0 (K = 1/2);
    the cell-centred grid v_j = -L + (j + 1/2) h by default."""
    v = workloads.velocity_grid(N, L_BKW, centred)
    v2 = v[:, None] ** 2 + v[None, :] ** 2
    return float(np.max(np.abs(o2.to_physical2d(Q, L_BKW, centred) - o2.bkw2d_Q(v2, o2.bkw2d_K(0.0)))))


def test_centred_grid_transforms():
    """On the cell-centred grid v_j = -L + (j + 1/2) h: to_physical2d against the
    literal sum of g_k e^{i pi k.v_j / L}, and the projection of the inputs
    module as its inverse for a band-limited g."""
    rng = np.random.default_rng(3)
    N, L = 8, 3.0
    ks = np.arange(-N // 2 + 1, N // 2)
    g = np.zeros((N, N), np.complex128)
    for k1 in ks:
        for k2 in ks:
            if (k1, k2) <= (0, 0):
                continue
            c = complex(rng.normal(), rng.normal())
            g[k1 % N, k2 % N] = c
            g[-k1 % N, -k2 % N] = np.conj(c)
    g[0, 0] = 0.4
    v = workloads.velocity_grid(N, L, centred=True)
    assert abs(v[0] + L - L / N) < 1e-15 and abs(v.sum()) < 1e-13
    lit = np.array([[sum(g[k1 % N, k2 % N] * np.exp(1j * math.pi * (k1 * a + k2 * b) / L)
                         for k1 in ks for k2 in ks).real for b in v] for a in v])
    phys = o2.to_physical2d(g, L, centred=True)
    assert np.max(np.abs(phys - lit)) < 1e-13
    assert np.max(np.abs(workloads.to_spectral_2d(phys, centred=True) - g)) < 1e-14


@pytest.mark.parametrize("N", [8, 16])
def test_table1_small_grids(N):
    """Table 1 at N = 8, 16 (all four kernels), where the error is the truncation
    of the narrow initial profile (K = 1/2).  With f sampled, and the error
    taken, on the cell-centred grid v_j = -L + (j + 1/2) h, the printed values
    are reproduced to within 15% (measured 0.87-1.05 of the printed value);
    on the grid v_j = -L + j h they come out 3.4-12x larger, because that grid
    holds the point v = 0 where the truncated profile errs most."""
    ref = table1()[N]
    f = workloads.to_spectral_2d(workloads.bkw2d_profile_on_grid(N, L_BKW, o2.bkw2d_K(0.0), centred=True),
                                 centred=True)
    errs = {}
    for name in KERNELS:
        d = o2.Discretization2D(N, L_BKW, R_BKW, 0.0, o2.PAPER_KERNELS_2D[name], N, 32)
        errs[name] = bkw_table1_error(o2.collision_direct2d(f, d), N)
        print(N, name, f"{errs[name]:.4e}", "paper", f"{ref[name]:.4e}")
    for name in KERNELS:
        assert 0.8 < errs[name] / ref[name] < 1.2, (name, errs[name], ref[name])
