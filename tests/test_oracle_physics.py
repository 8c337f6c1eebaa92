"""Pins of the oracle's time steps: applied to the scalar linear equation
f' = lam f, one step must multiply f by the method's stability polynomial,
1 + z + z^2/2 (Heun) and 1 + z + z^2/2 + z^3/6 + z^4/24 (classical RK4),
z = lam dt -- the textbook definition of the two methods -- and RK4's error
against the exact exp(z) must fall as dt^5 per step."""
import math

import numpy as np
import pytest

import oracle


@pytest.mark.parametrize("lam", [-0.7, 0.3 + 1.1j, -2.0 - 0.5j])
def test_step_polynomials_on_linear_equation(lam):
    f = np.array([1.0 + 0.25j, -0.5 + 2.0j, 0.125])
    dt = 0.37
    z = lam * dt
    lin = (lambda g: lam * g)
    heun = oracle.heun_step(f, None, dt, collide=lin)
    rk4 = oracle.rk4_step(f, None, dt, collide=lin)
    assert np.allclose(heun, f * (1 + z + z * z / 2), rtol=0, atol=1e-15)
    assert np.allclose(rk4, f * (1 + z + z * z / 2 + z ** 3 / 6 + z ** 4 / 24), rtol=0, atol=1e-15)


def test_rk4_local_error_order():
    lam = -1.3
    errs = []
    for dt in (0.2, 0.1, 0.05):
        one = oracle.rk4_step(np.array([1.0]), None, dt, collide=lambda g: lam * g)[0]
        errs.append(abs(one - math.exp(lam * dt)))
    # local error ~ C dt^5: halving dt divides it by about 32
    assert 25 < errs[0] / errs[1] < 40 and 25 < errs[1] / errs[2] < 40


def test_rk4_on_a_nonlinear_equation():
    """f' = -f^2 (a quadratic right-hand side, like Q): f(t) = f0 / (1 + f0 t);
    100 RK4 steps reach it to 1e-9, Heun's 100 steps only to ~1e-5."""
    f0, T, n = 2.0, 1.0, 100
    quad = (lambda g: -g * g)
    a = b = np.array([f0])
    for _ in range(n):
        a = oracle.rk4_step(a, None, T / n, collide=quad)
        b = oracle.heun_step(b, None, T / n, collide=quad)
    exact = f0 / (1 + f0 * T)
    assert abs(a[0] - exact) < 1e-9
    assert 1e-7 < abs(b[0] - exact) < 1e-4


# --------------------------------------------------------------- diagnostics
def test_to_physical_is_the_trigonometric_sum():
    """to_physical evaluates g(v_j) = sum_k g_k e^{i pi k.v_j / L} (Section 2):
    against the literal sum at every grid point of a 6^3 grid with random
    Hermitian coefficients, and as the inverse of the trapezoid projection of
    the inputs module (round trip to 1e-15 for a band-limited f)."""
    rng = np.random.default_rng(5)
    N, L = 6, 2.5
    ks = np.arange(-N // 2 + 1, N // 2)
    g = np.zeros((N, N, N), np.complex128)
    for k1 in ks:
        for k2 in ks:
            for k3 in ks:
                if (k1, k2, k3) < (0, 0, 0) or (k1, k2, k3) == (0, 0, 0):
                    continue
                c = complex(rng.normal(), rng.normal())
                g[k1 % N, k2 % N, k3 % N] = c
                g[-k1 % N, -k2 % N, -k3 % N] = np.conj(c)
    g[0, 0, 0] = 0.7
    v = -L + (2 * L / N) * np.arange(N)
    lit = np.zeros((N, N, N))
    for a in range(N):
        for b in range(N):
            for c in range(N):
                s = 0j
                for k1 in ks:
                    for k2 in ks:
                        for k3 in ks:
                            s += g[k1 % N, k2 % N, k3 % N] * np.exp(1j * math.pi * (k1 * v[a] + k2 * v[b] + k3 * v[c]) / L)
                lit[a, b, c] = s.real
    phys = oracle.to_physical(g, L)
    assert np.max(np.abs(phys - lit)) < 1e-13
    import workloads
    back = workloads.to_spectral(phys)
    assert np.max(np.abs(back - g)) < 1e-14


def test_moments_of_a_maxwellian_mixture():
    """mass, momentum and energy of sum_i w_i M_{u_i, T_i} are sum w_i,
    sum w_i u_i and sum w_i (|u_i|^2 + 3 T_i) (Section 1).  On a grid wide
    enough (tails e^{-30}) and fine enough that the dropped Nyquist modes are
    e^{-30} of the peak, the trapezoid rule reaches them to ~1e-12."""
    import workloads
    N, L = 64, 10.0
    w = [0.5, 0.3, 0.2]
    u = [(1.5, -0.5, 0.25), (-1.5, 1.0, 0.5), (0.0, 0.75, -1.25)]
    T = [0.6, 1.0, 1.2]
    f = sum(workloads.maxwellian_on_grid(N, L, wi, ui, Ti) for wi, ui, Ti in zip(w, u, T))
    mass, mom, energy = oracle.moments(workloads.to_spectral(f), L)
    assert abs(mass - sum(w)) < 1e-12
    mom_ref = np.sum([wi * np.array(ui) for wi, ui in zip(w, u)], axis=0)
    assert np.max(np.abs(mom - mom_ref)) < 1e-11
    e_ref = sum(wi * (np.dot(ui, ui) + 3 * Ti) for wi, ui, Ti in zip(w, u, T))
    assert abs(energy - e_ref) < 1e-11 * e_ref


def test_bkw_closed_form_is_the_rate_equation():
    """eq. QQ equals lambda (1 - K) d f_BKW / dK (eq. BKW with K' = lambda(1-K)),
    by a central difference in K."""
    lam, K, h = 1.0 / 6.0, 0.66, 1e-5
    v2 = np.array([0.0, 1.0, 4.0, 9.0, 16.0])
    dfdK = (oracle.bkw.f_bkw(v2, K + h) - oracle.bkw.f_bkw(v2, K - h)) / (2 * h)
    q = oracle.bkw.Q_bkw(v2, K, lam)
    # O(h^2) truncation and 1e-16/h rounding of the difference quotient
    assert np.max(np.abs(q - lam * (1 - K) * dfdK)) < 1e-8 * np.max(np.abs(q))


def test_entropy_dissipation_of_bkw_against_radial_integral():
    """D = \\int Q ln f dv for the BKW pair (f, Q) at t = 6.5 (eqs. BKW, QQ):
    the grid functional against the radial integral 4 pi \\int r^2 Q ln f dr by
    adaptive quadrature; D < 0 (H-theorem).  ln f is analytic in a strip of
    half-width 0.77 (the zeros of the bracket of eq. BKW at r^2 = -0.6), so
    the trapezoid sum errs by about e^{-2 pi 0.77 / h}: 4e-9 at h = 1/4."""
    from scipy.integrate import quad
    lam = 1.0 / 6.0
    K = 1.0 - math.exp(-6.5 * lam)
    ref = 4 * math.pi * quad(lambda r: r * r * oracle.bkw.Q_bkw(r * r, K, lam) * math.log(oracle.bkw.f_bkw(r * r, K)),
                             0, 12, limit=400, epsabs=1e-15, epsrel=1e-13)[0]
    N, L = 64, 8.0
    f = oracle.bkw.on_grid(oracle.bkw.f_bkw, N, L, K)
    q = oracle.bkw.on_grid(oracle.bkw.Q_bkw, N, L, K, lam)
    import workloads
    D = oracle.entropy_dissipation(workloads.to_spectral(q), f, L)
    assert ref < 0 and D < 0
    assert abs(D - ref) < 1e-8 * abs(ref), (D, ref)
