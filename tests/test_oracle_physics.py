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
