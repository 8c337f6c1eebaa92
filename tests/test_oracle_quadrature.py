"""Pins of the oracle's quadrature rules against closed-form integrals.

Gauss-Legendre and Gauss-Jacobi rules must integrate polynomials exactly up to
degree 2n-1 (the property that defines them); the sphere rule must integrate
spherical monomials exactly up to its degree and be centrally symmetric.
"""
import math

import numpy as np
import pytest
from scipy.special import beta as B, gamma as G

from oracle.quadrature import (LEBEDEV_DEGREE, gauss_jacobi_unit, radial_gauss_legendre,
                               sphere_lebedev)


@pytest.mark.parametrize("n", [4, 16, 32, 64])
def test_gauss_legendre_exact_on_polynomials(n):
    R = 4.0
    rho, w = radial_gauss_legendre(n, R)
    assert np.all((rho > 0) & (rho < R))
    for deg in range(0, min(2 * n, 40)):
        exact = R ** (deg + 1) / (deg + 1)
        got = np.sum(w * rho ** deg)
        assert abs(got - exact) <= 1e-13 * exact, (n, deg)


def _sphere_monomial(a, b, c):
    # \int_{S^2} x^a y^b z^c; zero unless all even
    if a % 2 or b % 2 or c % 2:
        return 0.0
    return 2.0 * G((a + 1) / 2) * G((b + 1) / 2) * G((c + 1) / 2) / G((a + b + c + 3) / 2)


@pytest.mark.parametrize("M", [6, 14, 26, 38, 50, 110, 302])
def test_lebedev_exactness_and_symmetry(M):
    s, w = sphere_lebedev(M)
    assert s.shape == (M, 3)
    assert abs(w.sum() - 4 * math.pi) < 1e-13
    np.testing.assert_allclose(np.linalg.norm(s, axis=1), 1.0, atol=1e-15)
    deg = LEBEDEV_DEGREE[M]
    for a in range(deg + 1):
        for b in range(deg + 1 - a):
            for c in range(deg + 1 - a - b):
                got = np.sum(w * s[:, 0] ** a * s[:, 1] ** b * s[:, 2] ** c)
                assert abs(got - _sphere_monomial(a, b, c)) < 1e-13, (M, a, b, c)
    # central symmetry with equal weights (used by the GPU path's antipodal pairing)
    for i in range(M):
        j = np.argmin(np.linalg.norm(s + s[i], axis=1))
        assert np.linalg.norm(s[j] + s[i]) < 1e-14
        assert abs(w[j] - w[i]) < 1e-15


@pytest.mark.parametrize("n,s,r", [(8, 0.5, 0.0), (32, 0.25, 0.0), (64, 0.75, 0.0),
                                   (64, 0.0, 0.5), (64, 0.5, 0.5), (64, -1.0, 0.0)])
def test_gauss_jacobi_exact_on_polynomials(n, s, r):
    t, w = gauss_jacobi_unit(n, s, r)
    assert np.all((t > 0) & (t < 1))
    for k in range(0, min(2 * n, 30)):
        exact = B(k + 1 - s, 1 - r)            # \int_0^1 t^{k-s} (1-t)^{-r} dt
        got = np.sum(w * t ** k)
        assert abs(got - exact) <= 2e-15 * max(1.0, exact) + 1e-15, (n, s, r, k)
