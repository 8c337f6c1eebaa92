"""Quadrature rules used by the fast method's low-rank split of the weight G.

Section 4 (eq. approxG): the radial integral over |q| in [0, R] uses
N_|q| = O(N) Gauss-Legendre points; the integral over the direction q-hat in
S^2 uses a spherical rule (the paper uses spherical designs, which are not
available here; Lebedev rules of the requested size stand in for them).

The angular weight F (eq. FF) is a 1-D integral in t = sin^2(theta/2) once the
azimuth has been integrated exactly; its weight t^{-s} (1-t)^{-r} is handled by
Gauss-Jacobi quadrature on [0, 1].

Test infrastructure only: nothing in the GPU product path imports this file.
"""
from __future__ import annotations

import functools

import numpy as np
from numpy.polynomial.legendre import leggauss
from scipy.integrate import lebedev_rule
from scipy.special import roots_jacobi

# Lebedev size -> algebraic degree of exactness (rules available in SciPy)
LEBEDEV_DEGREE = {
    6: 3, 14: 5, 26: 7, 38: 9, 50: 11, 74: 13, 86: 15, 110: 17, 146: 19,
    170: 21, 194: 23, 230: 25, 266: 27, 302: 29, 350: 31,
}


def radial_gauss_legendre(n: int, R: float):
    """n-point Gauss-Legendre nodes rho_p and weights w_p on [0, R] (eq. approxG)."""
    x, w = leggauss(n)
    return 0.5 * R * (x + 1.0), 0.5 * R * w


@functools.lru_cache(maxsize=None)
def _lebedev(M: int):
    if M not in LEBEDEV_DEGREE:
        raise ValueError(f"no Lebedev rule with {M} points")
    x, w = lebedev_rule(LEBEDEV_DEGREE[M])
    sig = np.ascontiguousarray(x.T, dtype=np.float64)       # [M, 3]
    sig /= np.linalg.norm(sig, axis=1, keepdims=True)
    return sig, np.asarray(w, dtype=np.float64)


def sphere_lebedev(M: int):
    """M-point Lebedev rule on S^2: unit points [M,3] and weights summing to 4 pi."""
    s, w = _lebedev(M)
    return s.copy(), w.copy()


def _refine_jacobi(n: int, alpha: float, beta: float, u0: np.ndarray):
    """Newton-polish Gauss-Jacobi nodes in 40-digit arithmetic and recompute the
    weights from the classical formula
        w_i = 2^{a+b+1} G(n+a+1) G(n+b+1) / (G(n+a+b+1) n!) / ((1-u_i^2) P_n'(u_i)^2).
    (SciPy's double-precision weights are good to ~1e-12 only.)"""
    import mpmath as mp
    with mp.workdps(40):
        a, b = mp.mpf(alpha), mp.mpf(beta)

        def p_and_dp(x):
            # three-term recurrence for P_k^{(a,b)}(x)
            p0 = mp.mpf(1)
            p1 = (a - b) / 2 + (a + b + 2) * x / 2
            if n == 1:
                pn, pm = p1, p0
            else:
                pm, pn = p0, p1
                for k in range(2, n + 1):
                    c = 2 * k + a + b
                    a1 = 2 * k * (k + a + b) * (c - 2)
                    a2 = (c - 1) * (a * a - b * b)
                    a3 = (c - 2) * (c - 1) * c
                    a4 = 2 * (k + a - 1) * (k + b - 1) * c
                    pm, pn = pn, ((a2 + a3 * x) * pn - a4 * pm) / a1
            # derivative: (2n+a+b)(1-x^2) P_n' = n[(a-b) - (2n+a+b) x] P_n + 2(n+a)(n+b) P_{n-1}
            c = 2 * n + a + b
            dp = (n * ((a - b) - c * x) * pn + 2 * (n + a) * (n + b) * pm) / (c * (1 - x * x))
            return pn, dp

        const = (mp.mpf(2) ** (a + b + 1) * mp.gamma(n + a + 1) * mp.gamma(n + b + 1)
                 / (mp.gamma(n + a + b + 1) * mp.factorial(n)))
        us, ws = [], []
        for x0 in u0:
            x = mp.mpf(float(x0))
            for _ in range(6):
                pn, dp = p_and_dp(x)
                dx = pn / dp
                x -= dx
                if abs(dx) < mp.mpf(10) ** -38:
                    break
            pn, dp = p_and_dp(x)
            us.append(x)
            ws.append(const / ((1 - x * x) * dp * dp))
        return us, ws


@functools.lru_cache(maxsize=None)
def _jacobi01(n: int, s: float, r: float):
    # weight (1-u)^alpha (1+u)^beta on [-1,1] with alpha = -r, beta = -s;
    # u = 2t - 1 maps it to 2^{alpha+beta} (1-t)^alpha t^beta on [0,1], dt = du/2
    import mpmath as mp
    u0, _ = roots_jacobi(n, -r, -s)
    us, ws = _refine_jacobi(n, -r, -s, u0)
    with mp.workdps(40):
        scale = mp.mpf(2) ** (mp.mpf(r) + mp.mpf(s) - 1)
        t = np.array([float((u + 1) / 2) for u in us])
        w = np.array([float(wi * scale) for wi in ws])
    return t, w


def gauss_jacobi_unit(n: int, s: float, r: float = 0.0):
    """n-point Gauss rule for \\int_0^1 t^{-s} (1-t)^{-r} g(t) dt."""
    t, w = _jacobi01(int(n), float(s), float(r))
    return t.copy(), w.copy()
