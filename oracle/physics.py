"""Moments, entropy dissipation and the time step of the Galerkin system (CPU, FP64).

* mass rho_N = (2L)^3 f_0 (Remark 4.1);
* momentum and energy \\int Q v, \\int Q |v|^2 and \\int f v, \\int f |v|^2 by the
  trapezoid rule on the N^3 grid (the invariants of Section 1);
* H-functional dissipation D = \\int Q ln f <= 0 (Section 1, H-theorem), summed
  over grid points where f exceeds 1e-14 max f;
* the Galerkin ODE d f_k / dt = Q_k (Section 2) advanced by Heun's method
  (explicit trapezoid): f* = f + dt Q(f), f <- f + dt/2 (Q(f) + Q(f*)), or by
  the classical fourth-order Runge-Kutta method the paper's experiments use
  (Section 5).

Test infrastructure only: nothing in the GPU product path imports this file.
"""
from __future__ import annotations

import math

import numpy as np

from .collision import Discretization, collision_direct


def grid(N: int, L: float) -> np.ndarray:
    return -L + (2.0 * L / N) * np.arange(N)


def to_physical(ghat: np.ndarray, L: float) -> np.ndarray:
    """g(v_j) = sum_k g_k e^{i pi k.v_j / L} on v_j = -L + j 2L/N (real part)."""
    N = ghat.shape[0]
    k = np.fft.fftfreq(N, 1.0 / N).astype(np.int64)
    k[N // 2] = 0
    sgn = np.where(k % 2 == 0, 1.0, -1.0)
    g = ghat * sgn[:, None, None] * sgn[None, :, None] * sgn[None, None, :]
    return np.real(np.fft.ifftn(g)) * float(N) ** 3


def moments(fhat: np.ndarray, L: float):
    """(mass, momentum[3], energy) of the spectral function on the grid."""
    N = fhat.shape[0]
    f = to_physical(fhat, L)
    v = grid(N, L)
    h3 = (2.0 * L / N) ** 3
    V1, V2, V3 = np.meshgrid(v, v, v, indexing="ij")
    mass = (2.0 * L) ** 3 * float(np.real(fhat[0, 0, 0]))
    mom = np.array([h3 * np.sum(f * V1), h3 * np.sum(f * V2), h3 * np.sum(f * V3)])
    energy = h3 * np.sum(f * (V1 ** 2 + V2 ** 2 + V3 ** 2))
    return mass, mom, energy


def entropy_dissipation(qhat: np.ndarray, f_samples: np.ndarray, L: float) -> float:
    """D = h^3 sum_j Q(v_j) ln f(v_j) over f(v_j) > 1e-14 max f."""
    N = qhat.shape[0]
    q = to_physical(qhat, L)
    mask = f_samples > 1e-14 * f_samples.max()
    return float((2.0 * L / N) ** 3 * np.sum(q[mask] * np.log(f_samples[mask])))


def heun_step(fhat: np.ndarray, d: Discretization, dt: float, collide=None, **kw) -> np.ndarray:
    """One Heun step; `collide(f)` replaces Q (default: the direct sum with d)."""
    Q = collide if collide is not None else (lambda g: collision_direct(g, d, **kw))
    q1 = Q(fhat)
    fs = fhat + dt * q1
    q2 = Q(fs)
    return fhat + 0.5 * dt * (q1 + q2)


def rk4_step(fhat: np.ndarray, d: Discretization, dt: float, collide=None, **kw) -> np.ndarray:
    """One classical Runge-Kutta step:
    k1 = Q(f), k2 = Q(f + dt/2 k1), k3 = Q(f + dt/2 k2), k4 = Q(f + dt k3),
    f <- f + dt/6 (k1 + 2 k2 + 2 k3 + k4)."""
    Q = collide if collide is not None else (lambda g: collision_direct(g, d, **kw))
    k1 = Q(fhat)
    k2 = Q(fhat + 0.5 * dt * k1)
    k3 = Q(fhat + 0.5 * dt * k2)
    k4 = Q(fhat + dt * k3)
    return fhat + dt / 6.0 * (k1 + 2.0 * k2 + 2.0 * k3 + k4)
