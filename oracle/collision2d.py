"""The two-dimensional operator (d = 2) by direct summation (CPU, FP64).

Same construction as the 3-D oracle (`collision`), with the circle in place of
the sphere:

    Q_k = sum_j T_j(k) sum_{m in K_N, k-m in K_N} e^{-i pi rho_j m.sigma_j / L} f_{k-m} f_m,
    T_j(k) = w_p w_q rho_p^{1+gamma} F(k, rho_p, sigma_q)          (eq. realQ, d - 1 = 1),

K_N = {-N/2+1 .. N/2-1}^2, a Gauss-Legendre rule in |q| on [0, R] and the
midpoint rule with N_sigma points on the circle (the paper's choice for its
2-D tests, Section 5.2).  The angular weight (eq. FF2D1) with sigma written
in the frame (q, q_perp) and the two halves of the circle folded together is

    F = 2 \\int_0^pi b(cos th) [ e^{i x (1 - cos th)} cos(y sin th) - 1 ] d th,
    x = a k.q,  y = a k.q_perp,  a = pi |q| / (2L),

and with t = sin^2(th/2), for b = c t^{-1-s} (1-t)^{-r},

    F = 2 c \\int_0^1 t^{-(s+1/2)} (1-t)^{-(r+1/2)} K(t) dt,
    K(t) = [ e^{2ixt} cos(Y) - 1 ] / t,   Y = 2 y sqrt(t (1-t)),

a smooth integrand handled by Gauss-Jacobi quadrature (needs s, r < 1/2; the
paper's 2-D kernels b1-b4 all qualify).  Pinned by the cutoff closed form
(eq. cutoff2D), a 50-digit quadrature of eq. FF2D1 in theta, the BKW rate
lambda = 1/8 of Section 5.2, a literal loop over eq. sum with F integrated
over the circle as in eq. FF, the invariants, and the paper's Table 1.
`F2d_eps_split` is the paper's own approximate precompute of F (Section 4.1),
kept as a labelled variant whose convergence to `psi2d` is measured.

Test infrastructure only: nothing in the GPU product path imports this file.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional

import numpy as np

from .angular import AngularKernel
from .quadrature import gauss_jacobi_unit, radial_gauss_legendre

# The paper's 2-D kernels of Section 5.2, in t = sin^2(th/2):
#   b1 = 1/(2 pi)                                   c = 1/(2 pi), s = -1
#   b2 = 3/(32 sin(th/2))            = 3/32 t^{-1/2}              s = -1/2
#   b3 = 1/(8 pi sin^2(th/2))        = t^{-1}/(8 pi)              s = 0
#   b4 = 5|cos(th/2)|/(256 sin^{5/2}(th/2)) = 5/256 t^{-5/4} (1-t)^{1/2}   s = 1/4, r = -1/2
PAPER_KERNELS_2D = {
    "b1": AngularKernel(c=1.0 / (2.0 * math.pi), s=-1.0, r=0.0, name="b1"),
    "b2": AngularKernel(c=3.0 / 32.0, s=-0.5, r=0.0, name="b2"),
    "b3": AngularKernel(c=1.0 / (8.0 * math.pi), s=0.0, r=0.0, name="b3"),
    "b4": AngularKernel(c=5.0 / 256.0, s=0.25, r=-0.5, name="b4"),
}


def _c1m(Y):
    """(1 - cos Y) / Y^2 (even in Y), with the power series below |Y| = 2."""
    Y = np.abs(np.asarray(Y, dtype=np.float64))
    out = np.empty_like(Y)
    small = Y < 2.0
    z = Y[small] ** 2
    # (1 - cos Y)/Y^2 = sum_{k>=1} (-1)^{k+1} Y^{2k-2} / (2k)!, Horner in Y^2
    coef = [(-1.0) ** (k + 1) / math.factorial(2 * k) for k in range(1, 14)]
    acc = np.full_like(z, coef[-1])
    for cf in coef[-2::-1]:
        acc = acc * z + cf
    out[small] = acc
    Yl = Y[~small]
    out[~small] = (1.0 - np.cos(Yl)) / (Yl * Yl)
    return out


def psi2d(x, y, kern: AngularKernel, n_jacobi: int = 64):
    """F(k, |q|, q) in 2-D as a function of x = a k.q and y = a k.q_perp."""
    if not (kern.s < 0.5 and kern.r < 0.5):
        raise ValueError("the 2-D weight needs s < 1/2 and r < 1/2")
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    shape = np.broadcast(x, y).shape
    x = np.broadcast_to(x, shape).reshape(-1)
    y = np.broadcast_to(y, shape).reshape(-1)
    t, w = gauss_jacobi_unit(n_jacobi, kern.s + 0.5, kern.r + 0.5)
    out = np.empty(x.shape, dtype=np.complex128)
    step = max(1, 2_000_000 // len(t))
    for i0 in range(0, x.size, step):
        xs = x[i0:i0 + step, None]
        ys = y[i0:i0 + step, None]
        tt = t[None, :]
        xt = xs * tt
        Y = 2.0 * ys * np.sqrt(tt * (1.0 - tt))
        cY = np.cos(Y)
        K_re = -2.0 * np.sin(xt) ** 2 / tt * cY - 4.0 * ys * ys * (1.0 - tt) * _c1m(Y)
        K_im = np.sin(2.0 * xt) / tt * cY
        out[i0:i0 + step] = (K_re @ w) + 1j * (K_im @ w)
    out *= 2.0 * kern.c
    return out.reshape(shape)


def psi2d_cutoff_closed_form(x, y, C):
    """Eq. cutoff2D: b = C gives F = 2 pi C [ e^{ix} J0(sqrt(x^2 + y^2)) - 1 ]."""
    from scipy.special import j0
    return 2.0 * math.pi * C * (np.exp(1j * np.asarray(x)) * j0(np.hypot(x, y)) - 1.0)


def F2d_eps_split(x, y, kern: AngularKernel, eps: float = math.pi / 1000, n_outer: int = 400):
    """The paper's 2-D precompute (Section 4.1): on [0, eps] and [2 pi - eps, 2 pi]
    the exponential of eq. FF2D1 is replaced by its second-order Taylor
    polynomial and integrated exactly; [eps, 2 pi - eps] by plain quadrature.
    An approximation of F whose error is reported, not used for parity.

    The two end pieces together (the odd terms in y cancel): in t = sin^2(th/2),
    4c \\int_0^{t_eps} t^{-s-1/2}(1-t)^{-r-1/2} [ i x - x^2 t - y^2 (1-t) ] dt,
    written with incomplete beta functions (needs s, r < 1/2)."""
    from numpy.polynomial.legendre import leggauss
    from scipy.special import beta as beta_fn, betainc
    s, r, c = kern.s, kern.r, kern.c
    te = math.sin(0.5 * eps) ** 2

    def ib(p_, q_):   # \\int_0^te t^{p-1} (1-t)^{q-1} dt
        return betainc(p_, q_, te) * beta_fn(p_, q_)

    ends = 4.0 * c * (1j * x * ib(0.5 - s, 0.5 - r) - x * x * ib(1.5 - s, 0.5 - r) - y * y * ib(0.5 - s, 1.5 - r))
    u, wu = leggauss(n_outer)
    mid = 0.0j
    for a, b_ in ((eps, math.pi), (math.pi, 2.0 * math.pi - eps)):
        th = a + 0.5 * (b_ - a) * (u + 1.0)
        t = np.sin(0.5 * th) ** 2
        bb = c * t ** (-1.0 - s) * (1.0 - t) ** (-r)
        mid += 0.5 * (b_ - a) * np.sum(wu * bb * (np.exp(1j * (x * (1 - np.cos(th)) - y * np.sin(th))) - 1.0))
    return ends + mid


def bkw_lambda_2d(kern: AngularKernel, n: int = 200) -> float:
    """lambda = 1/4 \\int_{S^1} (1 - cos^2 th) b d sigma (Section 5.1, d = 2), in t:
    sin^2 th = 4 t (1-t), d th = dt / sqrt(t(1-t)) on each half circle."""
    # integrand b sin^2 th / sqrt(t(1-t)) = 4 c t^{-s-1/2} (1-t)^{-r+1/2}, times 2 half circles
    t, w = gauss_jacobi_unit(n, kern.s + 0.5, kern.r - 0.5)
    return float(0.25 * 2.0 * 4.0 * kern.c * np.sum(w))


@dataclasses.dataclass(frozen=True)
class Discretization2D:
    N: int
    L: float
    R: float
    gamma: float
    kernel: AngularKernel
    N_rho: int
    N_sigma: int
    n_jacobi: int = 64


def mode_vectors2d(N: int) -> np.ndarray:
    """All k in K_N (2-D) as an integer array [(N-1)^2, 2], k1 slowest."""
    r = np.arange(-N // 2 + 1, N // 2, dtype=np.int64)
    g = np.stack(np.meshgrid(r, r, indexing="ij"), axis=-1)
    return g.reshape(-1, 2)


def circle_midpoint(n: int):
    """Midpoint rule on the circle: sigma_q = (cos th_q, sin th_q), th_q = (q + 1/2) 2 pi / n."""
    th = (np.arange(n) + 0.5) * (2.0 * math.pi / n)
    return np.stack([np.cos(th), np.sin(th)], axis=-1), np.full(n, 2.0 * math.pi / n)


def quadrature_nodes2d(d: Discretization2D):
    rho, wr = radial_gauss_legendre(d.N_rho, d.R)
    sig, ws = circle_midpoint(d.N_sigma)
    rho_j = np.repeat(rho, d.N_sigma)
    wr_j = np.repeat(wr, d.N_sigma)
    sig_j = np.tile(sig, (d.N_rho, 1))
    ws_j = np.tile(ws, d.N_rho)
    return rho_j, sig_j, wr_j * ws_j * rho_j ** (1.0 + d.gamma)


def weight_table2d(d: Discretization2D, k_out: np.ndarray) -> np.ndarray:
    rho, sig, wq = quadrature_nodes2d(d)
    a = math.pi * rho / (2.0 * d.L)
    kf = k_out.astype(np.float64)
    x = a[:, None] * (sig @ kf.T)
    perp = np.stack([-sig[:, 1], sig[:, 0]], axis=-1)
    y = a[:, None] * (perp @ kf.T)
    return wq[:, None] * psi2d(x, y, d.kernel, d.n_jacobi)


def collision_direct2d(fhat: np.ndarray, d: Discretization2D, k_out: Optional[np.ndarray] = None,
                       T: Optional[np.ndarray] = None, k_block: int = 512, j_block: int = 512):
    """Q_k for k_out [nk,2] (default all of K_N, returned N^2 in FFT order)."""
    N = d.N
    fhat = np.asarray(fhat, dtype=np.complex128)
    full = k_out is None
    if full:
        k_out = mode_vectors2d(N)
    k_out = np.asarray(k_out, dtype=np.int64).reshape(-1, 2)
    m = mode_vectors2d(N)
    fm = fhat[tuple(np.mod(m, N).T)]
    rho, sig, _ = quadrature_nodes2d(d)
    if T is None:
        T = weight_table2d(d, k_out)
    h = N // 2
    mdot = sig @ m.T.astype(np.float64)
    Q = np.zeros(len(k_out), dtype=np.complex128)
    for k0 in range(0, len(k_out), k_block):
        kb = k_out[k0:k0 + k_block]
        diff = kb[None, :, :] - m[:, None, :]
        valid = np.all(np.abs(diff) <= h - 1, axis=-1)
        fkm = fhat[tuple(np.mod(diff, N).transpose(2, 0, 1))]
        C = np.where(valid, fkm, 0.0) * fm[:, None]
        acc = np.zeros(len(kb), dtype=np.complex128)
        for j0 in range(0, len(rho), j_block):
            E = np.exp((-1j * math.pi / d.L) * rho[j0:j0 + j_block, None] * mdot[j0:j0 + j_block])
            acc += np.sum(T[j0:j0 + j_block, k0:k0 + k_block] * (E @ C), axis=0)
        Q[k0:k0 + k_block] = acc
    if not full:
        return Q
    out = np.zeros((N, N), dtype=np.complex128)
    out[tuple(np.mod(k_out, N).T)] = Q
    return out


def to_physical2d(ghat: np.ndarray, L: float, centred: bool = False) -> np.ndarray:
    """g(v_j) = sum_k g_k e^{i pi k.v_j / L} on v_j = -L + j 2L/N (real part), or
    on the cell-centred grid v_j = -L + (j + 1/2) 2L/N (centred=True, where
    e^{i pi k v_j / L} = (-1)^k e^{i pi k/N} e^{2 pi i k j/N})."""
    N = ghat.shape[0]
    k = np.fft.fftfreq(N, 1.0 / N).astype(np.int64)
    k[N // 2] = 0
    sgn = np.where(k % 2 == 0, 1.0, -1.0).astype(np.complex128)
    if centred:
        sgn = sgn * np.exp(1j * math.pi * k / N)
    return np.real(np.fft.ifft2(ghat * sgn[:, None] * sgn[None, :])) * float(N) ** 2


# BKW in 2-D (Section 5.1 with d = 2; C = 1/2, lambda = 1/8 for b1-b4)
def bkw2d_K(t: float) -> float:
    return 1.0 - 0.5 * math.exp(-t / 8.0)


def bkw2d_f(v2, K):
    v2 = np.asarray(v2, dtype=np.float64)
    return np.exp(-v2 / (2 * K)) / (2 * math.pi * K) * ((4 * K - 2) / (2 * K) + (1 - K) * v2 / (2 * K * K))


def bkw2d_Q(v2, K, lam=0.125):
    v2 = np.asarray(v2, dtype=np.float64)
    return (np.exp(-v2 / (2 * K)) / (2 * math.pi * K) * (1 - K) ** 2 / (4 * K ** 4) * lam
            * (8 * K * K - 8 * K * v2 + v2 * v2))
