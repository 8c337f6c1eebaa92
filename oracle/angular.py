"""Angular weight F(k, |q|, q-hat) of the non-cutoff collision operator (eq. FF).

F(k,|q|,q) = \\int_{S^2} b(sigma.q) ( e^{i a k.(q - sigma)} - 1 ) d sigma,  a = pi |q| / (2L).

Writing sigma in the frame of q (Section 2.1, eq. FF3D1) and integrating the
azimuth exactly gives a function of two scalars only,

    Psi(x, y) = 2 pi \\int_0^pi b(cos th) [ e^{i x (1 - cos th)} J0(y sin th) - 1 ] sin th d th,
    x = a k.q,   y = a |k - (k.q) q|,

which is the exact value of F (the paper's own midpoint rule in the azimuth
converges to the same number).  With t = sin^2(th/2) the kernels handled here
are b = c t^{-1-s} (1-t)^{-r}; the singularity at t = 0 is the non-integrable
angular singularity of Section 1 (nu = 2s for r = 0), and

    Psi = 4 pi c \\int_0^1 t^{-s} (1-t)^{-r} K(t) dt,
    K(t) = [ e^{2ixt} J0(Y) - 1 ] / t,   Y = 2 y sqrt(t (1-t)),

whose integrand is smooth.  K is evaluated without cancellation:
e^{2ixt} - 1 = -2 sin^2(xt) + i sin(2xt) and J0(Y) - 1 = -Y^2 j1m(Y) with
j1m(Y) = (1 - J0(Y)) / Y^2 summed as a series for small Y.

The Debye-Yukawa kernel of Section 5.6 and its cutoff (`DebyeKernel`) use
the same K with a composite rule for their logarithmic weight.

Also here, as independent pins of Psi:
  * `F_sphere`: eq. FF3D1 done as a 2-D (t, azimuth) product rule, no Bessel
    function (the paper's azimuthal route);
  * `psi_cutoff_closed_form`: eq. cutoff3D for constant b;
  * `psi_small_argument`: the second-order expansion of Section 2.1's proof;
  * `F_eps_split`: the paper's own precompute of Section 4.1 (second-order
    Taylor on [0, eps], quadrature on [eps, pi]) -- an approximation whose
    error against the exact integral is reported, not used for parity.

Test infrastructure only: nothing in the GPU product path imports this file.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np
from scipy.special import betainc, beta as beta_fn, j0

from .quadrature import gauss_jacobi_unit


@dataclasses.dataclass(frozen=True)
class AngularKernel:
    """b(cos th) = c * t^{-1-s} * (1-t)^{-r},  t = sin^2(th/2)."""
    c: float
    s: float
    r: float = 0.0
    name: str = ""

    def b_of_theta(self, th):
        t = np.sin(0.5 * np.asarray(th)) ** 2
        return self.c * t ** (-1.0 - self.s) * (1.0 - t) ** (-self.r)

    @property
    def nu(self) -> float:
        """Order of the angular singularity at th -> 0: sin th b ~ th^{-1-nu}, nu = 2s
        (negative for an integrable kernel)."""
        return 2.0 * self.s


def power_kernel(s: float) -> AngularKernel:
    """c_s sin^{-(2+2s)}(th/2) with c_s = (1-s)(2-s)/(24 pi), so that the BKW
    rate lambda equals 1/6 as for the paper's 3-D kernels (Section 5.1)."""
    if not (0.0 <= s < 1.0):
        raise ValueError("s must lie in [0, 1)")
    return AngularKernel(c=(1.0 - s) * (2.0 - s) / (24.0 * math.pi), s=s, r=0.0, name=f"power{s}")


def cutoff_kernel(C: float = 1.0 / (4.0 * math.pi)) -> AngularKernel:
    """Constant b = C (the paper's b5 for C = 1/(4 pi)); t^{-1-s} with s = -1."""
    return AngularKernel(c=C, s=-1.0, r=0.0, name="cutoff")


# The paper's 3-D kernels of Section 5.3, rewritten in t = sin^2(th/2):
#   b6 = 1/(8 pi sin th sin(th/2))          = t^{-1} (1-t)^{-1/2} / (16 pi)
#   b7 = 1/(6 pi^2 sin th sin^2(th/2))      = t^{-3/2} (1-t)^{-1/2} / (12 pi^2)
#   b8 = 5 cos(th/2)/(192 pi sin th sin^{5/2}(th/2)) = 5 t^{-7/4} / (384 pi)
PAPER_KERNELS = {
    "b5": cutoff_kernel(1.0 / (4.0 * math.pi)),
    "b6": AngularKernel(c=1.0 / (16.0 * math.pi), s=0.0, r=0.5, name="b6"),
    "b7": AngularKernel(c=1.0 / (12.0 * math.pi ** 2), s=0.5, r=0.5, name="b7"),
    "b8": AngularKernel(c=5.0 / (384.0 * math.pi), s=0.75, r=0.0, name="b8"),
}


@dataclasses.dataclass(frozen=True)
class DebyeKernel:
    """The Debye-Yukawa kernel of Section 5.6 (eq. ApproximatedDebye):
    sin th B = |q| |log(2 sin(th/2))| / (2 sin(th/2)), i.e. Phi = |q| (gamma = 1)
    and sin th b = |log(2 sin(th/2))| / (2 sin(th/2)); zero for th < theta_cut
    (eq. ApproximatedDebyecutoff uses theta_cut = pi/10).

    With t = sin^2(th/2) (sin th d th = 2 dt) the weight is
        Psi = pi \\int_{t_c}^1 w(t) K(t) dt,  w(t) = |log(2 sqrt t)| (1-t)^{-1/2},
    K as for the power kernels.  w has a logarithmic singularity at t = 0, a
    kink at t = 1/4 and an inverse square root at t = 1; `rule` integrates it
    by a composite rule: Gauss-Jacobi for (1-t)^{-1/2} on [1/4, 1], Gauss-
    Legendre panels in geometric progression (ratio 8) on [t0, 1/4] (or
    [t_c, 1/4]), and on [0, t0] (t0 = 1e-6, no cutoff) Gauss-Laguerre after
    t = t0 e^{-u}, where |log(2 sqrt t)| is linear in u."""
    theta_cut: float = 0.0
    name: str = "debye"

    def b_of_theta(self, th):
        th = np.asarray(th, dtype=np.float64)
        sb = np.abs(np.log(2.0 * np.sin(0.5 * th))) / (2.0 * np.sin(0.5 * th))
        return np.where(th >= self.theta_cut, sb / np.sin(th), 0.0)

    prefactor = math.pi

    def rule(self, n_jacobi: int = 64):
        from scipy.special import roots_laguerre
        t0, ratio, nL = 1e-6, 8.0, 20
        ts, ws = [], []
        sB, wB = gauss_jacobi_unit(n_jacobi, 0.0, 0.5)
        tB = 0.25 + 0.75 * sB
        ts.append(tB)
        ws.append(wB * math.sqrt(0.75) * np.log(2.0 * np.sqrt(tB)))

        def panel(a, b, n):
            x, w = np.polynomial.legendre.leggauss(n)
            t = a + (b - a) * (x + 1.0) / 2.0
            return t, w * (b - a) / 2.0 * np.abs(np.log(2.0 * np.sqrt(t))) / np.sqrt(1.0 - t)

        tc = math.sin(0.5 * self.theta_cut) ** 2
        hi, k = 0.25, 0
        while True:
            lo = hi / ratio
            n = 32 if k == 0 else 24 if k == 1 else 16
            if self.theta_cut > 0.0 and lo <= tc:
                t, w = panel(tc, hi, n)
                ts.append(t)
                ws.append(w)
                break
            if lo <= t0:
                t, w = panel(t0, hi, n)
                ts.append(t)
                ws.append(w)
                if self.theta_cut == 0.0:
                    u, om = roots_laguerre(nL)
                    tL = t0 * np.exp(-u)
                    ts.append(tL)
                    ws.append(om * t0 * (u + math.log(1.0 / (4.0 * t0))) / 2.0 / np.sqrt(1.0 - tL))
                break
            t, w = panel(lo, hi, n)
            ts.append(t)
            ws.append(w)
            hi, k = lo, k + 1
        return np.concatenate(ts), np.concatenate(ws)


DEBYE_KERNELS = {"debye": DebyeKernel(0.0, "debye"), "debye_cut": DebyeKernel(math.pi / 10.0, "debye_cut")}


def _rule(kern, n_jacobi: int):
    """Nodes, weights and prefactor: Psi = prefactor * sum_i w_i K(t_i)."""
    if isinstance(kern, DebyeKernel):
        t, w = kern.rule(n_jacobi)
        return t, w, kern.prefactor
    t, w = gauss_jacobi_unit(n_jacobi, kern.s, kern.r)
    return t, w, 4.0 * math.pi * kern.c


def bkw_lambda(kern: AngularKernel) -> float:
    """lambda = 1/4 \\int_{S^2} (1 - (sigma.q)^2) b d sigma (Section 5.1)
    = 4 pi c B(1-s, 2-r) for b = c t^{-1-s}(1-t)^{-r}."""
    return 4.0 * math.pi * kern.c * beta_fn(1.0 - kern.s, 2.0 - kern.r)


# --------------------------------------------------------------------------
# Bessel helper
# --------------------------------------------------------------------------
def j1m(Y):
    """(1 - J0(Y)) / Y^2, with the power series below Y = 2."""
    Y = np.asarray(Y, dtype=np.float64)
    out = np.empty_like(Y)
    small = Y < 2.0
    z = 0.25 * Y[small] ** 2            # z <= 1 here
    # (1 - J0)/Y^2 = 1/4 * sum_{k>=1} (-1)^{k+1} z^{k-1} / (k!)^2, Horner in z,
    # 16 terms: the first dropped one is below 1e-28
    coef = [(-1.0) ** (k + 1) / math.factorial(k) ** 2 for k in range(1, 17)]
    acc = np.full_like(z, coef[-1])
    for cf in coef[-2::-1]:
        acc = acc * z + cf
    out[small] = 0.25 * acc
    Yl = Y[~small]
    out[~small] = (1.0 - j0(Yl)) / (Yl * Yl)
    return out


# --------------------------------------------------------------------------
# Psi(x, y): the exact weight, Bessel route
# --------------------------------------------------------------------------
def psi(x, y, kern, n_jacobi: int = 64):
    """F(k,|q|,q) = Psi(x, y) for arrays x = a k.q, y = a|k_perp| (same shape);
    kern is an AngularKernel or a DebyeKernel."""
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    shape = np.broadcast(x, y).shape
    x = np.broadcast_to(x, shape).reshape(-1)
    y = np.broadcast_to(y, shape).reshape(-1)
    t, w, pref = _rule(kern, n_jacobi)
    out = np.empty(x.shape, dtype=np.complex128)
    step = max(1, 2_000_000 // len(t))
    for i0 in range(0, x.size, step):
        xs = x[i0:i0 + step, None]
        ys = y[i0:i0 + step, None]
        tt = t[None, :]
        xt = xs * tt
        Y = 2.0 * ys * np.sqrt(tt * (1.0 - tt))
        jm = j1m(Y)
        J = 1.0 - Y * Y * jm
        e_re = -2.0 * np.sin(xt) ** 2 / tt            # (cos 2xt - 1)/t
        e_im = np.sin(2.0 * xt) / tt                  # sin(2xt)/t
        jm1_t = -4.0 * ys * ys * (1.0 - tt) * jm      # (J0(Y) - 1)/t
        K_re = e_re * J + jm1_t
        K_im = e_im * J
        out[i0:i0 + step] = (K_re @ w) + 1j * (K_im @ w)
    out *= pref
    return out.reshape(shape)


def F_weight(k, a, sigma, kern: AngularKernel, n_jacobi: int = 64):
    """F(k, rho, sigma) for integer modes k [nk,3], scalar a = pi rho/(2L), unit sigma [3]."""
    k = np.asarray(k, dtype=np.float64)
    sigma = np.asarray(sigma, dtype=np.float64)
    kd = k @ sigma
    kperp = np.linalg.norm(np.cross(k, sigma), axis=-1)
    return psi(a * kd, a * kperp, kern, n_jacobi)


# --------------------------------------------------------------------------
# independent pins of Psi
# --------------------------------------------------------------------------
def _frame(qhat):
    qhat = np.asarray(qhat, dtype=np.float64)
    qhat = qhat / np.linalg.norm(qhat)
    tmp = np.array([1.0, 0.0, 0.0]) if abs(qhat[0]) < 0.9 else np.array([0.0, 1.0, 0.0])
    h = np.cross(qhat, tmp)
    h /= np.linalg.norm(h)
    j = np.cross(qhat, h)
    return qhat, h, j


def F_sphere(k, a, qhat, kern: AngularKernel, n_t: int = 128, n_phi: int = 128):
    """eq. FF3D1 as a (t, azimuth) product rule: Gauss-Jacobi in t, trapezoid in phi.

    sigma = h sin th cos phi + j sin th sin phi + q cos th; no Bessel function.
    """
    k = np.asarray(k, dtype=np.float64)
    q, h, j = _frame(qhat)
    t, w = gauss_jacobi_unit(n_t, kern.s, kern.r)
    phi = 2.0 * math.pi * np.arange(n_phi) / n_phi
    cth = 1.0 - 2.0 * t
    sth = 2.0 * np.sqrt(t * (1.0 - t))
    kq, kh, kj = k @ q, k @ h, k @ j
    # Phi(t, phi) = a k.(q - sigma)
    Phi = a * (kq * (1.0 - cth)[:, None]
               - sth[:, None] * (kh * np.cos(phi)[None, :] + kj * np.sin(phi)[None, :]))
    em1 = -2.0 * np.sin(0.5 * Phi) ** 2 + 1j * np.sin(Phi)     # e^{i Phi} - 1
    inner = em1.sum(axis=1) * (2.0 * math.pi / n_phi)          # azimuth
    # d sigma = sin th d th d phi = 2 dt d phi;  b = c t^{-1-s}(1-t)^{-r}
    return 2.0 * kern.c * np.sum(w * inner / t)


def psi_cutoff_closed_form(x, y, C):
    """eq. cutoff3D: b = C gives F = 4 pi C [ e^{ix} sinc(sqrt(x^2+y^2)) - 1 ], sinc z = sin z / z."""
    x = np.asarray(x, dtype=np.float64)
    z = np.sqrt(x * x + np.asarray(y, dtype=np.float64) ** 2)
    return 4.0 * math.pi * C * (np.exp(1j * x) * np.sinc(z / math.pi) - 1.0)


def psi_small_argument(x, y, kern: AngularKernel):
    """Second-order expansion of Psi for small (x, y) (Taylor step of Section 2.1), r = 0."""
    s = kern.s
    return 4.0 * math.pi * kern.c * (2j * x / (1 - s) - 2.0 * x * x / (2 - s)
                                     - y * y / ((1 - s) * (2 - s)))


def F_eps_split(x, y, kern: AngularKernel, eps: float = math.pi / 1000, n_outer: int = 400):
    """The paper's precompute (Section 4.1, 3-D): second-order Taylor of e^{F} on
    th in [0, eps] integrated exactly, plain quadrature on [eps, pi].

    Part I after the azimuth: 2 pi \\int_0^eps b [ i x (1-cos th) - x^2 (1-cos th)^2 / 2
    - y^2 sin^2 th / 4 ] sin th dth, i.e. in t (t_eps = sin^2(eps/2)):
    4 pi c \\int_0^{t_eps} t^{-1-s}(1-t)^{-r} [ 2ixt - 2x^2 t^2 - y^2 t (1-t) ] dt,
    expressed with incomplete beta functions.  Part II uses Gauss-Legendre in th.
    """
    from numpy.polynomial.legendre import leggauss
    s, r, c = kern.s, kern.r, kern.c
    te = math.sin(0.5 * eps) ** 2

    def ib(p, q):   # \int_0^te t^{p-1} (1-t)^{q-1} dt
        return betainc(p, q, te) * beta_fn(p, q)

    I1 = ib(1 - s, 1 - r)        # \int t^{-s}(1-t)^{-r}
    I2 = ib(2 - s, 1 - r)        # \int t^{1-s}(1-t)^{-r}
    I3 = ib(1 - s, 2 - r)        # \int t^{-s}(1-t)^{1-r}
    partI = 4 * math.pi * c * (2j * x * I1 - 2 * x * x * I2 - y * y * I3)
    u, wu = leggauss(n_outer)
    th = eps + 0.5 * (math.pi - eps) * (u + 1.0)
    wth = 0.5 * (math.pi - eps) * wu
    b = kern.b_of_theta(th)
    integrand = b * (np.exp(1j * x * (1 - np.cos(th))) * j0(y * np.sin(th)) - 1.0) * np.sin(th)
    partII = 2 * math.pi * np.sum(wth * integrand)
    return partI + partII
