"""Direct evaluation of the discrete collision operator (CPU, FP64).

The fast method of Section 4 (eq. realQ) is an exact regrouping of the
weighted convolution of Section 2 (eq. sum),

    Q_k = sum_{l+m=k; l,m in K_N} G(l, m) f_l f_m,

with G replaced by its quadrature (eq. approxG):

    G(l, m) ~ sum_{p,q} w_p w_q Phi(rho_p) rho_p^2 e^{-i pi rho_p m.sigma_q / L} F(l+m, rho_p, sigma_q).

So the oracle is that finite sum written out, with no FFT:

    Q_k = sum_j T_j(k) sum_{m in K_N, k-m in K_N} e^{-i pi rho_j m.sigma_j / L} f_{k-m} f_m,
    T_j(k) = w_p w_q rho_p^{2+gamma} F(k, rho_p, sigma_q),        Phi(|q|) = |q|^gamma,

evaluated as Y = E C (a matrix product, E[j,m] the phases, C[m,k] = f_{k-m} f_m)
followed by Q_k = sum_j T_j(k) Y[j,k].  Every radial node and every sphere point
(the full sphere, no symmetry folding) contributes its own term.

Readings of the paper used here:
  * mode set K_N = {-N/2+1 .. N/2-1}^3 (the paper writes -N/2..N/2, which does
    not fit an N-point grid); arrays are N^3 in FFT order, Nyquist planes zero;
  * the convolution is the truncated sum over l, m, k in K_N (no aliasing);
  * the sphere rule is Lebedev (spherical designs are not available);
  * F is the exact angular integral (eq. FF), evaluated by `angular.psi`.

Test infrastructure only: nothing in the GPU product path imports this file.
"""
from __future__ import annotations

import dataclasses
import math
from concurrent.futures import ThreadPoolExecutor
from typing import Optional

import numpy as np

from .angular import AngularKernel, DebyeKernel, power_kernel, psi
from .quadrature import radial_gauss_legendre, sphere_lebedev


@dataclasses.dataclass(frozen=True)
class Discretization:
    N: int
    L: float
    R: float
    gamma: float
    kernel: AngularKernel
    N_rho: int
    M: int
    n_jacobi: int = 64

    @staticmethod
    def power(N, L, R, gamma, s, N_rho, M, n_jacobi=64):
        return Discretization(N, L, R, gamma, power_kernel(s), N_rho, M, n_jacobi)

    @staticmethod
    def debye(N, L, R, theta_cut, N_rho, M):
        """The Debye-Yukawa kernel of Section 5.6: Phi = |q| (gamma = 1)."""
        return Discretization(N, L, R, 1.0, DebyeKernel(theta_cut), N_rho, M)


def mode_vectors(N: int) -> np.ndarray:
    """All k in K_N as an integer array [(N-1)^3, 3], k1 slowest."""
    r = np.arange(-N // 2 + 1, N // 2, dtype=np.int64)
    g = np.stack(np.meshgrid(r, r, r, indexing="ij"), axis=-1)
    return g.reshape(-1, 3)


def fft_index(k: np.ndarray, N: int) -> np.ndarray:
    """FFT-order array index of integer modes (any shape [...,3] -> [...,3])."""
    return np.mod(k, N)


def quadrature_nodes(d: Discretization):
    """All (rho_p, sigma_q) nodes: rho [J], sigma [J,3], weight w_p w_q rho^{2+gamma} [J]."""
    rho, wr = radial_gauss_legendre(d.N_rho, d.R)
    sig, ws = sphere_lebedev(d.M)
    rho_j = np.repeat(rho, d.M)
    wr_j = np.repeat(wr, d.M)
    sig_j = np.tile(sig, (d.N_rho, 1))
    ws_j = np.tile(ws, d.N_rho)
    return rho_j, sig_j, wr_j * ws_j * rho_j ** (2.0 + d.gamma)


def weight_table(d: Discretization, k_out: np.ndarray, nodes=None) -> np.ndarray:
    """T_j(k) = w_p w_q rho_p^{2+gamma} F(k, rho_p, sigma_q) for all nodes j (or the
    listed ones), modes k: [J, nk]."""
    rho, sig, wq = quadrature_nodes(d)
    if nodes is not None:
        rho, sig, wq = rho[nodes], sig[nodes], wq[nodes]
    a = math.pi * rho / (2.0 * d.L)
    kf = k_out.astype(np.float64)
    kd = sig @ kf.T                                               # [J, nk]
    kk = np.sum(kf * kf, axis=1)[None, :]
    cr = np.cross(kf[None, :, :], sig[:, None, :])                # [J, nk, 3]
    kperp = np.sqrt(np.sum(cr * cr, axis=-1))
    x = a[:, None] * kd
    y = a[:, None] * kperp
    del kk, cr
    F = _parallel_psi(x, y, d.kernel, d.n_jacobi)
    return wq[:, None] * F


def _parallel_psi(x, y, kern, n_jacobi, workers=8):
    x = np.ascontiguousarray(x)
    y = np.ascontiguousarray(y)
    flat_x = x.reshape(-1)
    flat_y = y.reshape(-1)
    out = np.empty(flat_x.shape, dtype=np.complex128)
    n = flat_x.size
    chunks = [(i, min(n, i + max(1, n // (4 * workers) + 1))) for i in range(0, n, max(1, n // (4 * workers) + 1))]

    def run(c):
        i0, i1 = c
        out[i0:i1] = psi(flat_x[i0:i1], flat_y[i0:i1], kern, n_jacobi)

    if n > 20000:
        with ThreadPoolExecutor(workers) as ex:
            list(ex.map(run, chunks))
    else:
        for c in chunks:
            run(c)
    return out.reshape(x.shape)


def collision_direct(fhat: np.ndarray, d: Discretization, k_out: Optional[np.ndarray] = None,
                     k_block: int = 256, j_block: int = 512, T: Optional[np.ndarray] = None):
    """Q_k for the modes k_out [nk,3] (default: all of K_N, returned as N^3 FFT-order array).

    fhat: complex128 N^3 in FFT order (Nyquist entries are ignored).
    """
    N = d.N
    fhat = np.asarray(fhat, dtype=np.complex128)
    assert fhat.shape == (N, N, N)
    full = k_out is None
    if full:
        k_out = mode_vectors(N)
    k_out = np.asarray(k_out, dtype=np.int64).reshape(-1, 3)
    nk = len(k_out)
    m = mode_vectors(N)
    fm = fhat[tuple(fft_index(m, N).T)]                            # f_m
    rho, sig, _ = quadrature_nodes(d)
    J = len(rho)
    if T is None:
        T = weight_table(d, k_out)                                  # [J, nk]
    h = N // 2
    Q = np.zeros(nk, dtype=np.complex128)
    mf = m.T.astype(np.float64)
    for k0 in range(0, nk, k_block):
        kb = k_out[k0:k0 + k_block]
        diff = kb[None, :, :] - m[:, None, :]                       # k - m  [nm, kb, 3]
        valid = np.all(np.abs(diff) <= h - 1, axis=-1)
        fkm = fhat[tuple(fft_index(diff, N).transpose(2, 0, 1))]
        C = np.where(valid, fkm, 0.0) * fm[:, None]                 # C[m, k] = f_{k-m} f_m
        acc = np.zeros(len(kb), dtype=np.complex128)
        for j0 in range(0, J, j_block):
            mdot = sig[j0:j0 + j_block] @ mf                         # m.sigma_j  [jb, nm]
            E = np.exp((-1j * math.pi / d.L) * rho[j0:j0 + j_block, None] * mdot)
            Y = E @ C                                                # [jb, kb]
            acc += np.sum(T[j0:j0 + j_block, k0:k0 + k_block] * Y, axis=0)
        Q[k0:k0 + k_block] = acc
    if not full:
        return Q
    out = np.zeros((N, N, N), dtype=np.complex128)
    out[tuple(fft_index(k_out, N).T)] = Q
    return out
