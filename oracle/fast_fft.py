"""The fast algorithm of Section 4 (eq. realQ) on the CPU with FFTs (FP64).

    Q_k = sum_j T_j(k) [f conv (E_j f)]_k,   E_j(m) = e^{-i pi rho_j m.sigma_j / L},

where conv is the truncated convolution over K_N (eq. realQ's inner sum).  It
is evaluated as a product in physical space: both factors are placed on a
P^3 grid with P = 3N/2, transformed to the grid, multiplied pointwise and
transformed back, and only k in K_N is kept.  With |l_i|, |m_i|, |k_i| <= N/2 - 1
no index l + m - k other than 0 is a multiple of P, so nothing wraps around and
the result is exactly the truncated sum.  One pair of FFTs per quadrature node
(every node of the full sphere rule, no symmetry folding, no packing): the
paper's O(N_sigma N^{d+1} log N) method in its plainest form, used as the CPU
throughput baseline beside the GPU path.

Pinned against the direct sum (`collision.collision_direct`) on 8^3 and 16^3
grids by the CPU tests.  Test infrastructure only: nothing in the GPU product
path imports this file.
"""
from __future__ import annotations

import math
import os

import numpy as np
import scipy.fft as sfft

from .collision import Discretization, mode_vectors, quadrature_nodes, weight_table


def collision_fft(fhat: np.ndarray, d: Discretization, nodes=None, T=None, workers=None) -> np.ndarray:
    """Q (N^3, FFT order) summed over all quadrature nodes, or over `nodes` only
    (a partial sum, for timing).  T: precomputed weight_table rows of those nodes."""
    N = d.N
    P = 3 * N // 2
    workers = workers or os.cpu_count() or 1
    modes = mode_vectors(N)
    rho, sig, _ = quadrature_nodes(d)
    sel = np.arange(len(rho)) if nodes is None else np.asarray(nodes)
    if T is None:
        T = weight_table(d, modes, nodes=sel)
    pidx = tuple(np.mod(modes, P).T)                 # k -> padded grid index
    fm = np.asarray(fhat, dtype=np.complex128)[tuple(np.mod(modes, N).T)]
    grid = np.zeros((P, P, P), dtype=np.complex128)
    grid[pidx] = fm
    fv = sfft.ifftn(grid, workers=workers) * P ** 3        # f(x) = sum_m f_m e^{2 pi i m.x / P}
    mf = modes.astype(np.float64)
    Q = np.zeros(len(modes), dtype=np.complex128)
    for row, j in enumerate(sel):
        grid[...] = 0
        grid[pidx] = fm * np.exp((-1j * math.pi * rho[j] / d.L) * (mf @ sig[j]))
        gv = sfft.ifftn(grid, workers=workers) * P ** 3
        h = sfft.fftn(fv * gv, workers=workers) / P ** 3   # sum over l + m = k of f_l (E f)_m
        Q += T[row] * h[pidx]
    out = np.zeros((N, N, N), dtype=np.complex128)
    out[tuple(np.mod(modes, N).T)] = Q
    return out
