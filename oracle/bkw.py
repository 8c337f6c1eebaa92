"""The BKW exact solution for Maxwell molecules (Section 5.1, eq. BKW and eq. QQ), d = 3.

f(t,v) = (2 pi K)^{-3/2} e^{-|v|^2/2K} [ (5K - 3)/(2K) + (1-K)|v|^2/(2K^2) ],
K' = lambda (1 - K),  K = 1 - e^{-lambda t}  (constant C = 1),
Q(f,f) = (2 pi K)^{-3/2} e^{-|v|^2/2K} (1-K)^2/(4K^4) lambda [ 15 K^2 - 10 K |v|^2 + |v|^4 ].

It holds for any angular kernel with the same lambda, cutoff or not, which is
what makes it a pin of the non-cutoff operator.

Test infrastructure only: nothing in the GPU product path imports this file.
"""
from __future__ import annotations

import math

import numpy as np


def K_of_t(t: float, lam: float) -> float:
    return 1.0 - math.exp(-lam * t)


def f_bkw(v2, K):
    v2 = np.asarray(v2, dtype=np.float64)
    return (2 * math.pi * K) ** -1.5 * np.exp(-v2 / (2 * K)) * (
        (5 * K - 3) / (2 * K) + (1 - K) * v2 / (2 * K * K))


def Q_bkw(v2, K, lam):
    v2 = np.asarray(v2, dtype=np.float64)
    return ((2 * math.pi * K) ** -1.5 * np.exp(-v2 / (2 * K)) * (1 - K) ** 2 / (4 * K ** 4) * lam
            * (15 * K * K - 10 * K * v2 + v2 * v2))


def on_grid(fn, N: int, L: float, *args):
    v = -L + (2.0 * L / N) * np.arange(N)
    v2 = v[:, None, None] ** 2 + v[None, :, None] ** 2 + v[None, None, :] ** 2
    return fn(v2, *args)
