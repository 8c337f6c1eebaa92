r"""Seeded synthetic inputs for the collision-operator workloads.

This module only produces input data: velocity grids, sampled distribution
functions (Maxwellian mixtures, the BKW profile used as initial data) and their
spectral coefficients on the periodic box D_L = [-L, L]^3.  It holds none of
the collision operator's arithmetic.  Both the CPU oracle and the GPU library
consume what it returns, so neither side's arithmetic can leak into the other
through the inputs.

Conventions (Section 2 of the paper, Fourier-Galerkin space P_N):
  * grid points v_j = -L + j * (2L/N), j in {0..N-1}^3;
  * spectral coefficient f_k = (2L)^-3 \int_{D_L} f e^{-i pi k.v / L} dv,
    approximated by the trapezoid rule, i.e.
    f_k = N^-3 (-1)^(k1+k2+k3) DFT(f)_k;
  * arrays are N x N x N complex128 in FFT index order (index i <-> k = i for
    i < N/2, k = i - N otherwise); the Nyquist planes (i = N/2) are zero, so
    the mode set is K_N = {-N/2+1 .. N/2-1}^3.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Sequence, Tuple

import numpy as np

__all__ = [
    "velocity_grid", "mode_indices", "to_spectral", "maxwellian_on_grid",
    "MaxwellianMixture", "two_maxwellians", "random_mixture", "bkw_profile_on_grid",
    "ProblemConfig", "CFG_SMALL", "CFG_MEDIUM", "CFG_LARGE", "config_input",
    "cell_batch", "request_stream", "to_spectral_2d", "bkw2d_profile_on_grid", "random_mixture_2d",
    "broadband_spectrum", "broadband_spectrum_2d", "survey_mode_sample",
]


# --------------------------------------------------------------------------
# grids and the spectral projection
# --------------------------------------------------------------------------
def velocity_grid(N: int, L: float, centred: bool = False) -> np.ndarray:
    """1-D grid v_j = -L + j*2L/N, j = 0..N-1 (the same along each axis); with
    centred=True the cell-centred grid v_j = -L + (j + 1/2) 2L/N, symmetric about
    0 (the grid on which the paper's Table 1 is reproduced at every N)."""
    return -L + (2.0 * L / N) * (np.arange(N, dtype=np.float64) + (0.5 if centred else 0.0))


def mode_indices(N: int) -> np.ndarray:
    """Integer wavenumber of each FFT-order index along one axis (Nyquist -> -N/2)."""
    return np.fft.fftfreq(N, d=1.0 / N).astype(np.int64)


def to_spectral(f_phys: np.ndarray) -> np.ndarray:
    """Trapezoid-rule projection of grid samples onto P_N, Nyquist removed.

    f_k = N^-3 (-1)^(k1+k2+k3) sum_j f(v_j) e^{-2 pi i k.j/N}.
    Returns complex128 N^3 in FFT index order.
    """
    f_phys = np.asarray(f_phys, dtype=np.float64)
    N = f_phys.shape[0]
    assert f_phys.shape == (N, N, N) and N % 2 == 0
    k = mode_indices(N)
    sign = np.where(k % 2 == 0, 1.0, -1.0)
    fh = np.fft.fftn(f_phys) / float(N) ** 3
    fh *= sign[:, None, None] * sign[None, :, None] * sign[None, None, :]
    h = N // 2
    fh[h, :, :] = 0.0
    fh[:, h, :] = 0.0
    fh[:, :, h] = 0.0
    return fh.astype(np.complex128)


def maxwellian_on_grid(N: int, L: float, rho: float, u: Sequence[float], T: float) -> np.ndarray:
    """rho (2 pi T)^-3/2 exp(-|v-u|^2 / 2T) sampled on the N^3 grid (axis order v1, v2, v3)."""
    v = velocity_grid(N, L)
    g = [np.exp(-((v - u[d]) ** 2) / (2.0 * T)) for d in range(3)]
    norm = rho / (2.0 * math.pi * T) ** 1.5
    return norm * g[0][:, None, None] * g[1][None, :, None] * g[2][None, None, :]


@dataclasses.dataclass(frozen=True)
class MaxwellianMixture:
    """sum_i w_i M_{u_i, T_i}, each M of unit mass."""
    weights: Tuple[float, ...]
    centers: Tuple[Tuple[float, float, float], ...]
    temps: Tuple[float, ...]

    def sample(self, N: int, L: float) -> np.ndarray:
        f = np.zeros((N, N, N))
        for w, u, T in zip(self.weights, self.centers, self.temps):
            f += maxwellian_on_grid(N, L, w, u, T)
        return f


def two_maxwellians(seed: int) -> MaxwellianMixture:
    """Two unit-temperature Maxwellians at u = (+-2, 0, 0); w1 ~ U[0.4, 0.6], w2 = 1 - w1."""
    rng = np.random.default_rng(seed)
    w1 = float(rng.uniform(0.4, 0.6))
    return MaxwellianMixture((w1, 1.0 - w1), ((2.0, 0.0, 0.0), (-2.0, 0.0, 0.0)), (1.0, 1.0))


def random_mixture(seed: int) -> MaxwellianMixture:
    """2-5 Maxwellians, centres U[-3,3]^3, temperatures U[0.5,1.5], Dirichlet(1) weights."""
    rng = np.random.default_rng(seed)
    n = int(rng.integers(2, 6))
    centers = rng.uniform(-3.0, 3.0, size=(n, 3))
    temps = rng.uniform(0.5, 1.5, size=n)
    w = rng.dirichlet(np.ones(n))
    return MaxwellianMixture(tuple(float(x) for x in w),
                             tuple(tuple(float(c) for c in row) for row in centers),
                             tuple(float(t) for t in temps))


def bkw_profile_on_grid(N: int, L: float, K: float) -> np.ndarray:
    """The isotropic BKW profile with shape parameter K, sampled on the grid (3-D).

    (2 pi K)^-3/2 exp(-|v|^2/2K) [ (5K - 3)/(2K) + (1 - K)|v|^2 / (2K^2) ]
    (Section 5.1 of the paper); used only as initial data here.
    """
    v = velocity_grid(N, L)
    v2 = v[:, None, None] ** 2 + v[None, :, None] ** 2 + v[None, None, :] ** 2
    return (2 * math.pi * K) ** -1.5 * np.exp(-v2 / (2 * K)) * (
        (5 * K - 3) / (2 * K) + (1 - K) * v2 / (2 * K * K))


def to_spectral_2d(f_phys: np.ndarray, centred: bool = False) -> np.ndarray:
    """The 2-D projection: f_k = N^-2 sum_j f(v_j) e^{-i pi k.v_j/L}, i.e.
    N^-2 (-1)^(k1+k2) sum_j f(v_j) e^{-2 pi i k.j/N} on the grid v_j = -L + j h,
    with the extra factor e^{-i pi (k1+k2)/N} for samples on the cell-centred
    grid v_j = -L + (j + 1/2) h (centred=True); Nyquist removed; complex128 N^2
    in FFT index order."""
    f_phys = np.asarray(f_phys, dtype=np.float64)
    N = f_phys.shape[0]
    assert f_phys.shape == (N, N) and N % 2 == 0
    k = mode_indices(N)
    sign = np.where(k % 2 == 0, 1.0, -1.0).astype(np.complex128)
    if centred:
        sign = sign * np.exp(-1j * math.pi * k / N)
    fh = np.fft.fft2(f_phys) / float(N) ** 2 * sign[:, None] * sign[None, :]
    fh[N // 2, :] = 0.0
    fh[:, N // 2] = 0.0
    return fh.astype(np.complex128)


def bkw2d_profile_on_grid(N: int, L: float, K: float, centred: bool = False) -> np.ndarray:
    """The 2-D BKW profile (2 pi K)^-1 exp(-|v|^2/2K) [ (4K - 2)/(2K) + (1 - K)|v|^2/(2K^2) ]
    (Section 5.1 with d = 2), sampled on the N^2 grid (velocity_grid with
    `centred`); used only as initial data."""
    v = velocity_grid(N, L, centred)
    v2 = v[:, None] ** 2 + v[None, :] ** 2
    return np.exp(-v2 / (2 * K)) / (2 * math.pi * K) * ((4 * K - 2) / (2 * K) + (1 - K) * v2 / (2 * K * K))


def random_mixture_2d(seed: int, N: int, L: float) -> np.ndarray:
    """2-D analogue of `random_mixture` sampled on the N^2 grid: 2-5 Maxwellians,
    centres U[-3,3]^2 (scaled by L/8 for boxes smaller than L = 8), temperatures
    U[0.5,1.5] (same scaling squared), Dirichlet(1) weights."""
    rng = np.random.default_rng(seed)
    n = int(rng.integers(2, 6))
    scale = min(1.0, L / 8.0)
    centers = rng.uniform(-3.0, 3.0, size=(n, 2)) * scale
    temps = rng.uniform(0.5, 1.5, size=n) * scale ** 2
    w = rng.dirichlet(np.ones(n))
    v = velocity_grid(N, L)
    f = np.zeros((N, N))
    for wi, u, T in zip(w, centers, temps):
        f += wi / (2.0 * math.pi * T) * np.exp(-((v[:, None] - u[0]) ** 2 + (v[None, :] - u[1]) ** 2) / (2.0 * T))
    return f


def broadband_spectrum(N: int, seed: int, d: int = 3) -> np.ndarray:
    """Random spectral coefficients with a flat spectrum over K_N (d = 3 or 2):
    f_k = (a + i b)/sqrt(2), a, b ~ N(0, 1), for every k in K_N, made Hermitian
    (f_{-k} = conj f_k, f_0 real), Nyquist entries zero; FFT index order.  Its
    grid function is real but not positive: an input on which every mode of
    the output, up to the corners of K_N, carries weight (unlike smooth
    Maxwellians, whose edge modes are ~1e-30 of the peak)."""
    rng = np.random.default_rng(seed)
    shape = (N,) * d
    f = (rng.normal(size=shape) + 1j * rng.normal(size=shape)) / math.sqrt(2.0)
    # Hermitian part: f_k <- (f_k + conj f_{-k}) / sqrt 2 keeps unit variance
    fm = np.conj(np.flip(np.roll(f, -1, axis=tuple(range(d))), axis=tuple(range(d))))
    f = (f + fm) / math.sqrt(2.0)
    h = N // 2
    for ax in range(d):
        idx = [slice(None)] * d
        idx[ax] = h
        f[tuple(idx)] = 0.0
    f[(0,) * d] = f[(0,) * d].real
    return f.astype(np.complex128)


def broadband_spectrum_2d(N: int, seed: int) -> np.ndarray:
    """`broadband_spectrum` on the 2-D mode set K_N = {-N/2+1..N/2-1}^2."""
    return broadband_spectrum(N, seed, d=2)


def survey_mode_sample(N: int, seed: int, n_random: int = 128, inf_radius: int = 2) -> np.ndarray:
    """Output modes for sampled parity at large N: every k with |k|_inf <=
    inf_radius, the 8 corners (+-(N/2-1))^3 of K_N, and n_random uniform modes
    of K_N (seeded); duplicates removed, order kept.  int64 [n, 3]."""
    h = N // 2 - 1
    r = np.arange(-inf_radius, inf_radius + 1)
    near = np.stack(np.meshgrid(r, r, r, indexing="ij"), axis=-1).reshape(-1, 3)
    corners = np.array([(a, b, c) for a in (-h, h) for b in (-h, h) for c in (-h, h)])
    rng = np.random.default_rng(seed)
    rnd = rng.integers(-h, h + 1, size=(n_random, 3))
    out, seen = [], set()
    for k in np.concatenate([near, corners, rnd]):
        t = tuple(int(x) for x in k)
        if t not in seen:
            seen.add(t)
            out.append(t)
    return np.array(out, dtype=np.int64)


# --------------------------------------------------------------------------
# named workloads
# --------------------------------------------------------------------------
@dataclasses.dataclass(frozen=True)
class ProblemConfig:
    """Discretisation parameters of one collision-operator evaluation."""
    N: int
    L: float
    R: float
    gamma: float
    s: float
    N_rho: int
    M: int


# small case (the oracle covers every mode in seconds)
CFG_SMALL = ProblemConfig(N=16, L=8.0, R=4.0, gamma=0.0, s=0.5, N_rho=16, M=38)
# medium case: the throughput workload
CFG_MEDIUM = ProblemConfig(N=32, L=8.0, R=4.0, gamma=0.0, s=0.5, N_rho=32, M=110)
# large case
CFG_LARGE = ProblemConfig(N=64, L=10.0, R=5.0, gamma=0.0, s=0.5, N_rho=64, M=302)


def config_input(cfg: ProblemConfig, seed: int) -> np.ndarray:
    """Spectral initial data for a named configuration (complex128 N^3, FFT order)."""
    if cfg.N >= 64:
        mix = random_mixture(seed)
    else:
        mix = two_maxwellians(seed)
    return to_spectral(mix.sample(cfg.N, cfg.L))


def cell_batch(n_cells: int, seed: int, sizes=(16, 24, 32), probs=(0.5, 0.3, 0.2),
               L: float = 8.0) -> List[Tuple[int, np.ndarray]]:
    """Independent homogeneous cells: N drawn from `sizes` with `probs`; cell i's
    data is a random Maxwellian mixture seeded by seed + i."""
    rng = np.random.default_rng(seed)
    Ns = rng.choice(np.asarray(sizes), size=n_cells, p=np.asarray(probs))
    out = []
    for i, N in enumerate(Ns):
        mix = random_mixture(seed + 1 + i)
        out.append((int(N), to_spectral(mix.sample(int(N), L))))
    return out


def request_stream(rate_hz: float, duration_s: float, seed: int,
                   sizes=(16, 32, 48, 64), gammas=(-1.0, 0.0), ss=(0.25, 0.75)):
    """Poisson arrivals: list of (arrival_time_s, N, gamma, s, mixture_seed)."""
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    while True:
        t += float(rng.exponential(1.0 / rate_hz))
        if t > duration_s:
            break
        out.append((t, int(rng.choice(sizes)), float(rng.choice(gammas)),
                    float(rng.choice(ss)), int(rng.integers(0, 2**31 - 1))))
    return out
