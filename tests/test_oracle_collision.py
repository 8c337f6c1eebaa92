"""Pins of the oracle's direct weighted sum (eq. sum with eq. approxG).

* a literal O(N^6) loop over (l, m) pairs with F from the sphere route (no
  Bessel function, no matrix product) on a 4^3 grid;
* the exact invariants: Q_0 = 0 (Remark 4.1), Q real (Hermitian), bilinearity,
  covariance under non-grid translations and under the cube symmetries that the
  sphere rule shares;
* the physics of Section 1: conservation of momentum and energy to spectral
  accuracy, the H-theorem sign, Q(M, M) ~ 0 for a Maxwellian;
* the BKW closed form (Section 5.1, eq. QQ), with the error decreasing as the
  sphere rule is refined (cf. Table 2).
"""
import math

import numpy as np
import pytest

import oracle
import workloads
from oracle import bkw
from oracle.angular import F_sphere
from oracle.collision import mode_vectors, quadrature_nodes


def _disc(N, M=38, N_rho=None, L=8.0, R=4.0, gamma=0.0, s=0.5):
    return oracle.Discretization.power(N, L, R, gamma, s, N_rho or N, M)


def _relerr(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


@pytest.fixture(scope="module")
def small16():
    d = _disc(16)
    f = workloads.config_input(workloads.CFG_SMALL, 0)
    return d, f, oracle.collision_direct(f, d)


def test_literal_sum_on_4cube():
    """eq. sum written as a loop over l + m = k with G(l, m) from eq. approxG."""
    N, L = 4, 3.0
    d = oracle.Discretization.power(N, L, 2.0, 0.5, 0.5, 3, 6)
    rng = np.random.default_rng(7)
    f = workloads.to_spectral(rng.uniform(0.5, 1.5, (N, N, N)))
    Q = oracle.collision_direct(f, d)
    rho, sig, wq = quadrature_nodes(d)
    modes = [tuple(m) for m in mode_vectors(N)]
    inK = set(modes)
    Fcache = {}
    for k in modes:
        acc = 0.0j
        for m in modes:
            l = (k[0] - m[0], k[1] - m[1], k[2] - m[2])
            if l not in inK:
                continue
            G = 0.0j
            for j in range(len(rho)):
                key = (k, j)
                if key not in Fcache:
                    Fcache[key] = F_sphere(np.array(k), math.pi * rho[j] / (2 * L), sig[j], d.kernel,
                                           n_t=64, n_phi=48)
                G += wq[j] * np.exp(-1j * math.pi / L * rho[j] * np.dot(m, sig[j])) * Fcache[key]
            acc += G * f[l] * f[m]
        assert abs(acc - Q[k]) <= 1e-12 * np.abs(Q).max(), (k, acc, Q[k])


def test_exact_invariants(small16):
    d, f, Q = small16
    N = d.N
    assert Q[0, 0, 0] == 0.0                                   # Remark 4.1
    h = N // 2
    assert np.all(Q[h] == 0) and np.all(Q[:, h] == 0) and np.all(Q[:, :, h] == 0)
    # Hermitian symmetry: Q(v) is real
    Qm = np.conj(np.roll(np.flip(Q, axis=(0, 1, 2)), 1, axis=(0, 1, 2)))
    assert np.max(np.abs(Q - Qm)) < 1e-13 * np.abs(Q).max()


def test_bilinear_scaling_and_translation_8():
    d = _disc(8, M=14)
    N, L = d.N, d.L
    f = workloads.config_input(workloads.ProblemConfig(8, 8.0, 4.0, 0.0, 0.5, 8, 14), 3)
    Q = oracle.collision_direct(f, d)
    assert _relerr(oracle.collision_direct(1.7 * f, d), 1.7 ** 2 * Q) < 1e-14
    # non-grid translation u: f_k -> f_k e^{-i pi k.u/L}, Q_k -> Q_k e^{-i pi k.u/L}
    u = np.array([0.37, -0.81, 0.23])
    k = np.fft.fftfreq(N, 1.0 / N)
    ph = np.exp(-1j * math.pi / L * (k[:, None, None] * u[0] + k[None, :, None] * u[1]
                                     + k[None, None, :] * u[2]))
    Qs = oracle.collision_direct(f * ph, d)
    assert _relerr(Qs, Q * ph) < 1e-13


def test_cube_symmetry_8():
    """f invariant under axis permutations -> Q too (Lebedev rules are octahedral)."""
    N, L = 8, 6.0
    d = oracle.Discretization.power(N, L, 3.0, 0.0, 0.25, 6, 26)
    v = workloads.velocity_grid(N, L)
    V = np.meshgrid(v, v, v, indexing="ij")
    fphys = np.exp(-(V[0] ** 2 + V[1] ** 2 + V[2] ** 2)) * (1 + 0.3 * (V[0] * V[1] * V[2]) ** 2)
    f = workloads.to_spectral(fphys)
    Q = oracle.collision_direct(f, d)
    for perm in [(1, 0, 2), (2, 1, 0), (1, 2, 0)]:
        assert np.max(np.abs(np.transpose(Q, perm) - Q)) < 1e-13 * np.abs(Q).max()


def _moments_of(qhat, L):
    N = qhat.shape[0]
    q = oracle.to_physical(qhat, L)
    v = workloads.velocity_grid(N, L)
    V = np.meshgrid(v, v, v, indexing="ij")
    h3 = (2 * L / N) ** 3
    return (h3 * np.sum(q), np.array([h3 * np.sum(q * V[i]) for i in range(3)]),
            h3 * np.sum(q * (V[0] ** 2 + V[1] ** 2 + V[2] ** 2)))


def test_mass_and_h_theorem(small16):
    d, f, Q = small16
    mass, mom, energy = _moments_of(Q, d.L)
    assert abs(mass) < 1e-15
    fphys = workloads.two_maxwellians(0).sample(d.N, d.L)
    D = oracle.entropy_dissipation(Q, fphys, d.L)
    assert D < 0


def test_energy_conservation_improves_with_N():
    """Corollary 3.5: moments of Q converge spectrally; 8^3 -> 16^3 must improve."""
    e_err, p_err = [], []
    for N in (8, 16):
        d = _disc(N, M=14, N_rho=8)
        mix = workloads.two_maxwellians(1)
        f = workloads.to_spectral(mix.sample(N, d.L))
        Q = oracle.collision_direct(f, d)
        _, mom, energy = _moments_of(Q, d.L)
        e_err.append(abs(energy))
        p_err.append(np.abs(mom).max())
    assert e_err[1] < 0.5 * e_err[0]
    assert p_err[1] < 0.5 * p_err[0]


def test_maxwellian_is_equilibrium(small16):
    d, f, Q = small16
    M = workloads.to_spectral(workloads.maxwellian_on_grid(d.N, d.L, 1.0, (0.3, -0.2, 0.1), 1.4))
    QM = oracle.collision_direct(M, d)
    assert np.linalg.norm(QM) < 1e-2 * np.linalg.norm(Q)


@pytest.mark.slow
def test_bkw_closed_form_sphere_convergence():
    """3-D BKW at t = 6.5 with the setup of Table 2 (N = N_rho = 32, R = 6,
    L = (3+sqrt 2)R/4): the oracle's Q_k on sampled modes against the spectral
    coefficients of eq. QQ.  The error must fall as the sphere rule is refined
    and reach the order of magnitude of Table 2's finest rows (~1e-5 of max|Q|)."""
    R = 6.0
    L = (3 + math.sqrt(2)) * R / 4
    N = 32
    lam = 1.0 / 6.0
    K = bkw.K_of_t(6.5, lam)
    f = workloads.to_spectral(workloads.bkw_profile_on_grid(N, L, K))
    Qe = workloads.to_spectral(bkw.on_grid(bkw.Q_bkw, N, L, K, lam))
    ks = np.array([(0, 0, 0), (1, 0, 0), (1, 1, 1), (2, 0, 0), (3, 1, 0), (0, 0, 5),
                   (4, 4, 0), (2, 3, 6), (8, 0, 0), (-3, 7, 2)])
    idx = tuple(np.mod(ks, N).T)
    scale = np.abs(Qe).max()
    errs = {}
    for M in (38, 110, 302):
        d = oracle.Discretization(N, L, R, 0.0, oracle.PAPER_KERNELS["b8"], 32, M)
        Q = oracle.collision_direct(f, d, k_out=ks)
        errs[M] = np.abs(Q - Qe[idx]).max() / scale
    assert errs[38] > errs[110] > 0.9 * errs[302]
    assert errs[302] < 1e-4
    assert errs[38] > 1e-3


@pytest.mark.parametrize("N,gamma,s,N_rho,M", [(8, 0.0, 0.5, 6, 14), (16, -1.0, 0.25, 4, 26)])
def test_fft_form_equals_direct_sum(N, gamma, s, N_rho, M):
    """The FFT evaluation of eq. realQ (zero padding to 3N/2) equals the direct
    weighted sum: dealiasing is exact and the convolution is the truncated one."""
    L = 8.0
    d = oracle.Discretization.power(N, L, 4.0, gamma, s, N_rho, M)
    f = workloads.to_spectral(workloads.random_mixture(N).sample(N, L))
    modes = oracle.mode_vectors(N)
    T = oracle.weight_table(d, modes)
    q_direct = oracle.collision_direct(f, d, T=T)
    q_fft = oracle.collision_fft(f, d, T=T)
    assert np.linalg.norm(q_fft - q_direct) <= 1e-13 * np.linalg.norm(q_direct)
