"""Write the stored expected values used by the GPU parity tests at sizes where
the oracle cannot run inside a test: Q_k of the FP64 direct-sum oracle at a
sample of output modes, for the medium (32^3) and large (64^3) workloads.

Calls only `oracle` and `workloads` (seeded inputs).  Run from the repository
root:  python tests/golden/make_golden.py [name ...]
Also the paper's kernels b5 and b8 (Section 5.3) at N = 128 (paper128_*.npz,
with the kernel name in `kernel`), and the 2-D operator (d = 2, Section 5.2)
on broadband inputs at N = 64, all modes: tests/golden/<name>.npz with Q2 (complex128 N^2, FFT order) and params2
(N, L, R, gamma, N_rho, N_sigma, seed) and the kernel name.
Each 3-D case writes tests/golden/<name>.npz with arrays
  modes  int64 [n, 3]   sampled output modes k
  Q      complex128 [n] oracle Q_k
  params float64 [8]    N, L, R, gamma, s, N_rho, M, seed
  kind   input recipe code (0: two Maxwellians at +-2 e1, 1: random mixture,
         2: broadband random Hermitian spectrum, workloads.broadband_spectrum)
"""
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle      # noqa: E402
import workloads   # noqa: E402
from oracle import collision2d as o2   # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))

CASES = {
    # name: (N, L, R, gamma, s, N_rho, M, seed, kind, n_random)
    "medium_s050": (32, 8.0, 4.0, 0.0, 0.50, 32, 110, 0, 0, 48),
    "medium_s025": (32, 8.0, 4.0, 0.0, 0.25, 32, 110, 1, 0, 16),
    "medium_s075": (32, 8.0, 4.0, 0.0, 0.75, 32, 110, 2, 0, 16),
    "medium_gm1": (32, 8.0, 4.0, -1.0, 0.50, 32, 110, 3, 0, 16),
    "medium_gp1": (32, 8.0, 4.0, 1.0, 0.50, 32, 110, 4, 0, 16),
    "large_s050": (64, 10.0, 5.0, 0.0, 0.50, 64, 302, 0, 1, 16),
    # the large workload at gamma = -1, +1 (same input as large_s050)
    "large_gm1": (64, 10.0, 5.0, -1.0, 0.50, 64, 302, 0, 1, 24),
    "large_gp1": (64, 10.0, 5.0, 1.0, 0.50, 64, 302, 0, 1, 24),
}

# broadband inputs, sampled at every |k|_inf <= 2 mode, the 8 corners of K_N
# and 128 random modes (workloads.survey_mode_sample)
BROADBAND = {
    # name: (N, L, R, gamma, s, N_rho, M, seed)
    "broadband_N32": (32, 8.0, 4.0, 0.0, 0.50, 32, 110, 7),
    "broadband_N48": (48, 9.0, 4.5, 0.0, 0.75, 16, 110, 8),
    "broadband_N64": (64, 10.0, 5.0, 0.0, 0.50, 64, 302, 9),
    # N = 128 (P = 192: the three-pass plane and the 72-slot weight series at
    # the large workload's box, a|k| up to 86) with a small quadrature
    "broadband_N128": (128, 10.0, 5.0, 0.0, 0.50, 8, 6, 11),
}

# N = 128 on a smooth random Maxwellian mixture (kind 1), gamma = -1
CASES["huge_mix_gm1"] = (128, 10.0, 5.0, -1.0, 0.50, 8, 14, 12, 1, 16)


# the paper's kernels of Section 5.3 at N = 128 (general b = c t^{-1-s}(1-t)^{-r}),
# broadband input, every |k|_inf <= 1 mode, the corners and 40 random modes
PAPER_128 = {
    # name: (N, L, R, gamma, kernel, N_rho, M, seed)
    "paper128_b5": (128, 10.0, 5.0, 0.0, "b5", 8, 6, 13),
    "paper128_b8": (128, 10.0, 5.0, -1.0, "b8", 8, 6, 14),
}


def make_paper128(name):
    N, L, R, gamma, kname, N_rho, M, seed = PAPER_128[name]
    d = oracle.Discretization(N, L, R, gamma, oracle.PAPER_KERNELS[kname], N_rho, M)
    f = workloads.broadband_spectrum(N, seed)
    ks = workloads.survey_mode_sample(N, seed, n_random=40, inf_radius=1)
    t0 = time.time()
    q = oracle.collision_direct(f, d, k_out=ks, k_block=16, j_block=16)
    params = np.array([N, L, R, gamma, 0.0, N_rho, M, seed], dtype=np.float64)
    np.savez(os.path.join(HERE, name + ".npz"), modes=ks, Q=q, params=params, kind=np.array(2),
             kernel=np.array(kname))
    print(f"{name}: {len(ks)} modes in {time.time() - t0:.1f} s", flush=True)


# 2-D broadband cases at N = 64: the register pipeline at 16 pair-twos, the
# register / column-parity pipeline at Table 1's setting (512 pair-twos) and the
# LDS pipeline (1040 pair-twos)
CASES_2D = {
    # name: (N, L, R, gamma, kernel, N_rho, N_sigma, seed)
    "broadband2d_N64_reg": (64, 8.0, 4.0, 0.0, "b1", 8, 8, 31),
    "broadband2d_N64_tab1": (64, (3 + 2 ** 0.5) * 6.0 / 4, 6.0, 0.0, "b4", 64, 32, 32),
    "broadband2d_N64_lds": (64, 8.0, 4.0, 0.0, "b3", 65, 64, 33),
}


def make2d(name):
    N, L, R, gamma, kname, N_rho, N_sigma, seed = CASES_2D[name]
    d = o2.Discretization2D(N, L, R, gamma, o2.PAPER_KERNELS_2D[kname], N_rho, N_sigma)
    f = workloads.broadband_spectrum_2d(N, seed)
    t0 = time.time()
    q = o2.collision_direct2d(f, d)
    params = np.array([N, L, R, gamma, N_rho, N_sigma, seed], dtype=np.float64)
    np.savez(os.path.join(HERE, name + ".npz"), Q2=q, params2=params, kernel=np.array(kname))
    print(f"{name}: all {(N - 1) ** 2} modes in {time.time() - t0:.1f} s", flush=True)


def sample_modes(N, n_random, seed):
    h = N // 2 - 1
    fixed = [(0, 0, 0), (1, 0, 0), (0, 1, 0), (0, 0, 1), (1, 1, 1), (-1, 2, -3), (h, 0, 0), (0, -h, 0),
             (h, h, h), (-h, -h, -h), (h, -h, 1), (3, 5, -7)]
    rng = np.random.default_rng(seed + 1000)
    rnd = [tuple(int(x) for x in rng.integers(-h, h + 1, 3)) for _ in range(n_random)]
    out = []
    for k in fixed + rnd:
        if k not in out:
            out.append(k)
    return np.array(out, dtype=np.int64)


def input_of(N, L, seed, kind):
    if kind == 2:
        return workloads.broadband_spectrum(N, seed)
    mix = workloads.two_maxwellians(seed) if kind == 0 else workloads.random_mixture(seed)
    return workloads.to_spectral(mix.sample(N, L))


def make(name):
    if name in BROADBAND:
        N, L, R, gamma, s, N_rho, M, seed = BROADBAND[name]
        kind = 2
        ks = workloads.survey_mode_sample(N, seed)
    else:
        N, L, R, gamma, s, N_rho, M, seed, kind, nr = CASES[name]
        ks = sample_modes(N, nr, seed)
    d = oracle.Discretization.power(N, L, R, gamma, s, N_rho, M)
    f = input_of(N, L, seed, kind)
    t0 = time.time()
    if N >= 128:   # 2 M modes m: bound the [m, k] blocks to about 1 GB
        q = oracle.collision_direct(f, d, k_out=ks, k_block=16, j_block=16)
    else:
        q = oracle.collision_direct(f, d, k_out=ks, k_block=len(ks), j_block=64 if N >= 64 else 256)
    params = np.array([N, L, R, gamma, s, N_rho, M, seed], dtype=np.float64)
    np.savez(os.path.join(HERE, name + ".npz"), modes=ks, Q=q, params=params, kind=np.array(kind))
    print(f"{name}: {len(ks)} modes in {time.time() - t0:.1f} s", flush=True)


if __name__ == "__main__":
    for n in (sys.argv[1:] or list(CASES) + list(BROADBAND) + list(CASES_2D) + list(PAPER_128)):
        if n in CASES_2D:
            make2d(n)
        elif n in PAPER_128:
            make_paper128(n)
        else:
            make(n)
