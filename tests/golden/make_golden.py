"""Write the stored expected values used by the GPU parity tests at sizes where
the oracle cannot run inside a test: Q_k of the FP64 direct-sum oracle at a
sample of output modes, for the medium (32^3) and large (64^3) workloads.

Calls only `oracle` and `workloads` (seeded inputs).  Run from the repository
root:  python tests/golden/make_golden.py [name ...]
Each case writes tests/golden/<name>.npz with arrays
  modes  int64 [n, 3]   sampled output modes k
  Q      complex128 [n] oracle Q_k
  params float64 [8]    N, L, R, gamma, s, N_rho, M, seed
  kind   input recipe code (0: two Maxwellians at +-2 e1, 1: random mixture)
"""
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle      # noqa: E402
import workloads   # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))

CASES = {
    # name: (N, L, R, gamma, s, N_rho, M, seed, kind, n_random)
    "medium_s050": (32, 8.0, 4.0, 0.0, 0.50, 32, 110, 0, 0, 48),
    "medium_s025": (32, 8.0, 4.0, 0.0, 0.25, 32, 110, 1, 0, 16),
    "medium_s075": (32, 8.0, 4.0, 0.0, 0.75, 32, 110, 2, 0, 16),
    "medium_gm1": (32, 8.0, 4.0, -1.0, 0.50, 32, 110, 3, 0, 16),
    "medium_gp1": (32, 8.0, 4.0, 1.0, 0.50, 32, 110, 4, 0, 16),
    "large_s050": (64, 10.0, 5.0, 0.0, 0.50, 64, 302, 0, 1, 16),
}


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
    mix = workloads.two_maxwellians(seed) if kind == 0 else workloads.random_mixture(seed)
    return workloads.to_spectral(mix.sample(N, L))


def make(name):
    N, L, R, gamma, s, N_rho, M, seed, kind, nr = CASES[name]
    d = oracle.Discretization.power(N, L, R, gamma, s, N_rho, M)
    f = input_of(N, L, seed, kind)
    ks = sample_modes(N, nr, seed)
    t0 = time.time()
    q = oracle.collision_direct(f, d, k_out=ks, k_block=len(ks), j_block=128 if N >= 64 else 512)
    params = np.array([N, L, R, gamma, s, N_rho, M, seed], dtype=np.float64)
    np.savez(os.path.join(HERE, name + ".npz"), modes=ks, Q=q, params=params, kind=np.array(kind))
    print(f"{name}: {len(ks)} modes in {time.time() - t0:.1f} s")


if __name__ == "__main__":
    for n in (sys.argv[1:] or list(CASES)):
        make(n)
