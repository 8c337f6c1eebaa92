"""Pins of the seeded input generators.

The spectral projection (trapezoid rule, Section 2's inner product) of a
Maxwellian that has decayed at the box edge must reproduce its Fourier
coefficients (2L)^-3 e^{-i pi k.u/L} e^{-T (pi |k| / L)^2 / 2}, and the
generators must be deterministic in their seed.
"""
import math

import numpy as np

import workloads


def test_projection_of_maxwellian_matches_fourier_transform():
    N, L, T = 32, 8.0, 1.2
    u = (0.7, -0.4, 0.25)
    fh = workloads.to_spectral(workloads.maxwellian_on_grid(N, L, 1.0, u, T))
    k = workloads.mode_indices(N).astype(float)
    K1, K2, K3 = np.meshgrid(k, k, k, indexing="ij")
    exact = (2 * L) ** -3 * np.exp(-1j * math.pi / L * (K1 * u[0] + K2 * u[1] + K3 * u[2])) \
        * np.exp(-0.5 * T * (math.pi / L) ** 2 * (K1 ** 2 + K2 ** 2 + K3 ** 2))
    h = N // 2
    exact[h, :, :] = exact[:, h, :] = exact[:, :, h] = 0
    # aliasing ~ e^{-T (pi (N/2+1)/L)^2 / 2} and the box tail ~ e^{-(L-|u|)^2/2T}: both < 1e-9
    assert np.max(np.abs(fh - exact)) < 1e-9 * (2 * L) ** -3
    assert fh[h].max() == 0 and fh[:, h].max() == 0


def test_seeded_determinism_and_ranges():
    a = workloads.two_maxwellians(5)
    b = workloads.two_maxwellians(5)
    assert a == b and 0.4 <= a.weights[0] <= 0.6 and abs(sum(a.weights) - 1) < 1e-15
    m = workloads.random_mixture(11)
    assert 2 <= len(m.weights) <= 5 and abs(sum(m.weights) - 1) < 1e-12
    assert all(0.5 <= t <= 1.5 for t in m.temps)
    assert all(abs(c) <= 3 for cc in m.centers for c in cc)
    cells = workloads.cell_batch(64, 3)
    assert {n for n, _ in cells} <= {16, 24, 32}
    reqs = workloads.request_stream(100.0, 2.0, 1)
    assert all(r[1] in (16, 32, 48, 64) for r in reqs)
    assert 100 < len(reqs) < 300
