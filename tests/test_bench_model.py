"""The algorithmic flop and byte model behind bench.py's roofline objects.

The model counts, per pair-two (two antipodal pairs packed into one complex
transform), the length-P transforms of a zero-padded 3-D FFT pair whose input
is the (N-1)^3 cube of kept modes and whose kept output is that same cube
(eq. realQ of Section 4: one inverse and one forward transform per pair).
These tests count the transforms that pruning leaves by brute force over the
padded grid, compare the per-evaluation totals with the hot-path cost table
worked out from the paper's O(N_q N^{d+1} log N) accounting (Section 4), and
recompute the headline kernel's roof fraction from a committed kernel trace.
"""
import math
import os
import re

import numpy as np
import pytest

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _pruned_transform_counts(N):
    """Length-P transforms of one pruned inverse 3-D FFT (axis 3, then 2, then
    1) of the kept cube embedded in P^3, and of one pruned forward FFT that
    keeps only the cube: a transform along an axis is needed wherever its
    input line holds a nonzero value (inverse) or one of its outputs is kept
    (forward)."""
    P = 3 * N // 2
    n1 = N - 1
    nz = np.zeros((P, P, P), dtype=bool)
    nz[:n1, :n1, :n1] = True                  # where the kept modes sit (any placement works)
    inv = 0
    for axis in (2, 1, 0):
        inv += int(nz.any(axis=axis).sum())   # lines along `axis` with a nonzero input
        nz = nz.any(axis=axis, keepdims=True) & np.ones_like(nz)   # a transformed line is dense
    keep = np.zeros((P, P, P), dtype=bool)
    keep[:n1, :n1, :n1] = True
    fwd = 0
    need = keep
    for axis in (2, 1, 0):                    # last transform first: which lines feed a kept output
        fwd += int(need.any(axis=axis).sum())
        need = need.any(axis=axis, keepdims=True) & np.ones_like(need)
    return inv, fwd


@pytest.mark.parametrize("N", [8, 16, 32])
def test_flop_model_counts_the_pruned_transforms(N):
    P, n1 = 3 * N // 2, N - 1
    inv, fwd = _pruned_transform_counts(N)
    F = bench.fft_flops(P)
    per_pt = bench.flop_model(N, 2)            # one pair-two
    fft_part = (per_pt["zinv"] - 12.0 * n1 ** 3) + (per_pt["plane"] - 2.0 * P ** 3) \
        + (per_pt["zfwd"] - 48.0 * ((n1 * n1 + 1) // 2) * n1)
    assert fft_part == pytest.approx((inv + fwd) * F, rel=1e-12)
    # f on the padded grid: one pruned inverse transform per evaluation
    assert bench.flop_model(N, 2)["prep"] == pytest.approx(inv * F, rel=1e-12)


@pytest.mark.parametrize("N,npairs,gflop", [(16, 304, 0.234), (32, 1760, 12.9), (64, 9664, 658.0)])
def test_flop_model_matches_the_cost_table(N, npairs, gflop):
    """The hot-path cost table prices a pair at one pruned real C2R + R2C pair,
    2 x 2.5 P^3 log2(P^3) x 0.70 flops; the model's per-stage count lands
    within 10 % of it."""
    total = bench.flop_model(N, npairs)["total"] / 1e9
    assert abs(total - gflop) <= 0.10 * gflop, (N, total, gflop)


@pytest.mark.parametrize("esz,peak,ms", [(4, "fp32", 4.18), (8, "fp64", 8.37)])
def test_whole_path_roof_at_64(esz, peak, ms):
    """At N = 64 (9664 pairs) the binding roof is vector arithmetic: the
    weight table (9.8 GB FP32 as complex, here stored real) takes far less
    than the flops at the vector peak."""
    wp = bench.whole_path(64, 9664, esz, 1.0)
    assert wp["binding_roof"] == "alu"
    assert wp["t_roof_ms"] == pytest.approx(ms, rel=0.06)
    tb = bench.table_bytes(64, 9664, esz)
    assert tb == 9664 * ((63 * 63 + 1) // 2) * 63 * esz
    assert tb / bench.HBM_PEAK < 0.5 * wp["t_roof_ms"] * 1e-3


def test_roof_object_picks_the_binding_bound():
    alu = bench.roof(1e12, 1e9, 1.0, 157.3)
    assert alu["bound"] == "alu" and alu["frac"] == pytest.approx(1.0 / 157.3, abs=5e-5)
    hbm = bench.roof(1e9, 4e12, 1.0, 157.3)
    assert hbm["bound"] == "hbm" and hbm["frac"] == pytest.approx(0.5, rel=1e-6)


def test_headline_kernel_fraction_from_committed_trace():
    """The headline roofline object (plane stage at 32^3, FP32, one launch per
    evaluation) recomputed from the average duration in the committed kernel
    trace: 880 pair-twos' plane flops over that duration against the FP32
    vector peak."""
    path = os.path.join(ROOT, "profiles", "kernels_medium_N32.md")
    text = open(path).read()
    m = re.search(r"\| `k_plane_reg<float, 32, 48, 0>` \| (\d+) \| ([\d.]+) \| ([\d.]+) \|", text)
    assert m, "plane kernel row missing from the trace summary"
    avg_s = float(m.group(3)) * 1e-6
    flops = bench.flop_model(32, 1760)["plane"]
    frac = flops / avg_s / (bench.PEAK["fp32"] * 1e12)
    assert 0.30 < frac < 0.45, frac
    assert math.isclose(flops, 880 * bench.flop_model(32, 2)["plane"], rel_tol=1e-12)
