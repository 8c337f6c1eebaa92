#!/usr/bin/env python
"""Throughput of the non-cutoff collision operator on one MI355X.

A step is one Heun step (two evaluations of Q(f, f), eq. realQ, plus the
update) of the medium workload: N = 32^3 modes on [-8, 8]^3, R = 4,
N_rho = 32 Gauss-Legendre nodes, M = 110 Lebedev points, gamma = 0,
s = 0.5, dt = 0.01, two-Maxwellian initial data.  The headline `value` is
Q evaluations per second of the FP32-bulk / FP64-accumulate path; the plain
FP64 path is timed beside it, and both are checked against each other and
against the CPU oracle on a mode sample.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-large] [--no-cpu-baseline]

Prints one JSON line.  Inputs are resident in HBM before the timed region.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK = {"fp32": 157.3, "fp64": 78.6}          # TFLOP/s, MI355X vector ALU (dense)
HBM_PEAK = 8.0e12                                # B/s

MEDIUM = dict(N=32, L=8.0, R=4.0, gamma=0.0, s=0.5, N_rho=32, M=110)
LARGE = dict(N=64, L=10.0, R=5.0, gamma=0.0, s=0.5, N_rho=64, M=302)
DT = 0.01


# ---------------------------------------------------------------- flop model
def fft_flops(P: int) -> float:
    """Nominal flops of one complex length-P FFT: 5 P log2 P."""
    return 5.0 * P * math.log2(P)


def flop_model(N: int, npairs: int):
    """Algorithmic flops of one evaluation, split by kernel (pairs packed two by two).

    zinv  : (N-1)^2 length-P inverse transforms + 12 flops/mode of modulation
    plane : per z-plane, 2(N-1) + 2P length-P transforms + the complex*real product (2P^2)
    zfwd  : (N-1)^2 forward transforms + 48 flops per half-spectrum mode (split + weight + acc)
    prep  : f on the padded grid: (N-1)^2 + P(N-1) + P^2 transforms
    """
    P = 3 * N // 2
    n1 = N - 1
    nh = (n1 * n1 + 1) // 2
    npt = npairs // 2
    F = fft_flops(P)
    per_pt = {
        "zinv": n1 * n1 * F + 12.0 * n1 ** 3,
        "plane": P * ((2 * n1 + 2 * P) * F + 2.0 * P * P),
        "zfwd": n1 * n1 * F + 48.0 * nh * n1,
    }
    out = {k: v * npt for k, v in per_pt.items()}
    out["prep"] = (n1 * n1 + P * n1 + P * P) * F
    out["plane_per_pt"] = per_pt["plane"]
    out["total"] = sum(out[k] for k in ("zinv", "plane", "zfwd", "prep"))
    return out


def table_bytes(N: int, npairs: int, esz: int) -> int:
    n1 = N - 1
    return npairs * ((n1 * n1 + 1) // 2) * n1 * esz


STAGES = ("prep", "zinv", "plane", "zfwd", "finalize")


def stage_model(N: int, npairs: int, esz: int):
    """Algorithmic flops and HBM bytes per evaluation of each pipeline stage.

    Flops are the method's own (flop_model: FFTs at 5 P log2 P, modulation,
    product, split and weighting).  Bytes are the method's own HBM traffic
    only: the weight table (read once by the z-forward stage), f_hat read by the
    ingest and Q_hat written by the finalisation.  The pipeline intermediates
    (the z-inverse output A and the plane output B, written once and read
    once) are not algorithmic bytes: they appear as measured `traffic`."""
    fm = flop_model(N, npairs)
    n3 = N ** 3 * 16
    return {"prep": (fm["prep"], n3), "zinv": (fm["zinv"], 0), "plane": (fm["plane"], 0),
            "zfwd": (fm["zfwd"], table_bytes(N, npairs, esz)), "finalize": (0.0, n3)}


def roof(flops: float, nbytes: float, seconds: float, peak_tflops: float):
    """Roofline object of one kernel launch (or one evaluation): the bound is
    the larger of the two algorithmic times (bytes / 8 TB/s, flops / vector
    peak); `achieved` is that quantity per second, `frac` = achieved / peak."""
    t_alu = flops / (peak_tflops * 1e12)
    t_hbm = nbytes / HBM_PEAK
    if t_alu >= t_hbm:
        ach = flops / seconds / 1e12
        return {"bound": "alu", "achieved": round(ach, 3), "peak": peak_tflops, "unit": "TFLOP/s",
                "frac": round(ach / peak_tflops, 4)}
    ach = nbytes / seconds / 1e9
    return {"bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK / 1e9, "unit": "GB/s",
            "frac": round(ach / (HBM_PEAK / 1e9), 4)}


# --------------------------------------------------------------- GPU timing
def time_steps(bzq, torch, cfg, prec, fhat_np, steps, warmup):
    """Time `steps` Heun steps (one bzq_step call) with HIP events around the
    plane-stage launches only (the dominant kernel, for the roofline), then run
    the same steps again with events around every launch for the per-stage
    breakdown."""
    plan = bzq.Plan(cfg["N"], cfg["L"], cfg["R"], cfg["gamma"], cfg["s"], cfg["N_rho"], cfg["M"],
                    precision=prec)
    f0 = torch.from_numpy(fhat_np).to("cuda")
    plan.autotune(f0)                           # kernel schedule (cached after the first run)
    f = f0.clone()
    if warmup:
        plan.step(f, DT, warmup)
    f.copy_(f0)
    torch.cuda.synchronize()
    plan.set_timing(True, stages=("plane",))
    st = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e0.record(st)
    plan.step(f, DT, steps)
    e1.record(st)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = e0.elapsed_time(e1)
    plane = plan.stage_times()["plane"]
    # per-stage breakdown (events on every launch), outside the timed region
    f.copy_(f0)
    plan.set_timing(True)
    plan.step(f, DT, steps)
    stages = plan.stage_times()
    plan.set_timing(False)
    stages["plane_timed_region"] = plane
    q = plan.collision(f0)
    torch.cuda.synchronize()
    return plan, ms, wall, stages, q


def kernel_hash() -> str:
    h = hashlib.sha256()
    for name in ("kernels.hip", "fft.hpp"):
        with open(os.path.join(ROOT, "paper_2004_11239_amd", "csrc", name), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def sched_tag(sched: dict) -> str:
    return f"{sched['zinv']}/{sched['plane']}/{sched['zfwd']}/{sched['s_target']}"


def stage_variant_tag(sched: dict, stage: str) -> str:
    """The part of a schedule that selects a stage's kernel and launch shape."""
    if stage in ("zinv", "plane"):
        return str(sched[stage])
    if stage == "zfwd":
        return f"{sched['zfwd']}/{sched['s_target']}"
    return "-"


def traffic_from_profiles(workload: str, prec: str, sched: dict):
    """Measured HBM bytes per evaluation of each stage (FETCH_SIZE and WRITE_SIZE
    counters, scaled by the copy calibration) from the committed summary
    profiles/traffic_<workload>_<prec>.md: {stage: (read, write, launches per
    evaluation, kernel)}.  Stages whose record was taken with other kernel
    sources or another kernel variant are left out."""
    path = os.path.join(ROOT, "profiles", f"traffic_{workload}_{prec}.md")
    out = {}
    if not os.path.exists(path):
        return out
    h = kernel_hash()
    with open(path) as fh:
        for line in fh:
            if not line.startswith("traffic:"):
                continue
            vals = dict(kv.split("=", 1) for kv in line.split()[1:])
            st = vals.get("stage")
            if vals.get("kernel_hash") != h or st not in STAGES or vals.get("variant") != stage_variant_tag(sched, st):
                continue
            try:
                # kernel names are written without blanks
                out[vals["stage"]] = (float(vals["read_per_eval"]), float(vals["write_per_eval"]),
                                      float(vals["launches_per_eval"]), vals["kernel"])
            except (KeyError, ValueError):
                continue
    return out


def stage_rooflines(N: int, npairs: int, esz: int, stages: dict, n_evals: int, traffic: dict):
    """Roofline object per stage from the HIP-event durations of its launches
    (stages[name] = (total ms, launches) over n_evals evaluations): per launch,
    the algorithmic flops and bytes of stage_model divided by the launches of
    an evaluation, over the average launch duration; `traffic` is the measured
    HBM bytes per launch (read + write) when a matching counter record exists,
    with its ratio to the algorithmic bytes."""
    model = stage_model(N, npairs, esz)
    peak = PEAK["fp32"] if esz == 4 else PEAK["fp64"]
    out = {}
    for name in STAGES:
        if name not in stages or stages[name][1] == 0:
            continue
        ms, launches = stages[name]
        per_eval = launches / n_evals
        fl, by = model[name]
        avg_s = ms * 1e-3 / launches
        r = roof(fl / per_eval, by / per_eval, avg_s, peak)
        t = traffic.get(name)
        r["traffic"] = round((t[0] + t[1]) / per_eval) if t else None
        r["traffic_over_alg_bytes"] = (round((t[0] + t[1]) / by, 2) if (t and by > 0) else None)
        r.update({"avg_launch_ms": round(avg_s * 1e3, 5), "launches_per_eval": round(per_eval, 3),
                  "alg_flop_per_launch": fl / per_eval, "alg_bytes_per_launch": by / per_eval,
                  "ms_per_eval": round(ms / n_evals, 4)})
        out[name] = r
    return out


# ------------------------------------------------------- batched and served
def batch_bench(bzq, torch, n_cells, steps, seed=0):
    """Independent cells, N drawn from {16, 24, 32} (50/30/20 %), N_rho = N,
    M = 110, gamma = 0, s = 0.5, FP32 bulk; one graph-captured Heun step of the
    whole batch per step."""
    import workloads
    t0 = time.perf_counter()
    cells = workloads.cell_batch(n_cells, seed)
    plans = {N: bzq.Plan(N, 8.0, 4.0, 0.0, 0.5, N, 110, precision="fp32") for N in (16, 24, 32)}
    fs = [torch.from_numpy(f).to("cuda") for _, f in cells]
    for N, p in plans.items():                 # kernel schedule per plan, tuned on one of its cells
        p.autotune(fs[next(i for i, (n, _) in enumerate(cells) if n == N)])
    batch = bzq.Batch([plans[N] for N, _ in cells], fs, cells_per_launch=0)
    setup = time.perf_counter() - t0
    batch.step(0.01, 1, use_graph=True)          # capture + warm-up
    torch.cuda.synchronize()
    st = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(st)
    batch.step(0.01, steps, use_graph=True)
    e1.record(st)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    out = {"workload": f"{n_cells} cells, N in {{16,24,32}} (50/30/20%), N_rho=N, M=110, gamma=0, s=0.5, "
                       f"FP32 bulk / FP64 accumulate, graph-captured Heun step",
           "cells_steps_per_s": round(n_cells * steps / (ms * 1e-3), 2),
           "q_evals_per_s": round(2 * n_cells * steps / (ms * 1e-3), 2),
           "ms_per_step": round(ms / steps, 2), "steps": steps,
           "groups": batch.groups(), "setup_s": round(setup, 1),
           "workspace_gb": round(batch.device_bytes() / 1e9, 2)}
    # the batch's roofline: per cell, two evaluations of the whole-path floor
    # (the method's own flops and bytes at that N, binding roof per cell)
    counts = {}
    for N, _ in cells:
        counts[N] = counts.get(N, 0) + 1
    roof_ms = 0.0
    for N, n in counts.items():
        nreal = N * (110 // 2)
        roof_ms += 2 * n * whole_path(N, nreal + (nreal & 1), 4, 1.0)["t_roof_ms"]
    out["roofline"] = {"t_roof_ms_per_step": round(roof_ms, 2),
                       "frac_of_roof": round(roof_ms / (ms / steps), 4),
                       "cells_by_N": {str(k): v for k, v in sorted(counts.items())}}
    batch.destroy()
    # each size's cells alone (same plans, tuned cells per launch from the
    # cache): how far each group is from its own roof, and whether the groups'
    # times add up to the whole batch's
    per_group = []
    for N in sorted(counts):
        idx = [i for i, (n, _) in enumerate(cells) if n == N]
        b = bzq.Batch([plans[N]] * len(idx), [fs[i] for i in idx], cells_per_launch=0)
        b.step(0.01, 1, use_graph=True)
        torch.cuda.synchronize()
        g0, g1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        g0.record(st)
        b.step(0.01, steps, use_graph=True)
        g1.record(st)
        torch.cuda.synchronize()
        gms = g0.elapsed_time(g1) / steps
        nreal = N * (110 // 2)
        groof = 2 * len(idx) * whole_path(N, nreal + (nreal & 1), 4, 1.0)["t_roof_ms"]
        per_group.append({"N": N, "cells": len(idx), "cells_per_launch": b.groups()[0]["cells_per_launch"],
                          "ms_per_step": round(gms, 2), "t_roof_ms_per_step": round(groof, 2),
                          "frac_of_roof": round(groof / gms, 4)})
        b.destroy()
    out["groups_alone"] = per_group
    out["groups_alone_ms_sum"] = round(sum(g["ms_per_step"] for g in per_group), 2)
    return out


def serve_bench(bzq, rates, duration, precision="fp32", q_fraction=0.0, max_queued=32):
    """The served form: Poisson arrivals at each rate (req/s) for `duration`
    seconds against one server (plans stay cached across the rates; each new
    plan's schedule is tuned on its first request, during the warm-up), with
    a bounded queue of max_queued waiting requests."""
    from paper_2004_11239_amd import serve
    srv = bzq.Server(64 << 30, 4, max_queued=max_queued, tune=True)
    try:
        return [serve.run(r, duration, seed=0, slots=4, precision=precision, n_steps=10, server=srv,
                          max_queued=max_queued, q_fraction=q_fraction) for r in rates]
    finally:
        srv.destroy()


def whole_path(N, npairs, esz, per_eval_ms, traffic=None):
    """Whole-evaluation roofline: the method's own HBM bytes (weight table, f in,
    Q out) and its flops (flop_model) against the MI355X peaks; the binding
    roof is the larger of the two times.  With a complete per-stage traffic
    record, the measured HBM bytes per evaluation and their ratio to the
    algorithmic bytes."""
    fm = flop_model(N, npairs)
    tb = table_bytes(N, npairs, esz) + 2 * N ** 3 * 16
    t = per_eval_ms * 1e-3
    peak = PEAK["fp32"] if esz == 4 else PEAK["fp64"]
    t_roof = max(tb / HBM_PEAK, fm["total"] / (peak * 1e12))
    out = {"alg_gflop_per_eval": round(fm["total"] / 1e9, 3),
           "tflops_whole_path": round(fm["total"] / t / 1e12, 3),
           "alg_bytes_per_eval": tb, "hbm_gbps_alg": round(tb / t / 1e9, 1),
           "t_roof_ms": round(t_roof * 1e3, 4), "frac_of_roof": round(t_roof / t, 4),
           "binding_roof": "alu" if fm["total"] / (peak * 1e12) > tb / HBM_PEAK else "hbm"}
    if traffic and all(k in traffic for k in ("zinv", "plane", "zfwd")):
        meas = sum(v[0] + v[1] for v in traffic.values())
        out["traffic_per_eval"] = round(meas)
        out["traffic_over_alg_bytes"] = round(meas / tb, 2)
    return out


# ---------------------------------------------------------------- CPU oracle
def _blas_threads() -> int:
    try:
        from threadpoolctl import threadpool_info
        return max([i.get("num_threads", 1) for i in threadpool_info()] or [1])
    except Exception:
        return os.cpu_count() or 1


def cpu_baseline(cfg, fhat_np, n_modes=1536, seed=0):
    import numpy as np
    import oracle
    blas_threads = _blas_threads()
    d = oracle.Discretization.power(cfg["N"], cfg["L"], cfg["R"], cfg["gamma"], cfg["s"],
                                    cfg["N_rho"], cfg["M"])
    modes = oracle.mode_vectors(cfg["N"])
    rng = np.random.default_rng(seed)
    ks = modes[rng.choice(len(modes), size=n_modes, replace=False)]
    t0 = time.perf_counter()
    q = oracle.collision_direct(fhat_np, d, k_out=ks, k_block=256)
    t = time.perf_counter() - t0
    value = n_modes / (t * len(modes))
    return ks, q, t, {"value": value, "unit": "Q evals/s", "cores": int(blas_threads),
                      "kind": "oracle",
                      "sample": f"{n_modes} of {len(modes)} output modes of one evaluation at the "
                                f"medium workload in {t:.1f} s (direct weighted sum, FP64, weight "
                                f"table included); value = sample / (time x modes)"}


def cpu_fft_baseline(cfg, fhat_np, n_nodes=32, reps=5, seed=0):
    """The same fast algorithm on the host (oracle.collision_fft: one pair of FP64
    FFTs of P^3 per quadrature node, no pairing or packing), timed on a sample of
    nodes with their weights precomputed (as the GPU plan's are) and scaled to
    whole evaluations."""
    import numpy as np
    import oracle
    d = oracle.Discretization.power(cfg["N"], cfg["L"], cfg["R"], cfg["gamma"], cfg["s"],
                                    cfg["N_rho"], cfg["M"])
    J = cfg["N_rho"] * cfg["M"]
    nodes = np.sort(np.random.default_rng(seed).choice(J, size=n_nodes, replace=False))
    T = oracle.weight_table(d, oracle.mode_vectors(cfg["N"]), nodes=nodes)
    workers = os.cpu_count() or 1
    t0 = time.perf_counter()
    for _ in range(reps):
        oracle.collision_fft(fhat_np, d, nodes=nodes, T=T, workers=workers)
    t = (time.perf_counter() - t0) / reps
    return {"value": n_nodes / (t * J), "unit": "Q evals/s", "cores": workers, "kind": "cpu_fft",
            "sample": f"{n_nodes} of {J} quadrature nodes of one evaluation at the medium workload, "
                      f"{reps} repetitions, {t:.3f} s each (scipy.fft, FP64, weights precomputed); "
                      f"value = sample / (time x nodes)"}


def bench_2d(bzq, torch, n_evals=20):
    """The 2-D operator at Table 1's largest setting (N = N_rho = 64, N_sigma = 32,
    R = 6, L = (3 + sqrt 2) R / 4, kernel b3 of Section 5.2), BKW input at t = 0:
    evals/s in both precisions and the L_inf error against the closed-form Q."""
    import numpy as np
    import workloads
    N, R = 64, 6.0
    L = (3 + math.sqrt(2)) * R / 4
    K = 0.5
    # f sampled, and the error taken, on the cell-centred grid (Table 1's grid)
    f = workloads.to_spectral_2d(workloads.bkw2d_profile_on_grid(N, L, K, centred=True), centred=True)
    fd = torch.from_numpy(f).to("cuda")
    out = {"workload": "2-D collision N=64^2 N_rho=64 N_sigma=32 (midpoint) R=6 L=6.62 b3, BKW at t=0"}
    v = workloads.velocity_grid(N, L, centred=True)
    v2 = v[:, None] ** 2 + v[None, :] ** 2
    exact = np.exp(-v2 / (2 * K)) / (2 * math.pi * K) * (1 - K) ** 2 / (4 * K ** 4) * 0.125 * (
        8 * K * K - 8 * K * v2 + v2 * v2)
    kk = np.fft.fftfreq(N, 1.0 / N)
    sgn = np.where(np.arange(N) % 2 == 0, 1.0, -1.0) * np.exp(1j * math.pi * kk / N)
    for prec in ("fp32", "fp64"):
        plan = bzq.Plan2D(N, L, R, 0.0, (1.0 / (8 * math.pi), 0.0, 0.0), N, 32, precision=prec)
        q = torch.empty_like(fd)
        for _ in range(3):
            plan.collision(fd, q)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(n_evals):
            plan.collision(fd, q)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / n_evals
        qn = q.cpu().numpy()
        qphys = np.real(np.fft.ifft2(qn * sgn[:, None] * sgn[None, :])) * N * N
        out[prec] = {"evals_per_s": round(1e3 / ms, 2), "ms_per_eval": round(ms, 4),
                     "table1_linf_error": float(np.max(np.abs(qphys - exact)))}
        # whole-evaluation roofline: per pair-two 2 (N-1+P) length-P transforms
        # and the P^2 product; bytes: the weight table and f, Q
        P, n1 = 3 * N // 2, N - 1
        npairs = N * 16                      # N_rho = N radii x N_sigma / 2 circle pairs
        flops = npairs // 2 * (2 * (n1 + P) * fft_flops(P) + 2.0 * P * P)
        nbytes = npairs * ((n1 * n1 + 1) // 2) * (4 if prec == "fp32" else 8) + 2 * N * N * 16
        peak = PEAK["fp32" if prec == "fp32" else "fp64"]
        t_alu, t_hbm = flops / (peak * 1e12), nbytes / HBM_PEAK
        out[prec]["roofline"] = {"bound": "alu" if t_alu >= t_hbm else "hbm",
                                 "alg_gflop": round(flops / 1e9, 3), "alg_mb": round(nbytes / 1e6, 2),
                                 "tflops": round(flops / (ms * 1e-3) / 1e12, 2),
                                 "frac": round(max(t_alu, t_hbm) / (ms * 1e-3), 4)}
        plan.destroy()
    out["table1_paper_b3_N64"] = 3.1950e-09
    return out


def cpu_baseline_2d(n_modes=64, seed=0):
    """The 2-D oracle (direct weighted sum, FP64) at the 2-D bench setting,
    timed over a sample of output modes, scaled to evals/s."""
    import numpy as np
    import oracle
    import workloads
    N, R = 64, 6.0
    L = (3 + math.sqrt(2)) * R / 4
    f = workloads.to_spectral_2d(workloads.bkw2d_profile_on_grid(N, L, 0.5))
    d = oracle.collision2d.Discretization2D(N, L, R, 0.0, oracle.collision2d.PAPER_KERNELS_2D["b3"], N, 32)
    rng = np.random.default_rng(seed)
    ks = rng.integers(-(N // 2 - 1), N // 2, size=(n_modes, 2))
    t0 = time.perf_counter()
    oracle.collision2d.collision_direct2d(f, d, k_out=ks)
    t = time.perf_counter() - t0
    total = (N - 1) ** 2
    return {"value": round(n_modes / (t * total), 6), "unit": "Q evals/s", "cores": int(_blas_threads()),
            "kind": "oracle",
            "sample": f"{n_modes} of {total} output modes of one 2-D evaluation (N=64, N_rho=64, N_sigma=32) "
                      f"in {t:.1f} s (direct weighted sum, FP64, weight table included)"}


def bench_otf(bzq, torch, cfg, fhat_np, q_ref, n_evals=3):
    """Weights on the fly at the N = 64 workload: evals/s, plan bytes and plan
    creation time against the table plan, and the difference of the results."""
    import numpy as np
    fd = torch.from_numpy(fhat_np).to("cuda")
    out = {}
    for prec in ("fp32", "fp64"):
        row = {}
        for mode in ("table", "otf"):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            p = bzq.Plan(cfg["N"], cfg["L"], cfg["R"], cfg["gamma"], cfg["s"], cfg["N_rho"], cfg["M"],
                         precision=prec, weights=mode)
            torch.cuda.synchronize()
            t_create = time.perf_counter() - t0
            q = torch.empty_like(fd)
            p.collision(fd, q)
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(n_evals):
                p.collision(fd, q)
            e1.record()
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1) / n_evals
            row[mode] = {"ms_per_eval": round(ms, 3), "plan_create_s": round(t_create, 3),
                         "plan_device_MB": round(p.device_bytes() / 2 ** 20, 1)}
            if mode == "otf":
                qn = q.cpu().numpy()
                row["otf_vs_table_rel"] = float(np.linalg.norm(qn - qt) / np.linalg.norm(qt))
            else:
                qt = q.cpu().numpy()
            p.destroy()
            del p, q
            torch.cuda.empty_cache()
        out[prec] = row
    out["workload"] = "N=64^3 M=302 N_rho=64, the large workload"
    return out


HUGE = dict(N=128, L=10.0, R=5.0, gamma=0.0, s=0.5, N_rho=128, M=302)


def bench_n128(bzq, torch, cfg=HUGE):
    """N = 128 (P = 192) with weights on the fly, in the large workload's box:
    evals/s per precision, plan device memory against what a stored weight
    table would take, plan creation time, per-stage times and the FP32 result
    against the FP64 one."""
    import numpy as np
    import workloads
    f = workloads.to_spectral(workloads.random_mixture(0).sample(cfg["N"], cfg["L"]))
    fd = torch.from_numpy(f).to("cuda")
    out = {"workload": "N=128^3 L=10 R=5 N_rho=128 M=302 Lebedev gamma=0 s=0.5, weights on the fly "
                       "(random Maxwellian mixture, seed 0)"}
    qs = {}
    for prec in ("fp32", "fp64"):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        p = bzq.Plan(cfg["N"], cfg["L"], cfg["R"], cfg["gamma"], cfg["s"], cfg["N_rho"], cfg["M"],
                     precision=prec, weights="otf")
        torch.cuda.synchronize()
        t_create = time.perf_counter() - t0
        q = torch.empty_like(fd)
        p.collision(fd, q)                      # warm-up
        p.set_timing(True)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record()
        p.collision(fd, q)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1)
        st = p.stage_times()
        info = p.info()
        out[prec] = {"evals_per_s": round(1000.0 / ms, 3), "ms_per_eval": round(ms, 1),
                     "stage_ms_per_eval": {k: round(v[0], 1) for k, v in st.items()},
                     "plan_device_MB": round(p.device_bytes() / 2 ** 20, 1),
                     "table_plan_would_hold_GB": round(
                         bzq.plan_bytes_estimate(cfg["N"], cfg["N_rho"], cfg["M"], prec) / 2 ** 30, 1),
                     "plan_create_s": round(t_create, 2), "npairs": info["npairs"],
                     "pairs_per_chunk": info["pairs_per_chunk"]}
        qs[prec] = q.cpu().numpy()
        p.destroy()
        del p, q
        torch.cuda.empty_cache()
    out["err_fp32_vs_fp64"] = float(np.linalg.norm(qs["fp32"] - qs["fp64"]) / np.linalg.norm(qs["fp64"]))
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-large", dest="large", action="store_false",
                    help="skip the N=64 workload (timed by default beside the headline)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-otf", dest="otf", action="store_false",
                    help="skip the plans with weights on the fly (beside the N = 64 workload)")
    ap.add_argument("--no-n128", dest="n128", action="store_false",
                    help="skip the N = 128 plans with weights on the fly")
    ap.add_argument("--no-2d", dest="two_d", action="store_false",
                    help="skip the 2-D operator at Table 1's N = 64 setting")
    ap.add_argument("--batch-cells", type=int, default=4096, help="cells of the batched form (0: skip)")
    ap.add_argument("--serve-rates", default="10,25,50,100,200,500,1000,2000,5000",
                    help="request rates (req/s) of the served form ('': skip)")
    ap.add_argument("--serve-duration", type=float, default=3.0)
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="also run 3 device-to-device copies of MIB MiB (reference kernel for "
                         "the FETCH_SIZE / WRITE_SIZE counters) and exit")
    ap.add_argument("--profile-workload", choices=("medium", "large"), default=None,
                    help="only run --profile-evals evaluations of that workload with the tuned schedule "
                         "(for counter runs under rocprofv3) and exit")
    ap.add_argument("--profile-prec", choices=("fp32", "fp64"), default="fp32")
    ap.add_argument("--profile-evals", type=int, default=3)
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(json.dumps({"error": "bench.py measures one GPU: the library has no multi-GPU path "
                                   "(an evaluation would shard its quadrature pairs across GPUs and sum "
                                   "the partial Q with one all-reduce); run with --gpus 1"}))
        sys.exit(2)

    import numpy as np
    import torch
    import workloads
    from paper_2004_11239_amd import bzq

    if args.copy_calibration:
        n = args.copy_calibration * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration_bytes": n * 4, "copies": 3}))
        return

    if args.profile_workload:
        cfg = MEDIUM if args.profile_workload == "medium" else LARGE
        mix = workloads.two_maxwellians(0) if cfg is MEDIUM else workloads.random_mixture(0)
        fd = torch.from_numpy(workloads.to_spectral(mix.sample(cfg["N"], cfg["L"]))).to("cuda")
        plan = bzq.Plan(cfg["N"], cfg["L"], cfg["R"], cfg["gamma"], cfg["s"], cfg["N_rho"], cfg["M"],
                        precision=args.profile_prec)
        plan.autotune(fd)
        q = torch.empty_like(fd)
        torch.cuda.synchronize()
        print(json.dumps({"profile_start": True}), flush=True)
        for _ in range(args.profile_evals):
            plan.collision(fd, q)
        torch.cuda.synchronize()
        print(json.dumps({"profile_workload": args.profile_workload, "precision": args.profile_prec,
                          "evals": args.profile_evals, "schedule": plan.schedule(), "info": plan.info(),
                          "kernel_hash": kernel_hash()}), flush=True)
        return

    cfg = MEDIUM
    fhat = workloads.to_spectral(workloads.two_maxwellians(0).sample(cfg["N"], cfg["L"]))
    # FP32-bulk / FP64-accumulate (headline) and the plain FP64 path
    p32, ms32, wall32, st32, q32 = time_steps(bzq, torch, cfg, "fp32", fhat, args.steps, args.warmup)
    steps64 = max(3, args.steps // 2)
    p64, ms64, wall64, st64, q64 = time_steps(bzq, torch, cfg, "fp64", fhat, steps64, max(1, args.warmup // 2))
    st64.pop("plane_timed_region")
    q32n, q64n = q32.cpu().numpy(), q64.cpu().numpy()
    err32_64 = float(np.linalg.norm(q32n - q64n) / np.linalg.norm(q64n))

    info = p32.info()
    npairs = info["npairs"]
    evals32 = 2 * args.steps
    value = evals32 / (ms32 * 1e-3)
    value64 = 2 * steps64 / (ms64 * 1e-3)
    sched32 = p32.schedule()
    tr32 = traffic_from_profiles("medium", "fp32", sched32)
    # dominant kernel: the plane transforms (stage 2), timed inside the timed region
    plane_ms, plane_n = st32.pop("plane_timed_region")
    roof_obj = stage_rooflines(cfg["N"], npairs, 4, {"plane": (plane_ms, plane_n)}, evals32, tr32)["plane"]
    roof_obj["kernel"] = (tr32["plane"][3] if "plane" in tr32 else
                          f"plane stage, schedule {sched_tag(sched32)}")
    roof_obj["traffic_note"] = ("measured HBM bytes per launch: the z-inverse output read and the plane "
                                "output written (pipeline intermediates; the stage has no algorithmic bytes)")
    # the paper's integrator: classical RK4 steps (4 evaluations each) with the tuned plan
    fd_rk = torch.from_numpy(fhat).to("cuda")
    p32.step(fd_rk, DT, 1, method="rk4")
    torch.cuda.synchronize()
    r0, r1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    n_rk = max(2, args.steps // 2)
    r0.record()
    p32.step(fd_rk, DT, n_rk, method="rk4")
    r1.record()
    torch.cuda.synchronize()
    rk_ms = r0.elapsed_time(r1) / n_rk
    rk4 = {"ms_per_step": round(rk_ms, 4), "evals_per_s": round(4e3 / rk_ms, 2), "steps": n_rk}
    per_eval_ms = ms32 / evals32
    whole = whole_path(cfg["N"], npairs, 4, ms32 / evals32, tr32)
    stage_ms = {k: round(v[0] / evals32, 4) for k, v in st32.items()}

    out = {
        "metric": "Q(f,f) evals/sec at N=32^3 (FP32 bulk, FP64 accumulate; FP64 path beside it)",
        "value": round(value, 3),
        "unit": "Q evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms32 / args.steps, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "Heun step (2 Q evals) N=32^3 L=8 R=4 N_rho=32 M=110 Lebedev "
                               "gamma=0 s=0.5 dt=0.01, two-Maxwellian input",
                   "N": cfg["N"], "L": cfg["L"], "R": cfg["R"], "N_rho": cfg["N_rho"], "M": cfg["M"],
                   "gamma": cfg["gamma"], "s": cfg["s"], "precision": "fp32 bulk, fp64 accumulate",
                   "antipodal_pairs": npairs},
        "roofline": roof_obj,
        "schedule": {"fp32": sched32, "fp64": p64.schedule()},
        "fp64": {"value": round(value64, 3), "ms_per_step": round(ms64 / steps64, 4),
                 "stage_ms_per_eval": {k: round(v[0] / (2 * steps64), 4) for k, v in st64.items()},
                 "kernels": stage_rooflines(cfg["N"], npairs, 8, st64, 2 * steps64,
                                            traffic_from_profiles("medium", "fp64", p64.schedule())),
                 "whole_path": whole_path(cfg["N"], npairs, 8, ms64 / (2 * steps64),
                                          traffic_from_profiles("medium", "fp64", p64.schedule()))},
        "err_fp32_vs_fp64": err32_64,
        "rk4_step": rk4,
        "stage_ms_per_eval": stage_ms,
        "kernels": stage_rooflines(cfg["N"], npairs, 4, st32, evals32, tr32),
        "whole_path": whole,
        "wall_s": {"fp32": round(wall32, 3), "fp64": round(wall64, 3)},
    }
    if args.large:
        cl = LARGE
        fl = workloads.to_spectral(workloads.random_mixture(0).sample(cl["N"], cl["L"]))
        large = {}
        qs = {}
        for prec in ("fp32", "fp64"):
            p, ms, wall, st, q = time_steps(bzq, torch, cl, prec, fl, 2, 1)
            st.pop("plane_timed_region")
            esz = 4 if prec == "fp32" else 8
            npl = p.info()["npairs"]
            tr = traffic_from_profiles("large", prec, p.schedule())
            large[prec] = {"evals_per_s": round(4 / (ms * 1e-3), 3), "ms_per_eval": round(ms / 4, 3),
                           "stage_ms_per_eval": {k: round(v[0] / 4, 3) for k, v in st.items()},
                           "schedule": p.schedule(),
                           "kernels": stage_rooflines(cl["N"], npl, esz, st, 4, tr),
                           "whole_path": whole_path(cl["N"], npl, esz, ms / 4, tr)}
            qs[prec] = q.cpu().numpy()
            del p
            torch.cuda.empty_cache()
        large["err_fp32_vs_fp64"] = float(np.linalg.norm(qs["fp32"] - qs["fp64"]) / np.linalg.norm(qs["fp64"]))
        out["large_N64"] = large
        if args.otf:
            out["weights_on_the_fly"] = bench_otf(bzq, torch, cl, fl, qs["fp64"])
    if args.n128:
        out["n128_on_the_fly"] = bench_n128(bzq, torch)
    if args.two_d:
        out["two_d"] = bench_2d(bzq, torch)
    if args.batch_cells > 0:
        out["batched"] = batch_bench(bzq, torch, args.batch_cells, 2)
        torch.cuda.empty_cache()
    if args.serve_rates:
        rates = [float(r) for r in args.serve_rates.split(",")]
        out["served"] = serve_bench(bzq, rates, args.serve_duration)
        out["served_fp64"] = serve_bench(bzq, rates, args.serve_duration, precision="fp64")
        out["served_mixed_q"] = serve_bench(bzq, [rates[0]], args.serve_duration, q_fraction=0.5)
    if not args.no_cpu_baseline:
        ks, qo, t, cb = cpu_baseline(cfg, fhat)
        idx = tuple(np.mod(ks, cfg["N"]).T)
        out["err_vs_oracle_sample"] = {
            "fp32": float(np.linalg.norm(q32n[idx] - qo) / np.linalg.norm(qo)),
            "fp64": float(np.linalg.norm(q64n[idx] - qo) / np.linalg.norm(qo))}
        out["cpu_baseline"] = cb
        out["cpu_fft_baseline"] = cpu_fft_baseline(cfg, fhat)
        if args.two_d:
            out["two_d"]["cpu_baseline"] = cpu_baseline_2d()
    else:
        out["cpu_baseline"] = None
    print(json.dumps(out))


if __name__ == "__main__":
    main()
