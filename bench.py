"""Benchmark of the BSDE solver library on one MI355X.

A step is one whole pricing job of the d=5 American geometric-basket put
(local volatility level_j (1 + 0.25 exp(-(log(S/100))^2)) with levels
U[0.15, 0.35], rho = 0.2, r = 0.05, K = S0 = 100, T = 1, penalty 1;
4096 random spatial points x 10 time nodes, total degree 3 (84 basis
functions), M = 1000 paths, N = 50 Euler steps, 10 Picard iterations) with
FP64 paths, sums and update: problem set-up (grid, basis matrix, device
least-squares factorisation, upload), every Picard iteration on the GPU
(paths, driver, reductions, least-squares update), the price/delta query
and tear-down.  `value` is Euler path-steps per second of whole jobs.

The one JSON line also carries:
  roofline      of the dominant kernel (the Monte Carlo path kernel of the
                job): algorithmic FLOP per path-step counted from the
                kernel's arithmetic, times the path-steps of one launch,
                over the launch's mean duration (HIP events taken by the
                dispatch on the solve's stream), against the FP64 vector
                peak;
  fp32_paths    the same job with FP32 paths and FP64 sums;
  accuracy_gate |d price|/K and |d delta| against the stored FP64 oracle
                results of every benchmark workload, in both precisions,
                with pass/fail against the accuracy target (penalty-100
                workloads are labelled "Picard not converged");
  d1_amer_put   the d=1 American put workload (128x16 points, M=4000,
                N=50, 8 iterations) in FP32 paths, with the issue-cycle
                model of its path kernel as a secondary roofline;
  batched_vs_fp64_per_problem  the d=1, 2, 5 workloads at penalty 1 in
                one batched FP32-path solve (hipGraph) against the same
                three solved one by one in FP64;
  serving       the request mix (d in {1,2,5,10}) at saturation and at 0.5
                and 0.9 of it, p50/p99 with the request counts, and the
                alone-versus-mix check on sampled requests;
  cpu_baseline  the oracle on a bounded sample of the same job, on one core
                and over all host cores (disjoint point ranges).

    python bench.py [--gpus 1] [--steps K] [--warmup W]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

FP32_VECTOR_PEAK = 157.3e12   # FLOP/s, MI355X (packed FMA)
FP64_VECTOR_PEAK = 78.6e12
SIMD_ISSUE_CYCLES_PEAK = 256 * 4 * 2.4e9   # 256 CUs x 4 SIMDs x 2.4 GHz
METRIC = "Euler path-steps/s + priced requests/s (p50/p99) at stated price/delta error"

# Gates of the accuracy target: |d price| <= tol * K, |d delta| <= tol
GATE = {"fp64": (1e-4, 1e-4), "fp32": (5e-4, 5e-3)}


# ---------------------------------------------------------------------------
# Algorithmic work of the path kernel
# ---------------------------------------------------------------------------
def index_set(d, eta, q=1.0):
    """The multi-indices (t, x_1, .., x_d) of the basis: total degree <= eta
    and, for q < 1, sum_v nu_v^q <= eta^q (Section 4.2, eq. hyper_set)."""
    out = []

    def rec(prefix, left):
        if len(prefix) == d + 1:
            if q >= 1.0 or sum(v ** q for v in prefix) <= eta ** q * (1 + 1e-12):
                out.append(tuple(prefix))
            return
        for a in range(left + 1):
            rec(prefix + [a], left - a)

    rec([], eta)
    return out


def live_channel_entries(d, eta, q=1.0):
    """(p, entries of the channel table the path kernel multiplies): every
    basis function for u; for a first derivative in variate v the functions
    nu with nu + e_v in the set, for a second derivative in x_j, x_k those
    with nu + e_j + e_k in it (differentiation lowers a Chebyshev factor's
    degree, so the other rows of those channels are zero)."""
    S = set(index_set(d, eta, q))

    def has(nu, *vs):
        m = list(nu)
        for v in vs:
            m[v] += 1
        return tuple(m) in S

    first = sum(has(nu, v) for nu in S for v in range(d + 1))
    second = sum(has(nu, 1 + j, 1 + k) for nu in S for j in range(d)
                 for k in range(j, d))
    return len(S), len(S) + first + second


def flop_per_path_step(d, p, C, live, N, vol="bump", payoff="put_geom"):
    """Algorithmic floating-point operations per Euler path-step of the path
    kernel (FMA = 2, add or multiply = 1, exp/log/sqrt/sin/cos = 1 each;
    integer Philox work and compares 0), counted from the kernel's
    arithmetic.  Returns (total, of which the basis-row x channel-table
    contraction).  live is the number of entries of the p x C channel table
    the contraction multiplies (live_channel_entries; p C for a dense one).

    Per asset and Euler step:
      one normal, half a Box-Muller pair: two uniform maps (FMA each), log,
      scale, sqrt, the angle's scale, cos and sin, two radius products:
      (4 + 3 + 1 + 2 + 2) / 2 = 6;
      (L G)_j with the prefix sum of the uniform correlation: 2 FMAs (d > 1);
      bump volatility: square, exp, FMA = 4;
      Euler update: 3 FMAs = 6.
    Per path (amortised over N):
      U and tau: 4; bridge normals: 6 per generated normal (4 ceil(d/4));
      state at tau per asset: back to x (2), (L G) of step j* (4), frozen
      volatility (4), frozen drift (2), X_tau (8), bridge correlation (4);
      Chebyshev values: (2 d + 1) variates x (map 2 + 3 per recurrence);
      basis rows: one product per function and row, 2 (p - 1);
      contraction: 2 live (at tau) + 2 p (u at T);
      generator: 2 (C - 1) + d (d + 1) (covariances);
      payoffs at tau and T; driver, path term and FP64 sums: 12."""
    eta_rec = 3
    normal = 6.0
    corr = 4.0 if d > 1 else 0.0
    volf = 4.0 if vol == "bump" else 0.0
    per_asset_step = normal + corr + volf + 6.0
    bridge = 6.0 * 4 * ((d + 3) // 4)
    at_tau = d * (2 + 4 + 4 + 2 + 8 + 4)
    # Chebyshev degree: p = binom(d + 1 + eta, eta) for the total degree
    eta = 0
    from math import comb
    while comb(d + 1 + eta, eta) < p:
        eta += 1
    cheb = (2 * d + 1) * (2 + eta_rec * max(0, eta - 1))
    basis = 2 * (p - 1)
    contraction = 2.0 * live
    uT = 2.0 * p
    gen = 2 * (C - 1) + d * (d + 1)
    pay = 2 * ((2 * d + 3) if payoff in ("put", "call") else (d + 3))
    per_path = 4 + bridge + at_tau + cheb + basis + contraction + uT + gen + pay + 12
    total = d * per_asset_step + per_path / N
    return total, contraction / N


# Secondary roofline of the d=1 FP32 path kernel: issue cycles of one wave
# per Euler path-step, each algorithmic operation priced at the cheapest
# instruction form that computes it with the issue costs measured on gfx950
# (profiles/valu_issue_rates_gfx950.md): FP32 adds, multiplies and FMAs with
# vector operands 3.2 cycles, integer and logic forms with vector operands
# 2.25 (v_bitop3_b32 included), forms with a scalar or literal operand,
# 64-bit integer multiply-adds, conversions and funnel shifts 4.1,
# transcendentals 8.3.
ISSUE_COST = {"f32v": 3.2, "intv": 2.25, "four": 4.1, "trans": 8.3}
ISSUE_CYCLES_D1_FP32 = {
    # 1/4 Philox4x32-10 block: 16 v_mad_u64_u32, three XORs with a uniform
    # operand, 15 three-input XORs with vector operands
    "normal_philox": (16 * ISSUE_COST["four"] + 3 * ISSUE_COST["four"] +
                      15 * ISSUE_COST["intv"]) / 4,
    # 1/2 Box-Muller pair: conversion and funnel shift, log, sqrt, sin, cos,
    # the uniform map's FMA and three multiplies
    "normal_box_muller": (2 * ISSUE_COST["four"] + 4 * ISSUE_COST["trans"] +
                          4 * ISSUE_COST["f32v"]) / 2,
    # volatility: square, exp, FMA
    "local_vol": 2 * ISSUE_COST["f32v"] + ISSUE_COST["trans"],
    # Euler update: two FMAs and an add
    "euler": 3 * ISSUE_COST["f32v"],
    # the compare that selects step j*
    "record": ISSUE_COST["intv"],
    # per path over N = 50: U and bridge Philox blocks, one Box-Muller pair,
    # 137 other FP32 operations (56 of them the products with the 41 live
    # channel-table entries and u at T)
    "per_path": (2 * (16 * ISSUE_COST["four"] + 3 * ISSUE_COST["four"] +
                      15 * ISSUE_COST["intv"]) +
                 2 * (2 * ISSUE_COST["four"] + 4 * ISSUE_COST["trans"] +
                      4 * ISSUE_COST["f32v"]) + 137 * ISSUE_COST["f32v"]) / 50.0,
}

# HBM traffic of one launch of the headline path kernel, from rocprofv3
# FETCH_SIZE and WRITE_SIZE (separate --pmc runs, KiB per dispatch),
# scaled by the plain-copy calibration (FETCH_SIZE x 2.0, WRITE_SIZE x 1.0,
# profiles/copy_calibration.md).  Valid only for the kernel sources whose
# hash is recorded with it and for the tiling it was taken at; otherwise
# the line reports null.
TRAFFIC = [
    {"sources_sha16": "ea70fccb41332a0b", "tiling": [1, 4],
     "fetch_kib": 14090.0, "write_kib": 934600.0,
     "profile": "profiles/path_kernel_d5_fp64_geo_basket_d5.md"},
    {"sources_sha16": "ea70fccb41332a0b", "tiling": [4, 1],
     "fetch_kib": 24310.0, "write_kib": 3686000.0,
     "profile": "profiles/path_kernel_d5_fp64_geo_basket_d5.md"},
    {"sources_sha16": "ea70fccb41332a0b", "tiling": [2, 2],
     "fetch_kib": 17950.0, "write_kib": 1832000.0,
     "profile": "profiles/path_kernel_d5_fp64_geo_basket_d5.md"},
]
# Counter-derived figures of the same kernel (same profiles, same guard):
# VALU issue = SQ_INSTS_VALU x 4 cycles / 1024 SIMDs / cycles, matrix cores
# busy = SQ_VALU_MFMA_BUSY_CYCLES / 1024 SIMDs / cycles, FP64 vector FLOP
# issued = 64 (2 FMA + MUL + ADD + TRANS) instructions per launch.
COUNTERS = [
    {"sources_sha16": "ea70fccb41332a0b", "tiling": [1, 4],
     "valu_issue": 0.907, "mfma_busy": 0.0,
     "fp64_vector_flop_per_launch": 7.45e11, "fp64_matrix_flop_per_launch": 0.0,
     "profile": "profiles/path_kernel_d5_fp64_geo_basket_d5.md"},
    {"sources_sha16": "ea70fccb41332a0b", "tiling": [4, 1],
     "valu_issue": 0.909, "mfma_busy": 0.0,
     "fp64_vector_flop_per_launch": 7.57e11, "fp64_matrix_flop_per_launch": 0.0,
     "profile": "profiles/path_kernel_d5_fp64_geo_basket_d5.md"},
    {"sources_sha16": "ea70fccb41332a0b", "tiling": [2, 2],
     "valu_issue": 0.909, "mfma_busy": 0.0,
     "fp64_vector_flop_per_launch": 7.49e11, "fp64_matrix_flop_per_launch": 0.0,
     "profile": "profiles/path_kernel_d5_fp64_geo_basket_d5.md"},
]
FETCH_FACTOR, WRITE_FACTOR = 2.0, 1.0
KERNEL_SOURCES = ("paper_1102_4666_amd/csrc/bsde_path.h",
                  "paper_1102_4666_amd/csrc/bsde_common.h",
                  "paper_1102_4666_amd/csrc/bsde_f64_math.h",
                  "paper_1102_4666_amd/csrc/bsde_inst_d5.hip")


def kernel_sources_sha16():
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def _measured_for(recs, tiling):
    """The profile record of these kernel sources at this tiling, or None."""
    if tiling is None:
        return None
    for rec in recs or ():
        if list(tiling) == list(rec["tiling"]) and \
                rec["sources_sha16"] == kernel_sources_sha16():
            return rec
    return None


def traffic_bytes(tiling):
    rec = _measured_for(TRAFFIC, tiling)
    if rec is None:
        return None
    return (rec["fetch_kib"] * FETCH_FACTOR + rec["write_kib"] * WRITE_FACTOR) * 1024


def counter_figures(tiling, path_ms):
    """The profile's counter-derived figures when the kernel and tiling are
    the profiled ones (the FLOP rates over this run's launch time)."""
    rec = _measured_for(COUNTERS, tiling)
    if rec is None:
        return None
    t = path_ms * 1e-3
    return {"valu_issue": rec["valu_issue"], "mfma_busy": rec["mfma_busy"],
            "fp64_vector_tflops_issued": rec["fp64_vector_flop_per_launch"] / t / 1e12,
            "fp64_vector_frac_issued": rec["fp64_vector_flop_per_launch"] / t /
            FP64_VECTOR_PEAK,
            "fp64_matrix_tflops_issued": rec["fp64_matrix_flop_per_launch"] / t / 1e12,
            "profile": rec["profile"]}


# ---------------------------------------------------------------------------
# Jobs
# ---------------------------------------------------------------------------
def headline_workload(precision="fp64"):
    import workloads
    return workloads.geo_basket_d5(omega=1.0, precision=precision)


HEADLINE_NAME = ("d=5 American geometric-basket put, penalised BSDE (penalty 1), "
                 "bump local vol with levels U[0.15,0.35], rho=0.2, 4096 random "
                 "spatial points x 10 times, eta=3 (p=84), M=1000, N=50, "
                 "10 Picard iterations")

# (groups per point, paths per lane) set on every job by --tiling, in place
# of the autotuned choice
FORCED_TILING = None


def steps_of(cfg, n):
    return n * cfg["M"] * cfg["N"] * cfg["K_it"]


def run_job(cfg, stream, phases=None):
    """One pricing job; phases (if a dict) accumulates the host wall time of
    create / solve / query / destroy in milliseconds."""
    import paper_1102_4666_amd as bsde
    t0 = time.perf_counter()
    P = bsde.Problem(cfg)
    if FORCED_TILING is not None:
        P.set_tiling(*FORCED_TILING)
    t1 = time.perf_counter()
    P.solve(stream)
    t2 = time.perf_counter()
    price, delta = P.price_delta()
    timings = P.timings()
    n = P.n
    t3 = time.perf_counter()
    P.close()
    t4 = time.perf_counter()
    if phases is not None:
        for key, dt in (("create", t1 - t0), ("solve", t2 - t1),
                        ("query", t3 - t2), ("destroy", t4 - t3)):
            phases[key] = phases.get(key, 0.0) + 1e3 * dt
    return price[0], delta[0], timings, n


def timed_jobs(cfg, steps, warmup, stream, tune=True):
    """Autotunes the path tiling of cfg's kernel signature once, runs warmup
    untimed jobs, then times `steps` jobs between device synchronisations."""
    import torch

    import paper_1102_4666_amd as bsde
    if FORCED_TILING is not None:
        tiling = FORCED_TILING
    elif tune:
        with bsde.Problem(cfg) as P:
            tiling = P.autotune(stream)[:2]
    else:
        tiling = None
    for _ in range(warmup):
        run_job(cfg, stream)
    torch.cuda.synchronize()
    lat, kern, phases = [], [], {}
    t0 = time.perf_counter()
    for _ in range(steps):
        ts = time.perf_counter()
        price, delta, tim, n = run_job(cfg, stream, phases)
        lat.append(time.perf_counter() - ts)
        kern.append(tim)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    kern = np.array(kern)
    return {"wall": wall, "lat": lat, "path_ms": float(np.mean(kern[:, 0])),
            "other_ms": float(np.mean(kern[:, 1])),
            "solve_ms": float(np.mean(kern[:, 4])),
            "phases": {k: v / steps for k, v in phases.items()},
            "tiling": list(tiling) if tiling is not None else None,
            "n": n, "price": price, "delta": delta}


def roofline(cfg, n, path_ms, tiling, precision):
    d = cfg["d"]
    C = 2 + d + d * (d + 1) // 2
    p, live = live_channel_entries(d, cfg["eta"], cfg.get("q", 1.0))
    fl, fl_mfma = flop_per_path_step(d, p, C, live, cfg["N"], cfg.get("vol_kind", "bump"),
                                     cfg.get("payoff", "put"))
    launch_steps = n * cfg["M"] * cfg["N"]
    t = path_ms * 1e-3
    achieved = fl * launch_steps / t
    peak = FP64_VECTOR_PEAK if precision == "fp64" else FP32_VECTOR_PEAK
    return {"bound": "alu", "achieved": achieved / 1e12, "peak": peak / 1e12,
            "unit": "TFLOP/s", "frac": achieved / peak,
            "traffic": traffic_bytes(tiling) if precision == "fp64" else None,
            "kernel": "path_kernel<d=%d, eta=%d, %s>" % (
                d, cfg["eta"], "double" if precision == "fp64" else "float"),
            "launch_ms": path_ms, "path_steps_per_launch": launch_steps,
            "flop_per_path_step": fl,
            "of_which_contraction_flop_per_path_step": fl_mfma,
            "channel_table_entries": {"live": live, "dense": p * C},
            "target_frac": 0.5,
            "counters": counter_figures(tiling, path_ms) if precision == "fp64" else None}


def gate(precision, price, delta, ref_p, ref_d, K, omega):
    tp, td = GATE[precision]
    dp = abs(price - ref_p)
    dd = float(np.max(np.abs(np.asarray(delta) - np.asarray(ref_d))))
    out = {"abs_price_err_over_K": dp / K, "max_abs_delta_err": dd,
           "gate_price_over_K": tp, "gate_delta": td,
           "gate_pass": bool(dp <= tp * K and dd <= td)}
    if omega >= 100:
        out["label"] = "Picard not converged"
        out["price_err_over_max_K_price"] = dp / max(K, abs(ref_p))
    return out


def _golden(name):
    path = os.path.join(ROOT, "tests", "golden", name + ".json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        return json.load(f)


ACCURACY_CASES = ("eur_put_d1", "amer_put_d1_w1", "amer_put_d1_w100",
                  "amer_basket_d2_w1", "amer_basket_d2_w100",
                  "geo_basket_d5_w1", "geo_basket_d5_w100",
                  "geo_basket_d5_redraw_w1")


def accuracy_gate(stream):
    """Every benchmark workload in both precisions against the stored FP64
    oracle results of the same streams."""
    out = {}
    for name in ACCURACY_CASES:
        g = _golden(name)
        if g is None:
            continue
        for prec in ("fp64", "fp32"):
            cfg = dict(g["cfg"], precision=prec)
            price, delta, _, _ = run_job(cfg, stream)
            r = gate(prec, price, delta, g["price"][-1], g["delta"][-1],
                     cfg["K"], cfg["omega"])
            r.update(price=price, oracle_price=g["price"][-1])
            out["%s/%s" % (name, prec)] = r
    return out


def batched_vs_fp64(stream, reps=2):
    """The batched FP32-path form against the plain FP64 per-problem form on
    the same GPU at penalty 1, where both must pass the accuracy gate: the
    d = 1, 2 and 5 workloads and the d = 10 request shape of the serving mix
    solved in one bsde_solve_batch call (one persistent path launch per
    Picard step and signature, the signatures as parallel branches, the
    schedule captured as a hipGraph), against the same four solved one after
    the other by bsde_solve in FP64.  The d <= 5 results are gated against
    the stored oracle results; the d = 10 shape (too large for the oracle as
    a whole) against the FP64 per-problem result, whose per-point parity
    with the oracle tests/test_gpu_d10.py checks."""
    import torch

    import paper_1102_4666_amd as bsde
    import workloads
    names = ("amer_put_d1", "amer_basket_d2", "geo_basket_d5", "put_basket_d10")
    gold = {nm: _golden(nm + "_w1") for nm in names[:3]}

    def run(prec, batched):
        probs = [bsde.Problem(getattr(workloads, nm)(omega=1.0, precision=prec))
                 for nm in names]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        if batched:
            bsde.solve_batch(probs, stream, graph=True)
        else:
            for P in probs:
                P.solve(stream)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        steps = sum(P.n * P.cfg["M"] * P.cfg["N"] * P.cfg["K_it"] for P in probs)
        res = {}
        for nm, P in zip(names, probs):
            price, delta = P.price_delta()
            res[nm] = (price[0], delta[0], P.cfg["K"])
            P.close()
        return dt, steps, res

    out, results = {}, {}
    for prec, batched, key in (("fp32", True, "batched_fp32_paths"),
                               ("fp64", False, "per_problem_fp64")):
        run(prec, batched)  # warm-up (kernel load, tuning table)
        best = None
        for _ in range(reps):
            dt, steps, res = run(prec, batched)
            best = dt if best is None else min(best, dt)
        results[prec] = res
        out[key] = {"seconds": best, "path_steps": steps,
                    "path_steps_per_s": steps / best}
    for prec, key in (("fp32", "batched_fp32_paths"), ("fp64", "per_problem_fp64")):
        err = {}
        for nm in names:
            price, delta, K = results[prec][nm]
            g = gold.get(nm)
            if g is not None:
                err[nm] = gate(prec, price, delta, g["price"][-1], g["delta"][-1], K, 1.0)
            elif prec == "fp32":
                p64, d64, _ = results["fp64"][nm]
                err[nm] = dict(gate("fp32", price, delta, p64, d64, K, 1.0),
                               reference="FP64 per-problem result")
        out[key]["accuracy"] = err
        out[key]["all_gates_pass"] = all(e["gate_pass"] for e in err.values())
    out["problems"] = ("d=1 (128x16 grid, M=4000), d=2 (32^2x16, M=2000), "
                       "d=5 (4096x10, M=1000), d=10 (8192x10, eta=3, M=500); "
                       "N=50, 10 or 8 Picard iterations, penalty 1")
    out["speedup"] = out["per_problem_fp64"]["seconds"] / \
        out["batched_fp32_paths"]["seconds"]
    return out


def d1_leg(steps, stream):
    """The d=1 American put workload (penalty 1) in FP32 paths: whole-job
    throughput and its path kernel's roofline, with the issue-cycle model."""
    import workloads
    cfg = workloads.amer_put_d1(omega=1.0, precision="fp32")
    r = timed_jobs(cfg, steps, 1, stream)
    launch_steps = r["n"] * cfg["M"] * cfg["N"]
    cyc = sum(ISSUE_CYCLES_D1_FP32.values()) * launch_steps / 64
    t = r["path_ms"] * 1e-3
    return {"workload": "d=1 American put, penalty 1, bump local vol, 128x16 "
                        "points, eta=4, M=4000, N=50, 8 Picard iterations",
            "dtype": "f32 paths, f64 sums",
            "path_steps_per_s": steps_of(cfg, r["n"]) * steps / r["wall"],
            "ms_per_job": 1e3 * r["wall"] / steps, "tiling": r["tiling"],
            "roofline": roofline(cfg, r["n"], r["path_ms"], r["tiling"], "fp32"),
            "issue_cycle_model": {
                "cycles_per_wave_path_step": sum(ISSUE_CYCLES_D1_FP32.values()),
                "achieved_T_cycles_per_s": cyc / t / 1e12,
                "peak_T_cycles_per_s": SIMD_ISSUE_CYCLES_PEAK / 1e12,
                "frac": cyc / t / SIMD_ISSUE_CYCLES_PEAK}}


# ---------------------------------------------------------------------------
# Serving
# ---------------------------------------------------------------------------
def serve(n_requests, n_sat, n_check, seed=0, dims=(1, 2, 5, 10)):
    """Closed-loop saturation (n_sat requests submitted at once), then
    Poisson arrivals at 0.5 and 0.9 of the saturation rate (n_requests each);
    p50/p99 latency and throughput per phase; then n_check sampled requests
    of the last phase solved alone and compared with their served results."""
    import torch

    import paper_1102_4666_amd as bsde
    import workloads

    free, _ = torch.cuda.mem_get_info()
    budget = int(0.9 * free)
    rng = np.random.default_rng(seed)

    def make(count, first):
        return [workloads.serving_request(first + i, rng, dims) for i in range(count)]

    def run_phase(reqs, rate, tag):
        with bsde.Server(budget, max_inflight=64) as S:
            t0 = time.perf_counter()
            arrivals = np.cumsum(rng.exponential(1.0 / rate, size=len(reqs))) \
                if rate else np.zeros(len(reqs))
            out = []
            for cfg, ta in zip(reqs, arrivals):
                now = time.perf_counter() - t0
                if ta > now:
                    time.sleep(ta - now)
                out.append(S.submit(cfg))
                if len(out) % 100 == 0:
                    print("serving %s: %d/%d submitted after %.1f s, %d completed" %
                          (tag, len(out), len(reqs), time.perf_counter() - t0,
                           S.stats()["completed"]), file=sys.stderr, flush=True)
            res = []
            for j, t in enumerate(out):
                res.append(S.poll(t))
                if (j + 1) % 25 == 0:
                    print("serving %s: %d/%d done after %.1f s" %
                          (tag, j + 1, len(out), time.perf_counter() - t0),
                          file=sys.stderr, flush=True)
            wall = time.perf_counter() - t0
            st = S.stats()
        lat = np.array([r["latency_ms"] for r in res])
        per_d = {}
        for cfg, r in zip(reqs, res):
            per_d.setdefault(cfg["d"], []).append(r["latency_ms"])
        return {"offered_rate": rate, "requests": len(reqs),
                "failed": sum(r["status"] != 0 for r in res),
                "wall_s": wall, "requests_per_s": st["requests_per_s"],
                "path_steps_per_s": st["path_steps_per_s"],
                "p50_ms": float(np.percentile(lat, 50)),
                "p99_ms": float(np.percentile(lat, 99)),
                "p99_sample_note": "p99 of %d requests" % len(reqs),
                "latency_ms_by_d": {
                    "d=%d" % d: {"n": len(v), "p50": float(np.percentile(v, 50)),
                                 "max": float(np.max(v))}
                    for d, v in sorted(per_d.items())},
                "engine_steps": st["engine_steps"]}, res

    print("serving: saturation phase (%d requests)" % n_sat, file=sys.stderr, flush=True)
    sat, _ = run_phase(make(n_sat, 0), None, "saturation")
    x_sat = sat["requests_per_s"]
    print("serving: %.2f requests/s at saturation" % x_sat, file=sys.stderr, flush=True)
    r05, _ = run_phase(make(n_requests, 10000), 0.5 * x_sat, "0.5 load")
    reqs09 = make(n_requests, 20000)
    r09, res09 = run_phase(reqs09, 0.9 * x_sat, "0.9 load")
    # alone versus mix: sampled requests of the 0.9-load phase solved alone
    pick = np.random.default_rng(seed + 1).choice(len(reqs09), min(n_check, len(reqs09)),
                                                  replace=False)
    same = 0
    worst = 0.0
    for j in pick:
        cfg = reqs09[j]
        with bsde.Problem(cfg) as P:
            P.solve()
            pr, de = P.price_delta()
        served = res09[j]
        dmax = float(np.max(np.abs(de[0] - served["delta"][:cfg["d"]])))
        worst = max(worst, abs(pr[0] - served["price"]), dmax)
        same += int(pr[0] == served["price"] and dmax == 0.0)
    print("serving: alone-vs-mix on %d requests: %d bitwise equal" % (len(pick), same),
          file=sys.stderr, flush=True)
    return {"mix": "d in %s, K U[80,120], European/American (penalty 0/1) 50/50, "
                   "M in {500,1000,2000,4000} (d=10: 8192x10 random points, eta=3, "
                   "M=500), N=50, FP32 paths" % (list(dims),),
            "hbm_budget_bytes": budget, "saturation": sat,
            "load_0.5": r05, "load_0.9": r09,
            "alone_vs_mix": {"checked": len(pick), "bitwise_equal": same,
                             "max_abs_difference": worst}}


# ---------------------------------------------------------------------------
# CPU baseline: the oracle as it stands
# ---------------------------------------------------------------------------
def _cpu_chunk(args):
    import oracle
    cfg, alpha, a, b = args
    t = time.perf_counter()
    oracle.corrections(cfg, alpha, 1, a, b)
    return time.perf_counter() - t


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for ln in f:
                if ln.startswith("model name"):
                    return ln.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(cfg, seconds=10.0, max_procs=16):
    """The oracle on a bounded sample of the headline job: the per-point
    corrections of one Picard iteration with non-zero coefficients (the
    least-squares fit of the payoff at the points, so u^k, its time
    derivative, gradient and Hessian are evaluated on every path) for the
    first points of the grid.  One core, then one process per usable core
    (at most max_procs) over disjoint point ranges, the paper's own
    parallel axis."""
    import multiprocessing as mp

    import oracle
    n, p = oracle.sizes(cfg)
    pts = oracle.points(cfg)
    y = np.array([oracle.payoff(cfg, pts[i, 1:]) for i in range(n)])
    alpha = oracle.fit(cfg, y)
    t1 = _cpu_chunk((cfg, alpha, 0, 2)) / 2
    n1 = int(max(1, min(n, seconds / max(t1, 1e-6))))
    dt1 = _cpu_chunk((cfg, alpha, 0, n1))
    single = n1 * cfg["M"] * cfg["N"] / dt1
    cores = max(1, min(max_procs, len(os.sched_getaffinity(0))))
    per = n1
    ranges = [(cfg, alpha, (c * per) % n, min(n, (c * per) % n + per)) for c in range(cores)]
    ctx = mp.get_context("fork")
    with ctx.Pool(cores) as pool:
        t = time.perf_counter()
        pool.map(_cpu_chunk, ranges)
        wall = time.perf_counter() - t
    pts_done = sum(b - a for _, _, a, b in ranges)
    allc = pts_done * cfg["M"] * cfg["N"] / wall
    return {"value": allc, "unit": "path-steps/s", "cores": cores, "kind": "oracle",
            "sample": "iteration-1 corrections (coefficients of a least-squares "
                      "fit of the payoff) of %d points per process, M=%d, N=%d, "
                      "of the %d-point headline grid; %d processes over disjoint "
                      "point ranges, %.3g path-steps in %.1f s"
                      % (per, cfg["M"], cfg["N"], n, cores,
                         pts_done * cfg["M"] * cfg["N"], wall),
            "single_core": {"value": single, "unit": "path-steps/s",
                            "sample": "%d points in %.1f s" % (n1, dt1)},
            "host_cpu": cpu_model(), "nproc": os.cpu_count(),
            "usable_cores": len(os.sched_getaffinity(0))}


# ---------------------------------------------------------------------------
def _overrides(text):
    """'k=v,k=v' -> dict, values as int, float or string."""
    out = {}
    for item in filter(None, text.split(",")):
        k, v = item.split("=", 1)
        for conv in (int, float):
            try:
                out[k] = conv(v)
                break
            except ValueError:
                pass
        else:
            out[k] = v
    return out


def single_launches(names, euler_steps=None, precision="fp32", overrides=None):
    """One Picard iteration (one path-kernel launch) of each named workload:
    the runs behind the profiles.  Names: amer_put_d1, amer_basket_d2,
    geo_basket_d5, eur_put_d1_kernel (the kernel operator of Section 3.2),
    d10-serving (the d=10 request shape of the serving mix at M=500),
    call_basket_d10_hyperbolic (the hyperbolic-set kernel, p=221).
    euler_steps replaces N (separates per-step from per-path cost);
    overrides (a dict) replaces workload fields (eta, q, vol_kind, ...)."""
    import paper_1102_4666_amd as bsde
    import workloads
    out = {}
    for nm in names:
        if nm == "d10-serving":
            cfg = workloads.serving_request(1, np.random.default_rng(0), dims=(10,))
            cfg.update(M=500, K=100.0, omega=1.0, precision=precision)
        else:
            cfg = getattr(workloads, nm)(precision=precision)
        cfg.update(K_it=1)
        cfg.update(overrides or {})
        if euler_steps:
            cfg.update(N=euler_steps)
        with bsde.Problem(cfg) as P:
            if FORCED_TILING is not None:
                P.set_tiling(*FORCED_TILING)
            P.solve()
            out[nm] = {"path_kernel_ms": P.timings()[0],
                       "path_steps": P.n * cfg["M"] * cfg["N"]}
            if cfg.get("kernel_bw", 0.0) > 0.0:
                out[nm]["kernel_pairs"] = P.n * cfg["M"] * P.n
    return out


# The paper's d = 10 benchmark (Section 6.2.1): European call basket,
# Black-Scholes sigma = 0.2, rho = 0.2, K = S0 = 100, T = 1, r = 0.05,
# n = 1000 points redrawn every iteration, M = 30,000, N = 10, 10 Picard
# iterations; benchmark price 7.0207, CI (7.0125, 7.0288).
D10_BENCHMARK = 7.0207
# (eta, q, M): total degree 2 and 3, the hyperbolic sets eta = 5 with
# q = 0.5, 0.6, 0.7, and the paper's other two curves of Section 6.2.1,
# eta = 4, q = 0.6 and eta = 5, q = 0.6 at M = 5000
D10_SETS = ((2, 1.0, 30000), (3, 1.0, 30000), (4, 0.6, 30000), (5, 0.5, 30000),
            (5, 0.6, 30000), (5, 0.6, 5000), (5, 0.7, 30000))


def d10_sparsity_study(seeds=8):
    """Bias against sparsity of the index set: the paper's d = 10 call
    basket on the total-degree sets eta = 2, 3, the hyperbolic sets eta = 4,
    q = 0.6 and eta = 5, q = 0.5, 0.6, 0.7 (and q = 0.6 at M = 5000), each
    over `seeds` seeds; mean, seed spread and the difference from the
    benchmark price."""
    import paper_1102_4666_amd as bsde
    import workloads
    out = []
    for eta, q, M in D10_SETS:
        cfg = workloads.call_basket_d10_hyperbolic()
        cfg.update(eta=eta, q=q, M=M)
        prices, ms = [], []
        p = None
        for seed in range(seeds):
            t = time.perf_counter()
            with bsde.Problem(dict(cfg, seed=seed)) as P:
                P.solve()
                prices.append(float(P.price_delta()[0][0]))
                p = P.p if q == 1.0 else None
            ms.append(1e3 * (time.perf_counter() - t))
        if p is None:
            p = len(index_set(10, eta, q))
        m, sd = float(np.mean(prices)), float(np.std(prices, ddof=1))
        out.append({"eta": eta, "q": q, "M": M, "p": p, "mean_price": m, "seed_std": sd,
                    "std_of_mean": sd / np.sqrt(seeds), "bias": m - D10_BENCHMARK,
                    "ms_per_solve": float(np.mean(ms))})
        print("d=10 eta=%d q=%g M=%d p=%d: %.4f +- %.4f" % (eta, q, M, p, m, sd),
              file=sys.stderr, flush=True)
    return {"workload": "d=10 European call basket (Section 6.2.1), n=1000 uniform "
                        "points redrawn every iteration, domain +-1 sd, M=30000 "
                        "unless stated, N=10, 10 Picard iterations, FP32 paths",
            "benchmark": D10_BENCHMARK, "seeds": seeds, "sets": out}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--precision", default="fp64", choices=["fp32", "fp64"],
                    help="precision of the headline job (default fp64)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=10.0)
    ap.add_argument("--no-accuracy", action="store_true",
                    help="skip the gate check against stored oracle results")
    ap.add_argument("--serve", type=int, default=200, metavar="R",
                    help="requests per load level of the request-server "
                         "benchmark (0 = skip it)")
    ap.add_argument("--serve-sat", type=int, default=100, metavar="R",
                    help="requests of the closed-loop saturation phase")
    ap.add_argument("--serve-check", type=int, default=50, metavar="R",
                    help="served requests re-solved alone for the "
                         "alone-versus-mix check")
    ap.add_argument("--no-batched", action="store_true",
                    help="skip the batched-FP32 vs per-problem-FP64 comparison")
    ap.add_argument("--no-extra", action="store_true",
                    help="skip the FP32-path and d=1 legs")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 1 GiB device copy (calibrates the "
                         "HBM byte counters of the profiler)")
    ap.add_argument("--euler-steps", type=int, default=0, metavar="N",
                    help="with --single-launch: Euler steps per path "
                         "instead of the workload's")
    ap.add_argument("--set", default="", metavar="K=V,..",
                    help="with --single-launch: replace workload fields, e.g. "
                         "eta=2,q=1.0,vol_kind=const")
    ap.add_argument("--tiling", default="", metavar="G,P",
                    help="run every job at G workgroups per point and P paths "
                         "per lane instead of the autotuned tiling")
    ap.add_argument("--single-launch", default="", metavar="NAMES",
                    help="comma-separated workloads (amer_put_d1, amer_basket_d2, "
                         "geo_basket_d5, eur_put_d1_kernel, d10-serving, "
                         "call_basket_d10_hyperbolic): run one path-kernel "
                         "launch of each and print its time, nothing else")
    ap.add_argument("--study", default="", choices=["", "d10-sparsity"],
                    help="run a study instead of the benchmark: d10-sparsity = "
                         "price of the paper's d=10 call basket against the "
                         "index set (total degree 2, 3; hyperbolic eta=5, "
                         "q=0.5, 0.6, 0.7)")
    args = ap.parse_args()
    global FORCED_TILING
    if args.tiling:
        FORCED_TILING = tuple(int(v) for v in args.tiling.split(","))
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on exactly one GPU: the solver has no multi-GPU "
              "path (one problem's points would shard across GPUs with a "
              "p-vector all-reduce per iteration; not built)", file=sys.stderr)
        sys.exit(2)

    # the oracle's processes are forked before anything initialises the GPU
    cpu = None
    if not (args.no_cpu_baseline or args.copy_calibration or args.single_launch
            or args.study):
        print("cpu baseline", file=sys.stderr, flush=True)
        cpu = cpu_baseline(headline_workload("fp64"), args.cpu_seconds)

    import torch
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    if args.copy_calibration:
        src = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": src.numel() * 4,
                          "copy_bytes_written": dst.numel() * 4, "copies": 3}))
        return
    if args.study == "d10-sparsity":
        print(json.dumps(d10_sparsity_study()))
        return
    if args.single_launch:
        print(json.dumps(single_launches(args.single_launch.split(","),
                                         args.euler_steps or None, args.precision,
                                         _overrides(args.set))))
        return
    stream = torch.cuda.current_stream().cuda_stream

    print("headline: %d warm-up and %d timed jobs" % (args.warmup, args.steps),
          file=sys.stderr, flush=True)
    cfg = headline_workload(args.precision)
    r = timed_jobs(cfg, args.steps, args.warmup, stream)
    per_job = steps_of(cfg, r["n"])
    g = _golden("geo_basket_d5_w1")
    line = {
        "metric": METRIC,
        "value": per_job * args.steps / r["wall"],
        "unit": "path-steps/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": 1e3 * r["wall"] / args.steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64" if args.precision == "fp64" else "f32 paths, f64 sums",
        "data": "synthetic",
        "config": {"workload": HEADLINE_NAME, "path_steps_per_job": per_job,
                   "precision": args.precision},
        "requests_per_s": args.steps / r["wall"],
        "latency_ms": {"p50": 1e3 * float(np.percentile(r["lat"], 50)),
                       "p99": 1e3 * float(np.percentile(r["lat"], 99))},
        "path_kernel_ms": r["path_ms"], "tiling": r["tiling"],
        "job_phase_ms": r["phases"],
        "kernel_ms_per_iteration": {"path": r["path_ms"],
                                    "reduce_project_update": r["other_ms"]},
        "solve_ms": r["solve_ms"],
        "roofline": roofline(cfg, r["n"], r["path_ms"], r["tiling"], args.precision),
    }
    if g is not None:
        line["headline_accuracy"] = gate(args.precision, r["price"], r["delta"],
                                         g["price"][-1], g["delta"][-1], cfg["K"], 1.0)
    print("headline: %.4g path-steps/s" % line["value"], file=sys.stderr, flush=True)
    if not args.no_extra:
        other = "fp32" if args.precision == "fp64" else "fp64"
        c2 = headline_workload(other)
        r2 = timed_jobs(c2, args.steps, 1, stream)
        leg = {"dtype": "f32 paths, f64 sums" if other == "fp32" else "f64",
               "path_steps_per_s": steps_of(c2, r2["n"]) * args.steps / r2["wall"],
               "ms_per_job": 1e3 * r2["wall"] / args.steps, "tiling": r2["tiling"],
               "roofline": roofline(c2, r2["n"], r2["path_ms"], r2["tiling"], other)}
        if g is not None:
            leg["accuracy"] = gate(other, r2["price"], r2["delta"], g["price"][-1],
                                   g["delta"][-1], c2["K"], 1.0)
        line["fp32_paths" if other == "fp32" else "fp64_paths"] = leg
        line["d1_amer_put"] = d1_leg(max(5, args.steps), stream)
        print("extra legs done", file=sys.stderr, flush=True)
    if not args.no_accuracy:
        line["accuracy_gate"] = accuracy_gate(stream)
        print("accuracy gate done", file=sys.stderr, flush=True)
    if not args.no_batched:
        line["batched_vs_fp64_per_problem"] = batched_vs_fp64(stream)
        print("batched comparison done", file=sys.stderr, flush=True)
    if args.serve:
        line["serving"] = serve(args.serve, args.serve_sat, args.serve_check)
    if cpu is not None:
        line["cpu_baseline"] = cpu
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
