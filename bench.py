"""Benchmark of the BSDE solver library on one MI355X.

A step is one whole pricing job of the d=1 American put workload (local
volatility 0.2 (1 + 0.25 exp(-(log(S/100))^2)), penalty 100, 128 space x 16
time points, M=4000 paths, N=50 Euler steps, 8 Picard iterations):
problem set-up (grid, basis, least-squares factorisation, upload), all
Picard iterations on the GPU (path simulation, driver, reductions,
least-squares update), the price/delta query, and tear-down.

Prints one JSON line: Euler path-steps per second of whole jobs, the
roofline of the dominant kernel (the Monte Carlo path kernel, bound by
vector-ALU issue), per-job latency percentiles, the error of the result
against the FP64 oracle on the same random streams, and the oracle timed on
a bounded sample of the same workload on the host CPU.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--precision fp32|fp64]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# MI355X (gfx950): 256 CUs x 4 SIMDs at 2.4 GHz.  The path kernel is bound
# by vector-ALU issue; its roofline counts shader cycles of issue per SIMD:
# peak = 1024 SIMDs x 2.4e9 cycles/s.
SIMD_ISSUE_CYCLES_PEAK = 256 * 4 * 2.4e9
FP32_VECTOR_PEAK = 157.3e12                     # FLOP/s (packed FMA)
FP64_VECTOR_PEAK = 78.6e12
# HBM traffic of one path-kernel launch of the benchmark workload, from
# rocprofv3 FETCH_SIZE and WRITE_SIZE (separate runs, KiB per dispatch) by
# tiling (workgroups per point), scaled by the plain-copy calibration
# factors (x2.0 and x1.0).  The autotuner picks the tiling at run time;
# a tiling missing here reports null.
TRAFFIC_KIB = {"fp32": {1: (177, 64), 2: (305, 128), 4: (305, 256),
                        8: (305, 512), 16: (305, 1024)},
               "fp64": {1: (268, 64), 2: (396, 128), 4: (396, 256),
                        8: (396, 512), 16: (398, 1024)}}
FETCH_FACTOR, WRITE_FACTOR = 2.0, 1.0


def traffic_bytes(precision, groups):
    fw = TRAFFIC_KIB.get(precision, {}).get(groups)
    if fw is None:
        return None
    return (fw[0] * FETCH_FACTOR + fw[1] * WRITE_FACTOR) * 1024


# Algorithmic issue cycles per Euler path-step of one wave (64 paths) for
# the d = 1 local-volatility workload (N = 50 steps per path), derived
# operation by operation in the design doc section 6.  Issue cost per wave64
# instruction on gfx950, measured by paper_1102_4666_amd/probe/issue_rates.hip
# (profiles/valu_issue_rates_gfx950.md): 32-bit adds, multiplies, fused
# multiply-adds and logic operations (v_bitop3_b32 included) whose operands
# are all vector registers 2 cycles at best (2.1-3.3 measured), the same
# with a scalar or literal operand 4, 64-bit multiply-adds, 32-bit integer
# multiplies, conversions and funnel shifts 4, transcendentals 8 (they do
# not issue beside other vector instructions).  Each operation is priced at
# the cheapest form that computes it, so the bound is an optimistic one.
ISSUE_CYCLES_PER_WAVE_STEP = {
    "fp32": {
        # 1/4 Philox4x32-10 block (the work on the uniform counter words and
        # on m alone done once per path or on the scalar unit): 16
        # v_mad_u64_u32 (4), two XORs and one three-input XOR with a uniform
        # operand (4), 15 three-input XORs (2): 106
        "normal_philox": (16 * 4 + 3 * 4 + 15 * 2) / 4,
        # 1/2 Box-Muller pair: conversion, funnel shift (4); log, sqrt, sin,
        # cos (8); fused multiply-add and three multiplies (2)
        "normal_box_muller": (2 * 4 + 4 * 8 + 4 * 2) / 2,
        # volatility: y*y (2), exp (8), fused multiply-add (2)
        "local_vol": 2 + 8 + 2,
        # Euler update: two fused multiply-adds and an add (2)
        "euler": 3 * 2,
        # the compare that selects step j* (2)
        "record": 2,
        # per path over N = 50: U and bridge blocks (2 x 106), one Box-Muller
        # pair (48), 156 other operations at 2 (j*, theta, tau, X_tau, two
        # Chebyshev rows, the 15 x 4 contraction and u(T), driver and
        # generator, FP64 sums)
        "per_path": (2 * 106 + 48 + 156 * 2) / 50.0,
    },
    # FP64 paths use software transcendentals with no independent operation
    # count: the measured instructions per path-step, SQ_INSTS_VALU minus
    # SQ_INSTS_VALU_TRANS_F64 (162.7 - 1.1) at 4 cycles and 1.1 at 8
    "fp64": {"measured": 161.6 * 4 + 1.1 * 8},
}
FP32_FLOP_PER_PATH_STEP = 4.5 + 4 + 6 + 250 / 50.0


def workload(precision: str, omega: float = 100.0):
    import workloads
    return workloads.amer_put_d1(omega=omega, precision=precision)


# (groups per point, paths per lane) set on every job by --tiling, in place
# of the autotuned choice
FORCED_TILING = None


def run_job(cfg, stream, phases=None, solve_lock=None):
    """One pricing job; phases (if a dict) accumulates the host wall time
    of create / solve / query / destroy in milliseconds.  With solve_lock,
    the solve holds it (jobs of other threads create and query meanwhile)."""
    import paper_1102_4666_amd as bsde
    t0 = time.perf_counter()
    P = bsde.Problem(cfg)
    if FORCED_TILING is not None:
        P.set_tiling(*FORCED_TILING)
    if solve_lock is not None:
        solve_lock.acquire()
    t1 = time.perf_counter()
    try:
        P.solve(stream)
    finally:
        if solve_lock is not None:
            solve_lock.release()
    t2 = time.perf_counter()
    price, delta = P.price_delta()
    timings = P.timings()
    t3 = time.perf_counter()
    P.close()
    t4 = time.perf_counter()
    if phases is not None:
        for key, dt in (("create", t1 - t0), ("solve", t2 - t1),
                        ("query", t3 - t2), ("destroy", t4 - t3)):
            phases[key] = phases.get(key, 0.0) + 1e3 * dt
    return price[0], delta[0], timings


def run_jobs(cfg, n_jobs, streams):
    """n_jobs pricing jobs of cfg over len(streams) host threads, one HIP
    stream each: job j runs on thread j % depth.  The solves (the Picard
    iterations) take a lock, so that path kernels of two jobs never share
    the GPU; the set-up of a job (host work and its small device kernels)
    and the query and release of the previous one overlap the solve of
    another.  Returns per-job latencies (s), path-kernel ms, timings and the
    summed phase times."""
    import threading
    depth = len(streams)
    lat, path_ms, kern_ms = [0.0] * n_jobs, [0.0] * n_jobs, [None] * n_jobs
    phases = [dict() for _ in range(depth)]
    errors = []
    lock = threading.Lock() if depth > 1 else None

    def worker(w):
        try:
            for j in range(w, n_jobs, depth):
                ts = time.perf_counter()
                _, _, tim = run_job(cfg, streams[w], phases[w], lock)
                lat[j] = time.perf_counter() - ts
                path_ms[j] = tim[0]
                kern_ms[j] = tim
        except Exception as e:  # reported by the caller
            errors.append(e)

    threads = [threading.Thread(target=worker, args=(w,)) for w in range(depth)]
    for t in threads:
        t.start()
    for t in threads:
        t.join()
    if errors:
        raise errors[0]
    merged = {}
    for ph in phases:
        for k, v in ph.items():
            merged[k] = merged.get(k, 0.0) + v
    return lat, path_ms, kern_ms, merged


def accuracy(precision: str, stream):
    """Error against the stored FP64 oracle results of the same workload."""
    out = {}
    for omega in (100.0, 1.0):
        name = "amer_put_d1_w100" if omega == 100.0 else "amer_put_d1_w1"
        path = os.path.join(ROOT, "tests", "golden", name + ".json")
        if not os.path.exists(path):
            continue
        with open(path) as f:
            g = json.load(f)
        price, delta, _ = run_job(workload(precision, omega), stream)
        ref_p, ref_d = g["price"][-1], g["delta"][-1][0]
        out["omega=%g" % omega] = {
            "price": price, "oracle_price": ref_p,
            "abs_price_err_over_K": abs(price - ref_p) / 100.0,
            "rel_price_err": abs(price - ref_p) / max(1.0, abs(ref_p)),
            "delta": float(delta[0]), "oracle_delta": ref_d,
            "abs_delta_err": abs(float(delta[0]) - ref_d),
        }
    return out


def batched_vs_fp64(stream, reps: int = 2):
    """The batched FP32-path form against the plain FP64 per-problem form on
    the same GPU: three problems (the d = 1, 2 and 5 workloads, penalty
    100) solved in one bsde_solve_batch call (one persistent path launch per
    Picard step, the schedule captured as a hipGraph), against the same
    three solved one after the other by bsde_solve in FP64.  Both are
    checked against the stored FP64 oracle results of the same streams."""
    import torch

    import paper_1102_4666_amd as bsde
    import workloads
    names = ("amer_put_d1", "amer_basket_d2", "geo_basket_d5")
    gold = {}
    for nm in names:
        path = os.path.join(ROOT, "tests", "golden", nm + "_w100.json")
        if os.path.exists(path):
            with open(path) as f:
                g = json.load(f)
            gold[nm] = (g["price"][-1], g["delta"][-1])

    def run(prec, batched):
        probs = [bsde.Problem(getattr(workloads, nm)(precision=prec))
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
        steps = sum(P.n * P.cfg["M"] * P.cfg["N"] * P.cfg["K_it"]
                    for P in probs)
        err = {}
        for nm, P in zip(names, probs):
            price, delta = P.price_delta()
            if nm in gold:
                ref_p, ref_d = gold[nm]
                # prices of the penalised problem at penalty 100 are far
                # from K (the iteration diverges); errors relative to the
                # oracle's own price
                err[nm] = {"rel_price_err": abs(price[0] - ref_p) / max(1.0, abs(ref_p)),
                           "max_rel_delta_err": float(np.max(
                               np.abs(delta[0] - np.asarray(ref_d)) /
                               np.maximum(1.0, np.abs(ref_d))))}
            P.close()
        return dt, steps, err

    out = {}
    for prec, batched, key in (("fp32", True, "batched_fp32_paths"),
                               ("fp64", False, "per_problem_fp64")):
        run(prec, batched)  # warm-up (kernel load, tuning table)
        best = None
        for _ in range(reps):
            dt, steps, err = run(prec, batched)
            best = dt if best is None else min(best, dt)
        out[key] = {"seconds": best, "path_steps": steps,
                    "path_steps_per_s": steps / best, "error_vs_oracle": err}
    out["problems"] = "d=1 (128x16 grid, M=4000), d=2 (32^2x16, M=2000), " \
                      "d=5 (4096x10, M=1000); N=50, penalty 100"
    out["speedup"] = out["per_problem_fp64"]["seconds"] / \
        out["batched_fp32_paths"]["seconds"]
    return out


def cpu_baseline(cfg, seconds: float = 12.0):
    """The oracle on a bounded sample: per-point corrections of iteration 1
    (coefficients present, so u^k and its derivatives are evaluated on every
    path) for the first points of the grid, single thread."""
    import oracle
    n, p = oracle.sizes(cfg)
    alpha = np.zeros(p)
    t = time.perf_counter()
    oracle.corrections(cfg, alpha, 1, 0, 1)
    per_point = time.perf_counter() - t
    n_sub = int(max(1, min(n, seconds / max(per_point, 1e-6))))
    t = time.perf_counter()
    oracle.corrections(cfg, alpha, 1, 0, n_sub)
    dt = time.perf_counter() - t
    steps = n_sub * cfg["M"] * cfg["N"]
    return {"value": steps / dt, "unit": "path-steps/s", "cores": 1,
            "kind": "oracle",
            "sample": "iteration-1 corrections of the first %d of %d points "
                      "(M=%d, N=%d): %.3g path-steps in %.1f s" %
                      (n_sub, n, cfg["M"], cfg["N"], steps, dt)}


def serve(n_requests: int, seed: int = 0, dims=(1, 2, 5, 10)):
    """Serving run: closed-loop saturation, then Poisson arrivals at 0.5 and
    0.9 of the saturation rate; p50/p99 latency and throughput per phase."""
    import torch

    import paper_1102_4666_amd as bsde
    import workloads

    free, _ = torch.cuda.mem_get_info()
    budget = int(0.9 * free)
    rng = np.random.default_rng(seed)
    reqs = [workloads.serving_request(i, rng, dims) for i in range(n_requests)]

    def run_phase(rate):
        lat = []
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
            res = []
            for j, t in enumerate(out):
                res.append(S.poll(t))
                if (j + 1) % 10 == 0:
                    print("serving: %d/%d done after %.1f s" %
                          (j + 1, len(out), time.perf_counter() - t0),
                          file=sys.stderr, flush=True)
            wall = time.perf_counter() - t0
            st = S.stats()
        bad = [r["status"] for r in res if r["status"] != 0]
        per_d = {}
        for cfg, r in zip(reqs, res):
            per_d.setdefault(cfg["d"], []).append(r["latency_ms"])
        return {"offered_rate": rate, "requests": len(reqs), "failed": len(bad),
                "wall_s": wall, "requests_per_s": st["requests_per_s"],
                "path_steps_per_s": st["path_steps_per_s"],
                "p50_ms": st["p50_ms"], "p99_ms": st["p99_ms"],
                "latency_ms_by_d": {
                    "d=%d" % d: {"n": len(v),
                                 "p50": float(np.percentile(v, 50)),
                                 "max": float(np.max(v))}
                    for d, v in sorted(per_d.items())},
                "engine_steps": st["engine_steps"]}

    print("serving: saturation phase", file=sys.stderr, flush=True)
    sat = run_phase(None)
    print("serving: %.2f requests/s at saturation" % sat["requests_per_s"],
          file=sys.stderr, flush=True)
    x_sat = sat["requests_per_s"]
    return {"mix": "d in %s, K U[80,120], European/American 50/50, M in "
                   "{500,1000,2000,4000} (d=10: 8192x10 random points, "
                   "eta=3, every other request at M=500), FP32 paths"
                   % (list(dims),),
            "hbm_budget_bytes": budget, "saturation": sat,
            "load_0.5": run_phase(0.5 * x_sat),
            "load_0.9": run_phase(0.9 * x_sat)}


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
    """One Picard iteration (one path-kernel launch) of each named workload,
    FP32 paths, default tiling: the runs behind the profiles of the
    matrix-core kernels.  Names: amer_put_d1, amer_basket_d2, geo_basket_d5,
    eur_put_d1_kernel (the kernel operator of Section 3.2), d10-serving
    (the d=10 request shape of the serving mix at M=500),
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
                # the kernel operator weighs every (path, point) pair
                out[nm]["kernel_pairs"] = P.n * cfg["M"] * P.n
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--precision", default="fp32", choices=["fp32", "fp64"])
    ap.add_argument("--pipeline", type=int, default=1, metavar="DEPTH",
                    help="pricing jobs in flight (host threads): the set-up "
                         "of one overlaps the Picard iterations of another "
                         "(default 1: one job after the other)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--no-accuracy", action="store_true",
                    help="skip the error check against stored oracle results")
    ap.add_argument("--serve", type=int, default=24, metavar="R",
                    help="requests per load level of the request-server "
                         "benchmark (0 = skip it)")
    ap.add_argument("--no-batched", action="store_true",
                    help="skip the batched-FP32 vs per-problem-FP64 comparison")
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
                         "per lane instead of the autotuned tiling (for counter "
                         "runs that must see one tiling)")
    ap.add_argument("--single-launch", default="", metavar="NAMES",
                    help="comma-separated workloads (amer_put_d1, amer_basket_d2, "
                         "geo_basket_d5, eur_put_d1_kernel, d10-serving, "
                         "call_basket_d10_hyperbolic): run one "
                         "path-kernel launch of each and print its time, nothing "
                         "else")
    args = ap.parse_args()
    global FORCED_TILING
    if args.tiling:
        FORCED_TILING = tuple(int(v) for v in args.tiling.split(","))
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on exactly one GPU: the solver has no multi-GPU "
              "path (one problem's points would shard across GPUs with a "
              "p-vector all-reduce per iteration; not built)", file=sys.stderr)
        sys.exit(2)

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
                          "copy_bytes_written": dst.numel() * 4,
                          "copies": 3}))
        return
    if args.single_launch:
        print(json.dumps(single_launches(args.single_launch.split(","),
                                         args.euler_steps or None, args.precision,
                                         _overrides(args.set))))
        return
    if args.pipeline < 1:
        ap.error("--pipeline must be at least 1")
    stream = torch.cuda.current_stream().cuda_stream
    cfg = workload(args.precision)
    n = cfg["n_t"] * cfg["n_x"]
    steps_per_job = n * cfg["M"] * cfg["N"] * cfg["K_it"]

    # tune the path tiling of this kernel signature once; problems created
    # afterwards start with the recorded choice
    import paper_1102_4666_amd as bsde
    if FORCED_TILING is not None:
        tiling = FORCED_TILING
    else:
        with bsde.Problem(cfg) as P:
            tiling = P.autotune(stream)
    # job pipeline: one stream per host thread (default priority)
    streams = [stream] + [torch.cuda.Stream().cuda_stream
                          for _ in range(args.pipeline - 1)]
    run_jobs(cfg, args.warmup, streams)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    lat, path_ms, kern_ms, phases = run_jobs(cfg, args.steps, streams)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_per_step = 1e3 * wall / args.steps

    # roofline of the path kernel: algorithmic VALU slots per launch over
    # its mean duration (HIP events on the solve's stream)
    t_path = float(np.mean(path_ms)) * 1e-3
    launch_steps = n * cfg["M"] * cfg["N"]
    cyc = sum(ISSUE_CYCLES_PER_WAVE_STEP[args.precision].values()) * launch_steps / 64
    achieved = cyc / t_path
    line = {
        "metric": "Euler path-steps/s + priced requests/s (p50/p99) at stated price/delta error",
        "value": steps_per_job * args.steps / wall,
        "unit": "path-steps/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32 paths, f64 sums" if args.precision == "fp32" else "f64",
        "data": "synthetic",
        "config": {"workload": "d=1 American put, penalised BSDE (penalty 100), "
                               "bump local vol, 128x16 grid, M=4000, N=50, "
                               "8 Picard iterations, eta=4",
                   "path_steps_per_job": steps_per_job,
                   "jobs_in_flight": args.pipeline,
                   "precision": args.precision},
        "requests_per_s": args.steps / wall,
        "latency_ms": {"p50": 1e3 * float(np.percentile(lat, 50)),
                       "p99": 1e3 * float(np.percentile(lat, 99))},
        "path_kernel_ms": float(np.mean(path_ms)),
        "tiling": {"groups_per_point": tiling[0], "paths_per_lane": tiling[1]},
        "job_phase_ms": {k: v / args.steps for k, v in phases.items()},
        "kernel_ms_per_iteration": dict(zip(
            ["path", "reduce_project_update"],
            [float(x) for x in np.mean(kern_ms, axis=0)[:2]])),
        "solve_ms": float(np.mean(kern_ms, axis=0)[4]),
        "roofline": {"bound": "alu", "achieved": achieved / 1e12,
                     "peak": SIMD_ISSUE_CYCLES_PEAK / 1e12,
                     "unit": "T SIMD vector-issue cycles/s (algorithmic)",
                     "frac": achieved / SIMD_ISSUE_CYCLES_PEAK,
                     "traffic": traffic_bytes(args.precision, tiling[0])},
    }
    if args.precision == "fp32":
        fl = FP32_FLOP_PER_PATH_STEP * launch_steps / t_path
        line["fp32_vector_flops"] = {"achieved_tflops": fl / 1e12,
                                     "peak_tflops": FP32_VECTOR_PEAK / 1e12,
                                     "frac": fl / FP32_VECTOR_PEAK}
    if not args.no_accuracy:
        line["accuracy_vs_oracle"] = accuracy(args.precision, stream)
    if not args.no_batched:
        line["batched_vs_fp64_per_problem"] = batched_vs_fp64(stream)
    if args.serve:
        line["serving"] = serve(args.serve, dims=(1, 2, 5, 10))
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(workload("fp64"), args.cpu_seconds)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
