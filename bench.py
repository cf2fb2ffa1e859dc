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

# MI355X (gfx950): 256 CUs x 4 SIMDs x 16 lanes per cycle at 2.4 GHz.
VALU_PEAK_LANE_OPS = 256 * 4 * 16 * 2.4e9      # 3.93e13 full-rate lane-ops/s
FP32_VECTOR_PEAK = 157.3e12                     # FLOP/s (packed FMA)
FP64_VECTOR_PEAK = 78.6e12


def valu_ops_per_path_step(d: int, precision: str) -> float:
    """Algorithmic VALU issue slots per Euler path-step of the path kernel
    for the d=1 local-volatility workload, counted from the operations the
    method needs (quarter-rate transcendentals and 32-bit integer multiplies
    weigh 4 slots).  The derivation is written out in the design doc."""
    if d != 1:
        raise ValueError("op count stated for d = 1 only")
    if precision == "fp32":
        # per normal: 1/4 Philox4x32-10 block = 10 rounds x (4 mul x 4 + 4 xor) / 4
        philox = 10 * (4 * 4 + 4) / 4.0                 # 50
        box_muller = (2 + 2 + 4 * 4 + 3) / 2.0           # 11.5 (cvt, fma, log/sqrt/sin/cos, mul)
        vol = 4 + 4                                      # exp (quarter rate) + sub/mul/fma/mul
        euler = 2 + 4 + 3                                # drift, update, j* select
        per_path = 230                                   # U, bridge, basis, driver, sums
        return philox + box_muller + vol + euler + per_path / 50.0
    # FP64: transcendentals in software (log ~ 20, sincos ~ 40, exp ~ 20,
    # sqrt ~ 8 full-rate FP64 ops)
    philox = 10 * (4 * 4 + 4) / 4.0
    box_muller = (2 + 2 + 20 + 8 + 40 + 3) / 2.0
    vol = 20 + 4
    euler = 2 + 4 + 3
    per_path = 400
    return philox + box_muller + vol + euler + per_path / 50.0


def workload(precision: str, omega: float = 100.0):
    import workloads
    return workloads.config2(omega=omega, precision=precision)


def run_job(cfg, stream):
    import paper_1102_4666_amd as bsde
    P = bsde.Problem(cfg)
    P.solve(stream)
    price, delta = P.price_delta()
    timings = P.timings()
    P.close()
    return price[0], delta[0], timings


def accuracy(precision: str, stream):
    """Error against the stored FP64 oracle results of the same workload."""
    out = {}
    for omega in (100.0, 1.0):
        name = "config2_w100" if omega == 100.0 else "config2_w1"
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


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--precision", default="fp32", choices=["fp32", "fp64"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on exactly one GPU: the solver has no multi-GPU "
              "path (one problem's points would shard across GPUs with a "
              "p-vector all-reduce per iteration; not built)", file=sys.stderr)
        sys.exit(2)

    import torch
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream().cuda_stream
    cfg = workload(args.precision)
    n = cfg["n_t"] * cfg["n_x"]
    steps_per_job = n * cfg["M"] * cfg["N"] * cfg["K_it"]

    for _ in range(args.warmup):
        run_job(cfg, stream)
    torch.cuda.synchronize()
    lat = []
    path_ms = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        ts = time.perf_counter()
        _, _, tim = run_job(cfg, stream)
        lat.append(time.perf_counter() - ts)
        path_ms.append(tim[0])
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_per_step = 1e3 * wall / args.steps

    # roofline of the path kernel: algorithmic VALU slots per launch over
    # its mean duration (HIP events on the solve's stream)
    t_path = float(np.mean(path_ms)) * 1e-3
    ops = valu_ops_per_path_step(cfg["d"], args.precision) * n * cfg["M"] * cfg["N"]
    achieved = ops / t_path
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
                   "precision": args.precision},
        "requests_per_s": args.steps / wall,
        "latency_ms": {"p50": 1e3 * float(np.percentile(lat, 50)),
                       "p99": 1e3 * float(np.percentile(lat, 99))},
        "path_kernel_ms": float(np.mean(path_ms)),
        "roofline": {"bound": "alu", "achieved": achieved / 1e12,
                     "peak": VALU_PEAK_LANE_OPS / 1e12,
                     "unit": "T VALU lane-op slots/s",
                     "frac": achieved / VALU_PEAK_LANE_OPS,
                     "traffic": None},
    }
    line["accuracy_vs_oracle"] = accuracy(args.precision, stream)
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(workload("fp64"), args.cpu_seconds)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
