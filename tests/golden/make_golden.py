"""Writes the stored oracle results used by the full-size GPU parity tests.

Calls only the oracle (``oracle/``): the per-point corrections of every
iteration are spread over worker processes with ``oracle.solve_parallel``,
which runs the same oracle functions in the same order as ``oracle.solve``.

Each case writes ``<name>.json`` (problem, price and deltas of every
iteration, the corrections of a fixed sample of at most 2048 points, and
whole-grid sums) and ``<name>.c.npz`` (every per-point correction of every
iteration, FP64, array ``c`` of shape K_it x n, and the sample variance of
the path terms of every point, FP32, array ``var``: it sets each point's
tolerance scale).

    python tests/golden/make_golden.py eur_put_d1 [amer_put_d1 ...] [--workers 8]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import workloads  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))
MAX_STORED_POINTS = 2048


def stored_points(n: int) -> np.ndarray:
    """Indices of the points whose corrections are stored: all of them for
    n <= 2048, else a fixed seeded sample of 2048 (sorted)."""
    if n <= MAX_STORED_POINTS:
        return np.arange(n)
    rng = np.random.default_rng(12345)
    return np.sort(rng.choice(n, MAX_STORED_POINTS, replace=False))

# name -> (workload factory, kwargs)
CASES = {
    "eur_put_d1": (workloads.eur_put_d1, {}),
    "amer_put_d1_w100": (workloads.amer_put_d1, {"omega": 100.0}),
    "amer_put_d1_w1": (workloads.amer_put_d1, {"omega": 1.0}),
    "amer_basket_d2_w100": (workloads.amer_basket_d2, {"omega": 100.0}),
    "amer_basket_d2_w1": (workloads.amer_basket_d2, {"omega": 1.0}),
    "geo_basket_d5_w100": (workloads.geo_basket_d5, {"omega": 100.0}),
    "geo_basket_d5_w1": (workloads.geo_basket_d5, {"omega": 1.0}),
    "geo_basket_d5_redraw_w1": (workloads.geo_basket_d5, {"omega": 1.0, "redraw": 1}),
}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("names", nargs="+")
    ap.add_argument("--workers", type=int, default=8)
    args = ap.parse_args()
    for name in args.names:
        fn, kw = CASES[name]
        cfg = fn(**kw)
        cfg["precision"] = "fp64"
        t0 = time.time()
        res = oracle.solve_parallel(
            cfg, workers=args.workers,
            progress=lambda k: print("%s: iteration %d done (%.0fs)" %
                                     (name, k, time.time() - t0), flush=True))
        prices, deltas = [], []
        for a in res["alpha"]:
            pr, de = oracle.price_delta(cfg, a, [0.0], [cfg["S0"]])
            prices.append(float(pr[0]))
            deltas.append([float(x) for x in de[0]])
        idx = stored_points(res["n"])
        out = {
            "name": name, "cfg": cfg, "seconds": time.time() - t0,
            "price": prices, "delta": deltas, "n": res["n"],
            "idx": idx.tolist(),
            "c": res["c"][:, idx].tolist(),
            "c_l2": [float(np.linalg.norm(c)) for c in res["c"]],
            "c_sum": [float(np.sum(c)) for c in res["c"]],
        }
        path = os.path.join(HERE, name + ".json")
        with open(path, "w") as f:
            json.dump(out, f)
        np.savez_compressed(os.path.join(HERE, name + ".c.npz"),
                            c=np.asarray(res["c"], dtype=np.float64),
                            var=np.asarray(res["var"], dtype=np.float32))
        print("wrote", path, "price", prices[-1], flush=True)


if __name__ == "__main__":
    main()
