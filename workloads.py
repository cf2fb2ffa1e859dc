"""Seeded synthetic workloads shared by the tests, the smoke check and the
benchmark.

This module holds problem parameters only -- no arithmetic of the method.
Each workload is a plain dict understood by both the GPU binding
(``paper_1102_4666_amd``) and the oracle binding (``oracle``).

The option model is the log-price local-volatility model of Section 5 of
Labart & Lelong (arXiv:1102.4666), eq. 4, with the uniform-correlation
Brownian motion of Section 6.2; payoffs are the basket puts and calls of
eqs. put_payoff / call_payoff (plus a geometric basket).  The paper's
experiments use synthetic model parameters, never a dataset.
"""
from __future__ import annotations

import copy

import numpy as np


def problem(**kw) -> dict:
    """A d=1 Black-Scholes European put with small sizes, overridden by kw."""
    cfg = {
        "d": 1,
        "vol_kind": "const",   # "const" | "bump" | "dupire"
        "vol_level": [0.2],
        "bump_a": 0.0,
        "bump_c": 100.0,
        "rho": 0.0,
        "r": 0.05,
        "div": 0.0,
        "payoff": "put",       # put | call | put_geom | call_geom | fwd | quad
        "K": 100.0,
        "T": 1.0,
        "S0": [100.0],
        "grid": "tensor",      # tensor | random
        "redraw": 0,           # random grid: new points every iteration
        "kernel_bw": 0.0,      # > 0: the kernel operator (Section 3.2)
        "n_t": 8,
        "n_x": 16,
        "width": 4.0,
        "eta": 6,
        "q": 1.0,
        "M": 64,
        "N": 8,
        "K_it": 2,
        "omega": 0.0,
        "seed": 0,
        "precision": "fp64",   # fp64 | fp32 (FP32 paths, FP64 sums/update)
    }
    cfg.update(kw)
    d = cfg["d"]
    for key in ("vol_level", "S0"):
        v = np.broadcast_to(np.asarray(cfg[key], float), (d,))
        cfg[key] = [float(x) for x in v]
    return cfg


def vol_levels(d: int, seed: int = 0, lo: float = 0.15, hi: float = 0.35):
    """Per-asset volatility levels drawn uniformly in [lo, hi] (seeded)."""
    rng = np.random.default_rng(seed)
    return [float(x) for x in rng.uniform(lo, hi, size=d)]


# The benchmark workloads (the serving mix draws its requests from them).
def eur_put_d1() -> dict:
    """d=1 European put, Black-Scholes sigma=0.2, 64 space x 8 time points,
    M=1000, N=20, 5 Picard iterations, FP64, seed 0."""
    return problem(d=1, vol_kind="const", vol_level=0.2, r=0.05, K=100.0,
                   S0=100.0, T=1.0, payoff="put", omega=0.0, grid="tensor",
                   n_t=8, n_x=64, eta=4, M=1000, N=20, K_it=5,
                   precision="fp64", seed=0)


def amer_put_d1(omega: float = 100.0, precision: str = "fp32") -> dict:
    """d=1 American put (penalised BSDE, penalty 100), local volatility
    0.2 (1 + 0.25 exp(-(log(S/100))^2)), 128 space x 16 time points,
    M=4000, N=50, 8 Picard iterations."""
    return problem(d=1, vol_kind="bump", vol_level=0.2, bump_a=0.25,
                   bump_c=100.0, r=0.05, K=100.0, S0=100.0, T=1.0,
                   payoff="put", omega=omega, grid="tensor", n_t=16,
                   n_x=128, eta=4, M=4000, N=50, K_it=8,
                   precision=precision, seed=0)


def amer_basket_d2(omega: float = 100.0, precision: str = "fp32") -> dict:
    """d=2 American arithmetic-basket put, independent bump local vols,
    rho=0.3, 32^2 space x 16 time points, M=2000, N=50, 8 iterations."""
    return problem(d=2, vol_kind="bump", vol_level=0.2, bump_a=0.25,
                   bump_c=100.0, rho=0.3, r=0.05, K=100.0, S0=100.0, T=1.0,
                   payoff="put", omega=omega, grid="tensor", n_t=16, n_x=32,
                   eta=5, M=2000, N=50, K_it=8, precision=precision, seed=0)


def geo_basket_d5(omega: float = 100.0, precision: str = "fp32",
                  redraw: int = 0) -> dict:
    """d=5 American geometric-basket put, per-asset levels U[0.15, 0.35]
    (seeded), rho=0.2, 4096 random spatial points x 10 times, M=1000,
    N=50, 10 iterations (redraw=1: new spatial points every iteration)."""
    return problem(d=5, vol_kind="bump", vol_level=vol_levels(5, seed=0),
                   bump_a=0.25, bump_c=100.0, rho=0.2, r=0.05, K=100.0,
                   S0=100.0, T=1.0, payoff="put_geom", omega=omega,
                   grid="random", redraw=redraw, n_t=10, n_x=4096, eta=3,
                   M=1000, N=50, K_it=10, precision=precision, seed=0)


def eur_put_d1_kernel(precision: str = "fp32") -> dict:
    """d=1 European put, Black-Scholes sigma=0.2, with the kernel operator of
    Section 3.2 (bandwidth 0.1 in the mapped coordinates) in place of least
    squares: 64 space x 8 time points, M=1000, N=20, 5 Picard iterations."""
    return problem(d=1, vol_kind="const", vol_level=0.2, r=0.05, K=100.0,
                   S0=100.0, T=1.0, payoff="put", omega=0.0, grid="tensor",
                   n_t=8, n_x=64, eta=2, M=1000, N=20, K_it=5,
                   kernel_bw=0.1, precision=precision, seed=0)


def call_basket_d10_hyperbolic(precision: str = "fp32") -> dict:
    """d=10 European call basket of Section 6.2.1: Black-Scholes sigma=0.2,
    rho=0.2, K=S0=100, T=1, hyperbolic index set eta=5, q=0.6 (p=221), 1000
    points drawn uniformly at every iteration, domain +-1 standard deviation,
    M=30000, N=10, 10 iterations."""
    return problem(d=10, vol_level=0.2, rho=0.2, T=1.0, r=0.05, K=100.0,
                   S0=100.0, payoff="call", omega=0.0, grid="uniform",
                   redraw=1, n_x=1000, eta=5, q=0.6, N=10, K_it=10,
                   width=1.0, M=30000, precision=precision, seed=0)


def put_basket_d10(omega: float = 1.0, precision: str = "fp32", M: int = 500) -> dict:
    """The d = 10 request shape of the serving mix: arithmetic put on 10
    assets, bump local vol with levels U[0.15,0.35], rho = 0.2, 8192 random
    spatial points x 10 times, total degree 3 (p = 364), N = 50, 10 Picard
    iterations, M = 500."""
    return problem(d=10, vol_kind="bump", vol_level=vol_levels(10, 0),
                   bump_a=0.25, bump_c=100.0, rho=0.2, r=0.05, S0=100.0,
                   T=1.0, payoff="put", grid="random", n_t=10, n_x=8192, eta=3,
                   N=50, K_it=10, M=M, omega=omega, precision=precision)


def serving_request(idx: int, rng: np.random.Generator,
                    dims=(1, 2, 5, 10)) -> dict:
    """One request of the serving mix: d drawn from dims, strike U[80,120],
    European/American 50/50, M in {500,1000,2000,4000} (d = 10: M = 500,
    8192 random spatial points x 10 times), FP32 paths; the grid and Euler
    sizes of the benchmark workload of that dimension."""
    d = int(rng.choice(list(dims)))
    K = float(rng.uniform(80.0, 120.0))
    american = bool(rng.integers(0, 2))
    M = int(rng.choice([500, 1000, 2000, 4000]))
    if d == 1:
        base = amer_put_d1()
    elif d == 2:
        base = amer_basket_d2()
    elif d == 5:
        base = geo_basket_d5()
    else:
        base = put_basket_d10()
        M = 500   # the d = 10 request shape of the mix is stated at M = 500
    cfg = copy.deepcopy(base)
    cfg.update(K=K, M=M, omega=(1.0 if american else 0.0), seed=1 + idx,
               precision="fp32")
    return cfg


WORKLOADS = {"eur_put_d1": eur_put_d1, "amer_put_d1": amer_put_d1,
             "amer_basket_d2": amer_basket_d2, "geo_basket_d5": geo_basket_d5,
             "eur_put_d1_kernel": eur_put_d1_kernel, "put_basket_d10": put_basket_d10}
