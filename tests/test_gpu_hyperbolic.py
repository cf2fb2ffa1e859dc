"""Hyperbolic index sets (Section 4.2, eq. hyper_set) on the GPU against the
FP64 oracle.

1. d = 10, eta = 5 with q = 0.5, 0.6 and 0.7 (p = 111, 221, 386), and
   eta = 4 with q = 0.6 (p = 100): each set has path kernels of its own.  Whole solves at M = 512 paths per point (two
   paths per lane), N = 10 Euler steps, two Picard iterations, on uniform
   points (t, x) over [0, T] x D, every per-point correction, the price and
   the deltas compared with the oracle (which builds the same set itself).
2. A set without kernels of its own (d = 2, eta = 4, q = 0.6) runs on the
   total-degree kernel with the coefficients outside the set held at zero:
   the same comparison, in FP64 and FP32 paths.

3. The largest set (q = 0.7, p = 386) and the sparsest (eta = 4, q = 0.6,
   p = 100) at the shape of the paper's d = 10 runs (n = 1000 points,
   M = 30,000, N = 10) with the narrow domain of those runs (one standard deviation: many paths leave it, where Chebyshev
   values of degree 5 grow large), iteration 1 from the least-squares fit of
   the payoff at the points -- the polynomial handed to the oracle as its
   monomial coefficients and to the library as point values -- on 16
   sampled points.

Tolerances are those of every parity test: corrections within
1e-8 / 2e-3 (1 + |c| + sd) for FP64 / FP32 paths (sd the oracle's sample
standard deviation of the path terms at the point), |d price| <= 1e-4 K /
5e-4 K, |d delta| <= 1e-4 / 5e-3."""
import math
import multiprocessing as mp

import numpy as np
import pytest

import oracle
import paper_1102_4666_amd as bsde
from workloads import problem

pytestmark = pytest.mark.gpu
TOL = {"fp64": dict(c=1e-8, price=1e-4, delta=1e-4),
       "fp32": dict(c=2e-3, price=5e-4, delta=5e-3)}


def _compare(cfg, tiling=None, workers=8):
    ref = oracle.solve_parallel(cfg, workers=workers, chunk=16) if workers else oracle.solve(cfg)
    rp, rd = oracle.price_delta(cfg, ref["alpha"][-1], [0.0], [cfg["S0"]])
    with bsde.Problem(cfg) as P:
        if tiling:
            P.set_tiling(*tiling)
        P.solve()
        c = np.array([P.corrections(k)[0] for k in range(cfg["K_it"])])
        pr, de = P.price_delta()
        alpha = P.coefficients()
        p = P.p
    tol = TOL[cfg["precision"]]
    scale = 1.0 + np.abs(ref["c"]) + np.sqrt(np.maximum(ref["var"], 0.0))
    err = np.abs(c - ref["c"]) / scale
    print("  p = %d: max scaled correction error %.3g; price gpu %.8g oracle %.8g; "
          "max |d delta| %.3g" % (p, err.max(), pr[0], rp[0],
                                   np.abs(de[0] - rd[0]).max()), flush=True)
    assert err.max() <= tol["c"]
    assert abs(pr[0] - rp[0]) <= tol["price"] * cfg["K"]
    assert np.abs(de[0] - rd[0]).max() <= tol["delta"]
    return p, alpha


@pytest.mark.parametrize("eta,q,p_expected",
                         [(5, 0.5, 111), (5, 0.6, 221), (5, 0.7, 386), (4, 0.6, 100)])
def test_d10_hyperbolic_sets_against_oracle(eta, q, p_expected):
    n = int(math.ceil(1.25 * p_expected))
    cfg = problem(d=10, vol_kind="bump",
                  vol_level=[0.15 + 0.02 * j for j in range(10)], bump_a=0.25,
                  rho=0.2, payoff="call", S0=100.0, grid="uniform", n_x=n,
                  eta=eta, q=q, M=512, N=10, K_it=2, omega=1.0,
                  precision="fp32", seed=13)
    print("d=10 eta=%d q=%g (n=%d)" % (eta, q, n), flush=True)
    assert len(oracle.index_set(11, eta, q)) == p_expected
    p, _ = _compare(cfg, tiling=(1, 2))
    assert p == p_expected


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_hyperbolic_set_on_the_total_degree_kernel(prec):
    cfg = problem(d=2, vol_kind="bump", vol_level=[0.2, 0.3], bump_a=0.25,
                  rho=0.3, S0=[100.0, 100.0], n_t=6, n_x=8, eta=4, q=0.6,
                  M=400, N=8, K_it=3, omega=1.0, precision=prec, seed=14)
    print("d=2 eta=4 q=0.6 on the total-degree kernel, %s" % prec, flush=True)
    p, alpha = _compare(cfg, workers=0)
    # the total-degree kernel (p = binom(3 + 4, 4) = 35) with the 35 - 16
    # coefficients outside the set held at zero
    assert p == 35
    assert np.count_nonzero(alpha) == len(oracle.index_set(3, 4, 0.6)) == 16


def _corrections_at(args):
    cfg, alpha, k, i = args
    c, v = oracle.corrections(cfg, alpha, k, i, i + 1)
    return float(c[0]), float(v[0])


@pytest.mark.parametrize("eta,q,p_expected", [(5, 0.7, 386), (4, 0.6, 100)])
def test_d10_study_shape_iteration1_sampled(eta, q, p_expected):
    from workloads import call_basket_d10_hyperbolic
    cfg = call_basket_d10_hyperbolic()
    cfg.update(eta=eta, q=q, redraw=0, K_it=2)
    n, p = oracle.sizes(cfg)
    assert p == p_expected
    pts = oracle.points(cfg)
    y = np.array([oracle.payoff(cfg, pts[i, 1:]) for i in range(n)])
    alpha = oracle.fit(cfg, y)
    print("d=10 eta=%d q=%g at the study shape, iteration 1" % (eta, q), flush=True)
    with bsde.Problem(cfg) as P:
        P.fit_values(y, 1)
        P.solve()
        c1 = P.corrections(1)[0]
    idx = np.sort(np.random.default_rng(8).choice(n, 16, replace=False))
    with mp.get_context("fork").Pool(8) as pool:
        ref = pool.map(_corrections_at, [(cfg, alpha, 1, int(i)) for i in idx])
    worst = 0.0
    for i, (c, v) in zip(idx, ref):
        err = abs(c1[i] - c) / (1.0 + abs(c) + math.sqrt(max(v, 0.0)))
        worst = max(worst, err)
        assert err <= TOL["fp32"]["c"], (int(i), c1[i], c, err)
    print("  16 sampled points, max scaled error %.3g" % worst, flush=True)
