"""d = 10 path kernels against the FP64 oracle at the shapes they serve.

1. The serving mix's d = 10 request shape: local volatility with per-asset
   levels, rho = 0.2, 8192 random spatial points x 10 time nodes (81,920
   points), total degree eta = 3 (p = 364 Chebyshev functions, 67
   channels), N = 50 Euler steps, M = 512 paths per point -- two paths per
   lane in the default tiling, the path loop that reloads the kernel's
   spilled registers and runs the contraction over the live rows of the
   channel table once per path.  FP32 and FP64 paths.  Per-point
   corrections are compared on sampled points:
   iteration 0 from u^0 = 0, and iteration 1 from a degree-3 polynomial
   whose monomial coefficients are given to the oracle directly and whose
   values at the points are given to the library (its least-squares fit
   recovers the same polynomial in its Chebyshev basis).
2. Whole small solves (every correction, price and delta) of the total-
   degree eta = 3 set (FP32 and FP64 paths) and of the hyperbolic set
   eta = 5, q = 0.6 (p = 221; FP32 paths, the only kernel of that set) at
   M = 600 and N = 10, with the tiling forced to three paths per lane.

Tolerances as for every parity test: corrections within 2e-3 / 1e-8
(1 + |c| + sd) for FP32 / FP64 paths, with sd the oracle's sample standard
deviation of the path terms; |d price| <= 5e-4 K / 1e-4 K, |d delta| <=
5e-3 / 1e-4."""
import numpy as np
import pytest

import oracle
import paper_1102_4666_amd as bsde
from workloads import problem, vol_levels

pytestmark = pytest.mark.gpu
TOL = {"fp32": dict(c=2e-3, price=5e-4, delta=5e-3),
       "fp64": dict(c=1e-8, price=1e-4, delta=1e-4)}


def _serving_shape(**kw):
    cfg = problem(d=10, vol_kind="bump", vol_level=vol_levels(10, 0),
                  bump_a=0.25, bump_c=100.0, rho=0.2, r=0.05, S0=100.0,
                  T=1.0, payoff="put", grid="random", n_t=10, n_x=8192,
                  eta=3, N=50, M=512, K_it=1, omega=1.0, K=100.0,
                  precision="fp32", seed=7)
    cfg.update(kw)
    return cfg


def _sample(n, count=16, seed=5):
    rng = np.random.default_rng(seed)
    return np.sort(rng.choice(n, count, replace=False))


def _compare_sampled(cfg, alpha_mono, k, c_gpu, idx):
    tol = TOL[cfg["precision"]]["c"]
    worst = 0.0
    for i in idx:
        c, v = oracle.corrections(cfg, alpha_mono, k, int(i), int(i) + 1)
        err = abs(c_gpu[i] - c[0]) / (1.0 + abs(c[0]) + np.sqrt(max(v[0], 0.0)))
        worst = max(worst, err)
        assert err <= tol, (k, int(i), c_gpu[i], c[0], err)
    print("  k=%d: %d sampled points, max scaled error %.3g" % (k, len(idx), worst),
          flush=True)


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_d10_serving_shape_iteration0_sampled(prec):
    cfg = _serving_shape(K_it=1, precision=prec)
    print("d=10 serving shape, iteration 0, %s" % prec, flush=True)
    with bsde.Problem(cfg) as P:
        assert (P.n, P.p, P.C) == (81920, 364, 67)
        np.testing.assert_allclose(P.points(), oracle.points(cfg), rtol=0, atol=1e-13)
        P.solve()
        c0 = P.corrections(0)[0]
    _compare_sampled(cfg, None, 0, c0, _sample(cfg["n_t"] * cfg["n_x"]))


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_d10_serving_shape_iteration1_sampled(prec):
    cfg = _serving_shape(K_it=2, precision=prec)
    nu = oracle.index_set(11, 3)
    rng = np.random.default_rng(17)
    deg = nu.sum(axis=1)
    # u^1 = a degree-3 polynomial in the mapped coordinates z (the oracle's
    # monomial basis): a level near the payoff's and smaller terms of
    # higher degree, so that every derivative channel is exercised
    alpha = rng.normal(size=len(nu)) * np.array([4.0, 1.5, 0.5, 0.15])[deg]
    alpha[deg == 0] = 6.0
    B = oracle.basis_matrix(cfg)
    y = B @ alpha
    del B
    print("d=10 serving shape, iteration 1 from a fitted polynomial, %s" % prec,
          flush=True)
    with bsde.Problem(cfg) as P:
        P.fit_values(y, 1)
        P.solve()
        c1 = P.corrections(1)[0]
    _compare_sampled(cfg, alpha, 1, c1, _sample(cfg["n_t"] * cfg["n_x"], seed=6))


@pytest.mark.parametrize("eta,q,n,prec", [(3, 1.0, 400, "fp32"), (3, 1.0, 400, "fp64"),
                                          (5, 0.6, 260, "fp32")])
def test_d10_small_solve_three_paths_per_lane(eta, q, n, prec):
    # n points (t, x) uniform over [0, T] x D: a full-rank basis matrix as
    # soon as n >= p (time nodes shared by few spatial points would not
    # resolve the spatial functions of each time degree)
    cfg = problem(d=10, vol_kind="bump",
                  vol_level=[0.15 + 0.02 * j for j in range(10)], bump_a=0.25,
                  rho=0.2, payoff="call" if q < 1 else "put", S0=100.0,
                  grid="uniform", n_x=n, eta=eta, q=q, M=600, N=10, K_it=2,
                  omega=1.0, precision=prec, seed=11)
    print("d=10 small solve eta=%d q=%g %s" % (eta, q, prec), flush=True)
    # the oracle's loop with each iteration's points spread over worker
    # processes (identical results to oracle.solve)
    ref = oracle.solve_parallel(cfg, workers=8, chunk=16)
    rp, rd = oracle.price_delta(cfg, ref["alpha"][-1], [0.0], [cfg["S0"]])
    with bsde.Problem(cfg) as P:
        P.set_tiling(1, 3)
        P.solve()
        c = np.array([P.corrections(k)[0] for k in range(cfg["K_it"])])
        pr, de = P.price_delta()
    scale = 1.0 + np.abs(ref["c"]) + np.sqrt(np.maximum(ref["var"], 0.0))
    err = np.abs(c - ref["c"]) / scale
    print("  max scaled correction error %.3g; price gpu %.8g oracle %.8g" %
          (err.max(), pr[0], rp[0]), flush=True)
    tol = TOL[prec]
    assert err.max() <= tol["c"]
    assert abs(pr[0] - rp[0]) <= tol["price"] * cfg["K"]
    assert np.abs(de[0] - rd[0]).max() <= tol["delta"]
