"""Pins of the oracle's whole Picard loop (Algorithm "algodetail"):
the exact-expectation projected Picard map (no Monte Carlo), the
Black-Scholes price and delta, linearity in the payoff (put-call parity),
resumption from saved coefficients, the shrinking variance of the adaptive
control variate, Picard contraction, and the American-put bracket."""
import math

import numpy as np
import pytest

import oracle
import refs
from workloads import problem


def _price(cfg, alpha):
    S0 = cfg["S0"]
    pr, de = oracle.price_delta(cfg, alpha, [0.0], [S0])
    return pr[0], de[0]


def test_matches_exact_expectation_picard_d1():
    cfg = problem(d=1, n_t=8, n_x=32, eta=4, M=2000, N=1, K_it=3)
    pts = oracle.points(cfg)
    _, exact = refs.exact_picard_const_vol_1d(100.0, 100.0, 0.05, 0.2, 1.0,
                                              0.0, pts, 4, 4.0, 3)
    res = oracle.solve(cfg)
    got = [_price(cfg, a)[0] for a in res["alpha"]]
    # tolerances: 4.5 x the Monte Carlo std of each iterate (8 seeds)
    for k, tol in zip([1, 2, 3], [0.25, 0.055, 0.06]):
        assert abs(got[k] - exact[k]) < tol, (k, got[k], exact[k])


def test_matches_exact_expectation_picard_d2_correlated():
    cfg = problem(d=2, rho=0.3, vol_level=[0.2, 0.3], S0=[100.0, 100.0],
                  payoff="put_geom", n_t=6, n_x=12, eta=3, M=1000, N=1,
                  K_it=3)
    pts = oracle.points(cfg)
    exact = refs.exact_picard_const_vol(cfg, pts, 3)
    res = oracle.solve(cfg)
    got = [_price(cfg, a)[0] for a in res["alpha"]]
    for k, tol in zip([1, 2, 3], [0.13, 0.035, 0.06]):
        assert abs(got[k] - exact[k]) < tol, (k, got[k], exact[k])


def test_black_scholes_price_and_delta_d1():
    # 64 x 8 grid, eta = 4: the projection bias of this grid is -0.018
    # (exact-expectation iteration); Monte Carlo std of the price ~0.012.
    cfg = problem(d=1, n_t=8, n_x=64, eta=4, M=2000, N=1, K_it=4)
    res = oracle.solve(cfg)
    pr, de = _price(cfg, res["alpha"][-1])
    assert abs(pr - refs.bs_put(100, 100, 0.05, 0.2, 1.0)) < 0.08
    assert abs(de[0] - refs.bs_put_delta(100, 100, 0.05, 0.2, 1.0)) < 0.012


def test_linear_in_payoff_put_call_parity():
    # omega = 0 makes the algorithm linear in Phi on fixed random streams:
    # solve(call) - solve(put) = solve(mean e^x - K) up to rounding.
    base = problem(d=2, vol_kind="bump", vol_level=[0.2, 0.25], bump_a=0.25,
                   rho=0.2, S0=[100.0, 100.0], n_t=5, n_x=8, eta=3, M=200,
                   N=6, K_it=3)
    a_call = oracle.solve(dict(base, payoff="call"))["alpha"]
    a_put = oracle.solve(dict(base, payoff="put"))["alpha"]
    a_fwd = oracle.solve(dict(base, payoff="fwd"))["alpha"]
    scale = np.abs(a_fwd).max()
    np.testing.assert_allclose(a_call - a_put, a_fwd, atol=1e-10 * scale)


def test_resume_from_saved_coefficients_is_bitwise():
    cfg = problem(d=1, vol_kind="bump", vol_level=0.2, bump_a=0.25,
                  n_t=6, n_x=10, eta=4, M=64, N=10, K_it=4, omega=1.0)
    full = oracle.solve(cfg)
    head = oracle.solve(cfg, k_end=2)
    tail = oracle.solve(cfg, k_start=2, alpha_start=head["alpha"][-1])
    np.testing.assert_array_equal(full["alpha"][2], head["alpha"][-1])
    np.testing.assert_array_equal(full["alpha"][-1], tail["alpha"][-1])
    np.testing.assert_array_equal(full["c"][2:], tail["c"])


def test_control_variate_shrinks_the_variance():
    cfg = problem(d=1, n_t=8, n_x=32, eta=4, M=400, N=1, K_it=5)
    res = oracle.solve(cfg)
    mv = res["var"].mean(1)
    # calibrated: the mean variance falls ~5x by k = 4 on this grid (the
    # residual is the projection error of u^k near the domain edges)
    assert mv[-1] < mv[0] / 4 and mv[2] < mv[0] / 4, mv


@pytest.mark.parametrize("omega", [0.0, 1.0])
def test_picard_contraction(omega):
    cfg = problem(d=1, n_t=8, n_x=32, eta=4, M=1000, N=1, K_it=5,
                  omega=omega)
    a = oracle.solve(cfg)["alpha"]
    steps = [np.linalg.norm(a[k + 1] - a[k]) for k in range(len(a) - 1)]
    assert steps[1] < steps[0] and steps[2] < steps[1], steps


def test_penalty_term_matches_exact_expectation_and_bracket():
    # omega = 1: the penalised driver of eq. bsde-penal-2.
    cfg = problem(d=1, n_t=8, n_x=32, eta=4, M=2000, N=1, K_it=4, omega=1.0)
    pts = oracle.points(cfg)
    _, exact = refs.exact_picard_const_vol_1d(100.0, 100.0, 0.05, 0.2, 1.0,
                                              1.0, pts, 4, 4.0, 4)
    _, exact_eur = refs.exact_picard_const_vol_1d(100.0, 100.0, 0.05, 0.2,
                                                  1.0, 0.0, pts, 4, 4.0, 4)
    got = _price(cfg, oracle.solve(cfg)["alpha"][-1])[0]
    assert abs(got - exact[-1]) < 0.07
    # the penalty raises the price above the European one, below the
    # American (CRR) one
    crr = refs.crr_american_put(100, 100, 0.05, 0.2, 1.0, steps=2000)
    assert exact_eur[-1] + 0.05 < got < crr + 0.1


def test_redrawn_points_follow_the_exact_expectation_map():
    # Algorithm 1 with new random points at every iteration: the projection
    # of iteration k uses the points of iteration k.  With only 240 points
    # for 20 basis functions the exact-expectation iterates themselves move
    # by +-1 from one point set to the next; the Monte Carlo oracle tracks
    # the exact map on the same point sets (tolerances: 4.5 x the standard
    # deviation of the difference over 8 seeds).
    cfg = problem(d=2, rho=0.3, vol_level=[0.2, 0.3], S0=[100.0, 100.0],
                  payoff="put_geom", grid="random", redraw=1, n_t=6,
                  n_x=40, eta=3, M=1000, N=1, K_it=3)
    assert not np.array_equal(oracle.points(cfg, 0), oracle.points(cfg, 1))
    exact = refs.exact_picard_const_vol(cfg, lambda k: oracle.points(cfg, k), 3)
    fixed = refs.exact_picard_const_vol(cfg, oracle.points(cfg, 0), 3)
    res = oracle.solve(cfg)
    got = [_price(cfg, a)[0] for a in res["alpha"]]
    for k, tol in zip([1, 2, 3], [0.35, 0.19, 0.06]):
        assert abs(got[k] - exact[k]) < tol, (k, got[k], exact[k])
    # the redrawn point sets matter: the fixed-grid map is far away
    assert max(abs(a - b) for a, b in zip(exact[2:], fixed[2:])) > 5 * 0.19


def test_redraw_keeps_an_exact_solution_fixed():
    # the solution of the zero-variance problem lies in the span, so every
    # redrawn projection returns the same coefficients: alpha^k = alpha^0
    sig = np.array([0.2, 0.3])
    cfg = problem(d=2, r=0.0, vol_level=list(sig), rho=0.3, payoff="quad",
                  eta=3, grid="random", redraw=1, n_t=5, n_x=30, M=16, N=7,
                  S0=[100.0, 100.0], K_it=3)
    pts = oracle.points(cfg)
    C = np.array([[1, 0.3], [0.3, 1]])
    tau = 1.0 - pts[:, 0]
    y = (pts[:, 1:] - 0.5 * sig ** 2 * tau[:, None]).sum(1) ** 2 + \
        tau * float(sig @ C @ sig)
    a0 = oracle.fit(cfg, y)
    res = oracle.solve(cfg, 0, a0)
    for k in range(1, 4):
        np.testing.assert_allclose(res["alpha"][k], a0, rtol=0, atol=1e-8)
    assert np.abs(res["c"]).max() < 1e-10


def test_uniform_redrawn_points_follow_the_exact_expectation_map():
    # the literal point draw of Algorithm 1: (t, x) uniform over [0, T] x D,
    # new at every iteration; the Monte Carlo oracle tracks the exact
    # projected map on the same point sets (4.5 x the standard deviation of
    # the difference over 8 seeds)
    cfg = problem(d=2, rho=0.3, vol_level=[0.2, 0.3], S0=[100.0, 100.0],
                  payoff="put_geom", grid="uniform", redraw=1, n_x=240,
                  eta=3, M=1000, N=1, K_it=3)
    exact = refs.exact_picard_const_vol(cfg, lambda k: oracle.points(cfg, k), 3)
    res = oracle.solve(cfg)
    got = [_price(cfg, a)[0] for a in res["alpha"]]
    for k, tol in zip([1, 2, 3], [0.28, 0.25, 0.11]):
        assert abs(got[k] - exact[k]) < tol, (k, got[k], exact[k])
