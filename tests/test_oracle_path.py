"""Pins of the oracle's path term: the Euler scheme and its interpolation at
tau against exact Gaussian laws, the local-volatility Euler scheme against a
PDE price, the per-point Monte Carlo correction at k = 0 against the
Black-Scholes formula, and the zero-variance property of the adaptive
control variate when u^k is the exact solution."""
import math

import numpy as np
import pytest

import oracle
import refs
from workloads import problem


def test_euler_and_bridge_exact_for_constant_coefficients():
    sig = np.array([0.2, 0.3])
    cfg = problem(d=2, vol_level=list(sig), rho=0.5, r=0.05, div=[0.0, 0.02],
                  S0=[100.0, 80.0], N=5, T=1.0)
    t0 = 0.2
    x0 = np.log([100.0, 80.0])
    b = 0.05 - np.array([0.0, 0.02]) - 0.5 * sig ** 2
    C = np.array([[1, 0.5], [0.5, 1]])
    Sig = np.outer(sig, sig) * C
    n = 20000
    Z1 = np.empty((n, 2))
    Z2 = np.empty((n, 2))
    taus = np.empty(n)
    for m in range(n):
        P = oracle.path(cfg, t0, x0, 5, m, 0)
        tau = P["tau"]
        taus[m] = tau
        Z1[m] = (P["xtau"] - x0 - b * (tau - t0)) / math.sqrt(tau - t0)
        Z2[m] = (P["xT"] - P["xtau"] - b * (1.0 - tau)) / math.sqrt(1.0 - tau)
        np.testing.assert_allclose(P["sigstar"], sig)
        np.testing.assert_allclose(P["bstar"], b)
    for Z in (Z1, Z2):
        assert np.abs(Z.mean(0)).max() < 4.5 * math.sqrt(0.09 / n)
        np.testing.assert_allclose(np.cov(Z.T), Sig, atol=4.5 * 0.09 * math.sqrt(2 / n))
    # increments before and after tau are independent, and independent of tau
    cross = (Z1[:, :, None] * Z2[:, None, :]).mean(0)
    assert np.abs(cross).max() < 4.5 * 0.09 / math.sqrt(n)
    assert abs(np.corrcoef(taus, Z1[:, 0] ** 2)[0, 1]) < 4.5 / math.sqrt(n)


def test_frozen_coefficients_are_taken_at_the_last_node():
    cfg = problem(d=1, vol_kind="bump", vol_level=0.2, bump_a=0.25,
                  bump_c=100.0, r=0.03, div=0.01, N=7)
    for m in range(50):
        P = oracle.path(cfg, 0.1, [math.log(120.0)], 2, m, 3)
        s = oracle.vol(cfg, 0, 0.0, P["xstar"][0])
        assert P["sigstar"][0] == pytest.approx(s, rel=1e-15)
        assert P["bstar"][0] == pytest.approx(0.03 - 0.01 - s * s / 2, rel=1e-14)
    # theta -> 0 puts X_tau on X_{j*}: check the interpolation is continuous
    # in theta by comparing tau close to a node with the node itself
    close = []
    for m in range(3000):
        P = oracle.path(cfg, 0.1, [math.log(120.0)], 2, m, 3)
        if P["theta"] < 1e-3:
            close.append(abs(P["xtau"][0] - P["xstar"][0]))
    assert close and max(close) < 0.02


def test_local_vol_euler_matches_pde_price():
    # E[e^{-rT} (K - S_T)_+] under the bump local volatility, Euler N=50,
    # against an implicit finite-difference solution of the pricing PDE.
    cfg = problem(d=1, vol_kind="bump", vol_level=0.2, bump_a=0.25,
                  bump_c=100.0, r=0.05, N=50, M=60000, n_t=2, n_x=1, eta=1)
    c, v = oracle.corrections(cfg, None, 0, 0, 1)   # point (t=0, x=log S0)
    mc = math.exp(-0.05) * c[0]
    se = math.exp(-0.05) * math.sqrt(v[0] / cfg["M"])

    def vol(x):
        return 0.2 * (1 + 0.25 * np.exp(-(x - math.log(100.0)) ** 2))
    x, us, _ = refs.penalised_pde_1d(100.0, 100.0, 0.05, vol, 1.0, 0.0,
                                     nx=1201, nt=1000)
    fd = refs.interp_value_delta(x, us[0], 100.0)[0]
    assert abs(mc - fd) < 4.5 * se + 0.01


def test_first_correction_matches_black_scholes_per_point():
    # u^0 = 0 and omega = 0 give f(., 0) = 0, so c^0_i estimates
    # E[Phi(X_T) | X_{t_i} = x_i] = e^{r (T - t_i)} BS_put(e^{x_i}, T - t_i).
    cfg = problem(d=1, n_t=5, n_x=12, M=3000, N=1, eta=2)
    pts = oracle.points(cfg)
    c, v = oracle.corrections(cfg, None, 0, 0, len(pts))
    for (t, x), ci, vi in zip(pts, c, v):
        tau = 1.0 - t
        exact = math.exp(0.05 * tau) * refs.bs_put(math.exp(x), 100.0, 0.05, 0.2, tau)
        # where no path ends in the money the sample variance is 0; bound
        # the true variance by E[Phi^2] <= K E[Phi] there
        var = vi if vi > 0 else 100.0 * exact
        assert abs(ci - exact) <= 4.5 * math.sqrt(var / cfg["M"]) + 1e-12 * (1 + exact)


@pytest.mark.parametrize("d,rho", [(1, 0.0), (2, 0.3), (3, -0.2)])
def test_zero_variance_when_uk_is_the_solution(d, rho):
    # r = 0, f = 0, constant vols, Phi(x) = (sum x_j)^2: the solution
    # u = (sum_j x_j + mu_j (T-t))^2 + (T-t) sum_jk s_j s_k C_jk lies in the
    # span of degree-2 polynomials, so every path term a_m vanishes.
    sig = np.array([0.2, 0.3, 0.25][:d])
    cfg = problem(d=d, r=0.0, vol_level=list(sig), rho=rho, payoff="quad",
                  eta=3, n_t=6, n_x=6 if d < 3 else 4, M=16, N=7,
                  S0=[100.0] * d)
    pts = oracle.points(cfg)
    mu = -0.5 * sig ** 2
    C = np.full((d, d), rho)
    np.fill_diagonal(C, 1.0)
    tau = 1.0 - pts[:, 0]
    y = (pts[:, 1:] + mu * tau[:, None]).sum(1) ** 2 + tau * float(sig @ C @ sig)
    alpha = oracle.fit(cfg, y)
    c, v = oracle.corrections(cfg, alpha, 0, 0, len(pts))
    assert np.abs(c).max() < 1e-10
    assert v.max() < 1e-20
    for m in range(4):
        assert abs(oracle.path_term(cfg, alpha, pts[7, 0], pts[7, 1:], 7, m, 0)) < 1e-10


def test_dupire_volatility_has_the_stated_smile():
    # eq. vol_locale: at t = 0 and the spot s the volatility is
    # 0.6 (1.2 - 1) = 0.12; at every t the bottom of the smile sits at the
    # price S with S e^{rt} = s (the forward of the text), with value
    # 0.6 (1.2 - e^{-0.1 t}) e^{-0.05 sqrt t}; far from it the smile
    # flattens at 0.72 e^{-0.05 sqrt t}
    cfg = problem(d=1, vol_kind="dupire", r=0.05, S0=100.0)
    assert abs(oracle.vol(cfg, 0, 0.0, math.log(100.0)) - 0.12) < 1e-15
    for t in (0.0, 0.3, 1.0, 2.5):
        S = np.linspace(40.0, 160.0, 24001)
        v = np.array([oracle.vol(cfg, 0, t, math.log(s)) for s in S])
        assert abs(S[np.argmin(v)] - 100.0 * math.exp(-0.05 * t)) < 0.01
        damp = math.exp(-0.05 * math.sqrt(t))
        assert abs(v.min() - 0.6 * (1.2 - math.exp(-0.1 * t)) * damp) < 1e-8
        far = oracle.vol(cfg, 0, t, math.log(1000.0))
        assert abs(far - 0.72 * damp) < 1e-12


def test_time_dependent_local_vol_euler_matches_pde_price():
    # the Euler scheme evaluates sigma at the time of each step: the
    # Dupire-type European put against an implicit finite-difference
    # solution with the volatility at each step's time
    cfg = problem(d=1, vol_kind="dupire", vol_level=0.3, r=0.05, N=50,
                  M=60000, n_t=2, n_x=1, eta=1)
    c, v = oracle.corrections(cfg, None, 0, 0, 1)   # point (t=0, x=log S0)
    mc = math.exp(-0.05) * c[0]
    se = math.exp(-0.05) * math.sqrt(v[0] / cfg["M"])

    def vol_t(t, x):
        dev = np.exp(x) * math.exp(0.05 * t) - 100.0
        return 0.6 * (1.2 - math.exp(-0.1 * t) * np.exp(-0.001 * dev ** 2)) * \
            math.exp(-0.05 * math.sqrt(t))
    x, us, _ = refs.penalised_pde_1d(100.0, 100.0, 0.05, lambda x: x * 0, 1.0,
                                     0.0, nx=1201, nt=1000, vol_t=vol_t)
    fd = refs.interp_value_delta(x, us[0], 100.0)[0]
    assert abs(mc - fd) < 4.5 * se + 0.01
    # freezing the volatility at t = 0 would be a different model
    x0, us0, _ = refs.penalised_pde_1d(100.0, 100.0, 0.05,
                                       lambda x: vol_t(0.0, x), 1.0, 0.0,
                                       nx=1201, nt=1000)
    assert abs(refs.interp_value_delta(x0, us0[0], 100.0)[0] - fd) > 5 * (4.5 * se + 0.01)
