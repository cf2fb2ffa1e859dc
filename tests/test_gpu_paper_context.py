"""The paper's own d = 5 experiments (Section 6) run through the library
as context checks of the method at the paper's scale -- not parity: the
paper's benchmarks come from other Monte Carlo methods, and its figures
carry their own noise.

Set-up as printed in Section 6: n = 1000 points (t, x) uniform over
[0, T] x D, redrawn at every iteration (Algorithm 1),
eta = 3, q = 1, M = 50,000 (Black-Scholes European put basket, T = 3),
M = 30,000 and N = 10 (Dupire-type volatility of eq. vol_locale), M = 5000
(Black-Scholes American put basket, 5 iterations).  The domain half-width
is one volatility level times sqrt(T) around log S0: with the wider box
of the parity workloads (4 sigma sqrt(T)) the least-squares projection on
1000 random points in six variates is far noisier (seed-to-seed spread
0.5 on a 2.0 price).  Every workload runs over 8 seeds; the mean is
compared with the printed value, within a tolerance covering the paper's
confidence interval, the spread of our 8-seed mean and the reading
differences (time nodes, domain, Euler N where the paper gives none)."""
import numpy as np
import pytest

import paper_1102_4666_amd as bsde
from workloads import problem

pytestmark = pytest.mark.gpu

BASE = dict(grid="uniform", redraw=1, n_x=1000, eta=3, N=10, K_it=10,
            width=1.0, precision="fp32")


def _mean_over_seeds(cfg, seeds=8):
    prices, deltas = [], []
    for seed in range(seeds):
        with bsde.Problem(dict(cfg, seed=seed)) as P:
            P.solve()
            pr, de = P.price_delta()
        prices.append(pr[0])
        deltas.append(de[0])
    return np.mean(prices), np.std(prices, ddof=1), np.mean(deltas, axis=0)


def test_black_scholes_european_put_basket_d5():
    # Section 6.2.1, European put basket: benchmark 2.0353, CI (2.0323, 2.0383)
    cfg = problem(d=5, vol_level=0.2, rho=0.1, T=3.0, r=0.05, K=100.0,
                  S0=100.0, payoff="put", omega=0.0, M=50000, **BASE)
    m, s, _ = _mean_over_seeds(cfg)
    print("BS European put d=5: %.4f (seed std %.4f) vs 2.0353" % (m, s))
    assert abs(m - 2.0353) < 0.1


def test_dupire_european_put_basket_d5():
    # Section 6.3: benchmark 1.745899, CI (1.737899, 1.753899); delta -0.0625
    cfg = problem(d=5, vol_kind="dupire", vol_level=0.2, rho=0.0, T=1.0,
                  r=0.05, K=100.0, S0=100.0, payoff="put", omega=0.0,
                  M=30000, **BASE)
    m, s, dl = _mean_over_seeds(cfg)
    print("Dupire European put d=5: %.4f (seed std %.4f) vs 1.7459; "
          "delta %s vs -0.0625" % (m, s, np.round(dl, 4)))
    assert abs(m - 1.745899) < 0.15
    assert np.all(np.abs(dl + 0.0625) < 0.02)


def test_dupire_american_put_basket_d5():
    # Section 6.3: price around 6.30, no benchmark (delta / 0.1 dividends)
    cfg = problem(d=5, vol_kind="dupire", vol_level=0.2, rho=0.0, div=0.1,
                  T=1.0, r=0.05, K=100.0, S0=100.0, payoff="put", omega=1.0,
                  M=30000, **BASE)
    m, s, dl = _mean_over_seeds(cfg)
    print("Dupire American put d=5: %.4f (seed std %.4f) vs ~6.30; delta %s"
          % (m, s, np.round(dl, 4)))
    assert abs(m - 6.30) < 0.6


def test_black_scholes_american_put_basket_delta_d5():
    # Table tab:delta_put_amer_5, iteration 5: deltas -0.1090 ... -0.1113
    # (the five assets are exchangeable; their printed spread is noise)
    cfg = problem(d=5, vol_level=0.25, rho=0.2, div=0.1, T=1.0, r=0.05,
                  K=100.0, S0=100.0, payoff="put", omega=1.0, M=5000,
                  **dict(BASE, K_it=5))
    printed = np.array([-0.108961, -0.105648, -0.105725, -0.105647, -0.111274])
    m, s, dl = _mean_over_seeds(cfg)
    print("BS American put d=5: price %.4f; mean delta %.4f vs printed mean %.4f"
          % (m, dl.mean(), printed.mean()))
    assert abs(dl.mean() - printed.mean()) < 0.01


def test_black_scholes_european_call_basket_d10():
    # Section 6.2.1, European call basket d = 10 (Figure fig:call_euro_10):
    # M = 30,000, eta = 5, q = 0.6; benchmark 7.0207, CI (7.0125, 7.0288)
    cfg = problem(d=10, vol_level=0.2, rho=0.2, T=1.0, r=0.05, K=100.0,
                  S0=100.0, payoff="call", omega=0.0, M=30000,
                  **dict(BASE, eta=5, q=0.6))
    m, s, _ = _mean_over_seeds(cfg)
    print("BS European call d=10: %.4f (seed std %.4f) vs 7.0207" % (m, s))
    assert abs(m - 7.0207) < 0.35
