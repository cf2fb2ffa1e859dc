"""Pins of the oracle's set-up pieces: index sets (closed-form counts, brute
force for hyperbolic sets), grid points, Cholesky factor, least squares,
payoffs, local volatility and the derivatives of the polynomial expansion."""
import itertools
import math

import numpy as np
import pytest

import oracle
from workloads import problem


@pytest.mark.parametrize("dp,eta", [(1, 4), (2, 4), (2, 6), (3, 5), (6, 3),
                                    (11, 3)])
def test_total_degree_count_is_binomial(dp, eta):
    nu = oracle.index_set(dp, eta, 1.0)
    assert len(nu) == math.comb(dp + eta, eta)   # p = C(d' + eta, eta)
    assert len({tuple(r) for r in nu}) == len(nu)
    assert (nu.sum(1) <= eta).all() and (nu >= 0).all()
    assert (np.diff(nu.sum(1)) >= 0).all()       # graded order


@pytest.mark.parametrize("dp,eta,q", [(3, 4, 0.6), (4, 5, 0.5), (2, 6, 0.75)])
def test_hyperbolic_set_brute_force(dp, eta, q):
    got = {tuple(r) for r in oracle.index_set(dp, eta, q)}
    want = {nu for nu in itertools.product(range(eta + 1), repeat=dp)
            if sum(v ** q for v in nu) ** (1 / q) <= eta + 1e-9}
    assert got == want
    for nu in got:                               # downward closed
        for j in range(dp):
            if nu[j]:
                low = list(nu)
                low[j] -= 1
                assert tuple(low) in got


def test_tensor_grid_points():
    cfg = problem(d=2, vol_level=[0.2, 0.3], S0=[100.0, 50.0], n_t=5,
                  n_x=7, T=2.0, width=3.0)
    pts = oracle.points(cfg)
    assert pts.shape == (5 * 49, 3)
    lo, hi = oracle.domain(cfg)
    np.testing.assert_allclose(lo, np.log([100, 50]) - 3 * np.array([0.2, 0.3]) * np.sqrt(2))
    np.testing.assert_allclose(hi, np.log([100, 50]) + 3 * np.array([0.2, 0.3]) * np.sqrt(2))
    np.testing.assert_allclose(np.unique(pts[:, 0]), np.linspace(0, 2, 5))
    # time-major: point i = a * 49 + b; first asset is the fastest digit
    assert (pts[:49, 0] == 0).all() and (pts[49:98, 0] == 0.5).all()
    np.testing.assert_allclose(pts[:7, 1], np.linspace(lo[0], hi[0], 7))
    assert np.allclose(pts[:7, 2], lo[1])
    np.testing.assert_allclose(pts[0:49:7, 2], np.linspace(lo[1], hi[1], 7))


def test_random_grid_points():
    cfg = problem(d=3, vol_level=[0.2, 0.25, 0.3], S0=100.0, grid="random",
                  n_t=3, n_x=3000)
    pts = oracle.points(cfg)
    lo, hi = oracle.domain(cfg)
    assert pts.shape == (9000, 4)
    x = pts[:3000, 1:]
    assert (x > lo).all() and (x < hi).all()
    # same spatial points at every time node
    np.testing.assert_array_equal(pts[:3000, 1:], pts[6000:, 1:])
    zc = (x - (lo + hi) / 2) / ((hi - lo) / 2)
    assert np.abs(zc.mean(0)).max() < 4 * np.sqrt(1 / 3 / 3000)


def test_cholesky():
    for d, rho in [(1, 0.0), (2, 0.3), (5, 0.2), (10, -0.1)]:
        L = oracle.cholesky(d, rho)
        C = np.full((d, d), rho)
        np.fill_diagonal(C, 1)
        np.testing.assert_allclose(L @ L.T, C, atol=1e-14)
        assert np.allclose(np.triu(L, 1), 0)
    with pytest.raises(ValueError):
        oracle.cholesky(3, -0.5)  # rho must exceed -1/(d-1)


def test_lstsq_matches_numpy():
    rng = np.random.default_rng(1)
    B = rng.normal(size=(200, 17))
    y = rng.normal(size=200)
    np.testing.assert_allclose(oracle.lstsq(B, y),
                               np.linalg.lstsq(B, y, rcond=None)[0],
                               rtol=1e-11, atol=1e-12)
    Bsq = rng.normal(size=(9, 9))               # square: interpolation
    np.testing.assert_allclose(Bsq @ oracle.lstsq(Bsq, y[:9]), y[:9],
                               atol=1e-11)
    Bdef = B.copy()
    Bdef[:, 3] = Bdef[:, 5]
    with pytest.raises(np.linalg.LinAlgError):
        oracle.lstsq(Bdef, y)
    with pytest.raises(np.linalg.LinAlgError):
        oracle.lstsq(B[:10], y[:10])              # n < p


def test_payoffs_and_vol():
    x = np.log([90.0, 120.0])
    base = problem(d=2, S0=[100.0, 100.0], vol_level=[0.2, 0.2], K=100.0)
    assert oracle.payoff(dict(base, payoff="put"), x) == pytest.approx(0.0)
    assert oracle.payoff(dict(base, payoff="call"), x) == pytest.approx(5.0)
    assert oracle.payoff(dict(base, payoff="fwd"), x) == pytest.approx(5.0)
    g = math.sqrt(90 * 120)
    assert oracle.payoff(dict(base, payoff="put_geom"), x) == pytest.approx(0.0)
    assert oracle.payoff(dict(base, payoff="call_geom"), x) == pytest.approx(g - 100)
    assert oracle.payoff(dict(base, payoff="put_geom"), np.log([80.0, 90.0])) == \
        pytest.approx(100 - math.sqrt(7200))
    assert oracle.payoff(dict(base, payoff="quad"), x) == pytest.approx(x.sum() ** 2)
    bump = problem(vol_kind="bump", vol_level=0.2, bump_a=0.25, bump_c=100.0)
    assert oracle.vol(bump, 0, 0.3, math.log(100)) == pytest.approx(0.25)
    assert oracle.vol(bump, 0, 0.3, math.log(100) + 1) == pytest.approx(
        0.2 * (1 + 0.25 * math.exp(-1)))
    assert oracle.vol(bump, 0, 0.3, 20.0) == pytest.approx(0.2)


@pytest.mark.parametrize("d,eta", [(1, 6), (2, 4), (3, 3)])
def test_expansion_derivatives_match_finite_differences(d, eta):
    cfg = problem(d=d, eta=eta, vol_level=[0.2, 0.3, 0.25][:d],
                  S0=[100.0, 90.0, 110.0][:d])
    p = len(oracle.index_set(d + 1, eta))
    rng = np.random.default_rng(d)
    alpha = rng.normal(size=p)
    t = 0.37
    x = np.log(np.array([100.0, 90.0, 110.0][:d])) + rng.normal(scale=0.2, size=d)
    u, ut, ux, uxx = oracle.evaluate(cfg, alpha, t, x)
    h = 1e-5
    up = oracle.evaluate(cfg, alpha, t + h, x)[0]
    um = oracle.evaluate(cfg, alpha, t - h, x)[0]
    assert ut == pytest.approx((up - um) / (2 * h), rel=1e-6, abs=1e-6)
    for j in range(d):
        e = np.zeros(d)
        e[j] = h
        gp = oracle.evaluate(cfg, alpha, t, x + e)
        gm = oracle.evaluate(cfg, alpha, t, x - e)
        assert ux[j] == pytest.approx((gp[0] - gm[0]) / (2 * h), rel=1e-6, abs=1e-6)
        np.testing.assert_allclose(uxx[j], (gp[2] - gm[2]) / (2 * h), rtol=1e-5,
                                   atol=1e-5)
    np.testing.assert_allclose(uxx, uxx.T, rtol=1e-12, atol=1e-12)


def test_fit_reproduces_polynomial_and_its_derivatives():
    # u(t, x) = (x1 + 2 x2 - 0.3 t)^2 + t x1 lies in the span for eta >= 2
    cfg = problem(d=2, eta=3, n_t=5, n_x=5, vol_level=[0.2, 0.3],
                  S0=[100.0, 100.0])
    pts = oracle.points(cfg)
    y = (pts[:, 1] + 2 * pts[:, 2] - 0.3 * pts[:, 0]) ** 2 + pts[:, 0] * pts[:, 1]
    a = oracle.fit(cfg, y)
    t, x = 0.4, np.array([4.5, 4.7])
    u, ut, ux, uxx = oracle.evaluate(cfg, a, t, x)
    s = x[0] + 2 * x[1] - 0.3 * t
    assert u == pytest.approx(s ** 2 + t * x[0], rel=1e-11)
    assert ut == pytest.approx(-0.6 * s + x[0], rel=1e-9)
    np.testing.assert_allclose(ux, [2 * s + t, 4 * s], rtol=1e-9)
    np.testing.assert_allclose(uxx, [[2, 4], [4, 8]], rtol=1e-8)


def test_uniform_points_cover_time_and_domain():
    # Algorithm 1: n points uniform over [0, T] x D, redrawn per iteration
    from scipy import stats
    cfg = problem(d=3, vol_level=[0.2, 0.3, 0.25], grid="uniform", n_x=20000,
                  T=2.0, redraw=1)
    lo, hi = oracle.domain(cfg)
    p0 = oracle.points(cfg, 0)
    assert p0.shape == (20000, 4)
    assert stats.kstest(p0[:, 0] / 2.0, "uniform").pvalue > 1e-3
    for j in range(3):
        u = (p0[:, 1 + j] - lo[j]) / (hi[j] - lo[j])
        assert u.min() > 0 and u.max() < 1
        assert stats.kstest(u, "uniform").pvalue > 1e-3
    # coordinates of one point are independent draws
    assert abs(np.corrcoef(p0[:, 0], p0[:, 1])[0, 1]) < 0.03
    p1 = oracle.points(cfg, 1)
    assert not np.array_equal(p0, p1)
    np.testing.assert_array_equal(p0, oracle.points(dict(cfg, redraw=0), 5))
