"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle on
identical Philox streams, element by element on small problems that span
several workgroups and a ragged tail of paths.

Tolerances (price error relative to the strike K, dollar deltas absolute):
FP64 path: |d price| <= 1e-4 K, |d delta| <= 1e-4, per-point corrections
within 1e-8 (1 + |c|); FP32 paths with FP64 sums: |d price| <= 5e-4 K,
|d delta| <= 5e-3, per-point corrections within 2e-3 (1 + |c|)."""
import math

import numpy as np
import pytest

import oracle
import paper_1102_4666_amd as bsde
from gpu_util import assert_close_c, run_gpu
from workloads import problem

pytestmark = pytest.mark.gpu

TOL = {"fp64": dict(c=1e-8, price=1e-4, delta=1e-4),
       "fp32": dict(c=2e-3, price=5e-4, delta=5e-3)}

CASES = {
    # d = 1 European Black-Scholes put
    "eur_bs": problem(d=1, n_t=6, n_x=20, eta=4, M=300, N=7, K_it=3),
    # d = 1 American put, bump local vol, penalty 1 and 100
    "amer_bump_w1": problem(d=1, vol_kind="bump", bump_a=0.25, n_t=6,
                            n_x=20, eta=4, M=300, N=10, K_it=3, omega=1.0),
    "amer_bump_w100": problem(d=1, vol_kind="bump", bump_a=0.25, n_t=6,
                              n_x=20, eta=4, M=300, N=10, K_it=3,
                              omega=100.0),
    # d = 2 correlated arithmetic basket put with dividends
    "d2_basket": problem(d=2, vol_kind="bump", vol_level=[0.2, 0.3],
                         bump_a=0.25, rho=0.3, div=[0.0, 0.02],
                         S0=[100.0, 95.0], n_t=4, n_x=6, eta=3, M=260, N=6,
                         K_it=2, omega=1.0),
    # d = 3 call on the arithmetic mean, negative correlation
    "d3_call": problem(d=3, vol_level=[0.2, 0.25, 0.3], rho=-0.2,
                       payoff="call", S0=100.0, n_t=3, n_x=4, eta=2, M=200,
                       N=5, K_it=2),
    # d = 5 geometric put on random points
    "d5_geom": problem(d=5, vol_kind="bump", vol_level=[0.15, 0.2, 0.25, 0.3, 0.35],
                       bump_a=0.25, rho=0.2, payoff="put_geom", S0=100.0,
                       grid="random", n_t=3, n_x=40, eta=2, M=100, N=4,
                       K_it=2, omega=100.0),
    # d = 10, eta = 2 and 3 (FP32 and FP64 paths)
    "d10_eta2": problem(d=10, vol_kind="bump", vol_level=[0.15 + 0.02 * j for j in range(10)],
                        bump_a=0.25, rho=0.2, payoff="put", S0=100.0,
                        grid="random", n_t=3, n_x=70, eta=2, M=80, N=4,
                        K_it=2, omega=1.0),
    "d10_eta3": problem(d=10, vol_level=0.2, rho=0.3, payoff="call_geom",
                        S0=100.0, grid="random", n_t=4, n_x=300, eta=3,
                        M=16, N=3, K_it=2),
    # points (t, x) uniform over [0, T] x D, fixed and redrawn
    "d2_uniform": problem(d=2, vol_kind="bump", vol_level=[0.2, 0.3],
                          bump_a=0.25, rho=0.3, S0=[100.0, 100.0],
                          grid="uniform", n_x=150, eta=3, M=260, N=6,
                          K_it=2, omega=1.0),
    "d5_uniform_redraw": problem(d=5, vol_kind="bump",
                                 vol_level=[0.15, 0.2, 0.25, 0.3, 0.35],
                                 bump_a=0.25, rho=0.2, payoff="put",
                                 S0=100.0, grid="uniform", redraw=1,
                                 n_x=300, eta=3, M=100, N=4, K_it=3,
                                 omega=1.0),
    # the Dupire-type local volatility of eq. vol_locale (time-dependent)
    "d1_dupire": problem(d=1, vol_kind="dupire", vol_level=0.3, n_t=6,
                         n_x=20, eta=4, M=300, N=10, K_it=3, omega=1.0),
    "d2_dupire": problem(d=2, vol_kind="dupire", vol_level=0.3, rho=0.2,
                         S0=[100.0, 110.0], n_t=4, n_x=6, eta=3, M=260, N=6,
                         K_it=2, omega=1.0),
    "d5_dupire": problem(d=5, vol_kind="dupire", vol_level=0.3, div=0.1,
                         S0=100.0, grid="random", n_t=4, n_x=60, eta=3,
                         M=100, N=4, K_it=2, omega=1.0),
    # random points redrawn at every Picard iteration (Algorithm 1), the
    # least-squares factorisation redone on the device each time
    "d2_redraw": problem(d=2, vol_kind="bump", vol_level=[0.2, 0.3],
                         bump_a=0.25, rho=0.3, S0=[100.0, 100.0],
                         grid="random", redraw=1, n_t=4, n_x=40, eta=3,
                         M=260, N=6, K_it=3, omega=1.0),
    "d5_redraw": problem(d=5, vol_kind="bump",
                         vol_level=[0.15, 0.2, 0.25, 0.3, 0.35], bump_a=0.25,
                         rho=0.2, payoff="put_geom", S0=100.0, grid="random",
                         redraw=1, n_t=3, n_x=60, eta=2, M=100, N=4, K_it=3,
                         omega=1.0),
    # the hyperbolic index set eta = 5, q = 0.6 (p = 221) of the paper's
    # d = 10 runs, with a kernel of its own
    "d10_hyperbolic": problem(d=10, vol_kind="bump",
                              vol_level=[0.15 + 0.02 * j for j in range(10)],
                              bump_a=0.25, rho=0.2, payoff="call", S0=100.0,
                              grid="random", n_t=6, n_x=300, eta=5, q=0.6,
                              M=16, N=3, K_it=2, omega=1.0),
}
FP32_ONLY = {"d10_hyperbolic"}


@pytest.fixture(scope="module")
def oracle_results():
    return {}


def _oracle(cache, name):
    if name not in cache:
        cfg = CASES[name]
        res = oracle.solve(cfg)
        pr, de = oracle.price_delta(cfg, res["alpha"][-1], [0.0], [cfg["S0"]])
        res["price"] = pr[0]
        res["delta"] = de[0]
        # the points of the last iteration (the grid when they are fixed)
        res["pts"] = oracle.points(cfg, cfg["K_it"] - 1 if cfg.get("redraw") else 0)
        cache[name] = res
    return cache[name]


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("name", list(CASES))
def test_parity_with_oracle(name, prec, oracle_results):
    cfg = dict(CASES[name], precision=prec)
    print("parity case", name, prec, flush=True)
    if name in FP32_ONLY and prec == "fp64":
        # the hyperbolic sets of d = 10 have FP32 path kernels only: the
        # library refuses FP64 paths with BSDE_EUNSUPPORTED rather than
        # running anything else
        with pytest.raises(bsde.BsdeError) as err:
            run_gpu(cfg)
        assert err.value.status == 6, err.value
        return
    ref = _oracle(oracle_results, name)
    got = run_gpu(cfg)
    tol = TOL[prec]
    np.testing.assert_allclose(got["pts"], ref["pts"], rtol=1e-15, atol=1e-15)
    assert_close_c(got["c"], ref["c"], tol["c"], "c")
    K = cfg["K"]
    assert abs(got["price"] - ref["price"]) <= tol["price"] * K, (got["price"], ref["price"])
    np.testing.assert_allclose(got["delta"], ref["delta"], rtol=0, atol=tol["delta"])
    # sample variances of the path terms: FP64 paths to rounding (both sides
    # form them from deviations from the mean), FP32 paths to their rounding
    # of the path terms
    np.testing.assert_allclose(got["var"], ref["var"],
                               rtol=1e-9 if prec == "fp64" else 5e-2,
                               atol=1e-12 if prec == "fp64" else 1e-2)


def test_first_iteration_fp64_matches_per_point_oracle():
    # k = 0 with u^0 = 0 and omega = 0: c^0_i is the mean payoff of the
    # paths from point i (no dependence on the other points)
    cfg = problem(d=1, vol_kind="bump", bump_a=0.25, n_t=5, n_x=9, eta=4,
                  M=513, N=13, K_it=1)
    got = run_gpu(cfg)
    c_ref, v_ref = oracle.corrections(cfg, None, 0, 0, 45)
    assert_close_c(got["c"][0], c_ref, 1e-12, "c0")


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_zero_variance_on_gpu(prec):
    sig = np.array([0.2, 0.3])
    cfg = problem(d=2, r=0.0, vol_level=list(sig), rho=0.3, payoff="quad",
                  eta=3, n_t=5, n_x=6, M=256, N=7, S0=[100.0, 100.0],
                  K_it=1, precision=prec)
    from paper_1102_4666_amd import Problem
    with Problem(cfg) as P:
        pts = P.points()
        tau = 1.0 - pts[:, 0]
        C = np.array([[1, 0.3], [0.3, 1]])
        y = (pts[:, 1:] - 0.5 * sig ** 2 * tau[:, None]).sum(1) ** 2 + \
            tau * float(sig @ C @ sig)
        P.fit_values(y, 0)
        P.solve()
        c, v = P.corrections(0)
    scale = float(np.abs(y).max())
    lim = 1e-10 if prec == "fp64" else 2e-5
    assert np.abs(c).max() < lim * scale
    assert np.sqrt(v.max()) < lim * scale * 10


def test_tiling_changes_only_rounding():
    cfg = problem(d=1, vol_kind="bump", bump_a=0.25, n_t=5, n_x=10, eta=4,
                  M=700, N=9, K_it=2, omega=1.0)
    a = run_gpu(cfg, tiling=(1, 3))
    b = run_gpu(cfg, tiling=(3, 1))
    c = run_gpu(cfg, tiling=(2, 2))
    for x in (b, c):
        assert_close_c(x["c"], a["c"], 1e-12, "tiling")


def test_deterministic_and_resumable():
    cfg = problem(d=2, vol_kind="bump", vol_level=[0.2, 0.25], bump_a=0.25,
                  rho=0.1, S0=[100.0, 100.0], n_t=4, n_x=5, eta=3, M=300,
                  N=6, K_it=4, omega=1.0)
    a = run_gpu(cfg)
    b = run_gpu(cfg)
    np.testing.assert_array_equal(a["c"], b["c"])
    np.testing.assert_array_equal(a["alpha"], b["alpha"])
    from paper_1102_4666_amd import Problem
    with Problem(cfg) as P:
        P.set_coefficients(a["alpha"][2], 2)
        P.solve()
        np.testing.assert_array_equal(P.coefficients(4), a["alpha"][4])
        np.testing.assert_array_equal(P.corrections(3)[0], a["c"][3])


def test_degenerate_sizes():
    # one path per point (zero sample variance), one Euler step, and the
    # smallest tensor grid on which degree-2 polynomials are determined
    cfg = problem(d=1, n_t=3, n_x=2, eta=1, M=1, N=1, K_it=2)
    with pytest.raises(Exception):
        run_gpu(cfg)            # no kernel for eta = 1
    cfg = problem(d=1, n_t=3, n_x=3, eta=2, M=1, N=1, K_it=2)
    ref = oracle.solve(cfg)
    got = run_gpu(cfg)
    assert_close_c(got["c"], ref["c"], 1e-9, "degenerate")
    assert (got["var"] == 0).all()


@pytest.mark.parametrize("d,grid,n_x,eta", [(2, "tensor", 6, 3),
                                            (5, "random", 200, 3)])
def test_least_squares_reproduces_polynomials(d, grid, n_x, eta):
    # A polynomial of total degree <= eta lies in the span of the basis, so
    # the projection of its values on the grid (Section 3.2, the
    # least-squares operator built on the device by CholeskyQR2) gives it
    # back exactly, with its gradient, anywhere in the domain.
    from paper_1102_4666_amd import Problem
    cfg = problem(d=d, grid=grid, n_t=5, n_x=n_x, eta=eta, M=1, N=1, K_it=1,
                  rho=0.1 if d > 1 else 0.0)
    rng = np.random.default_rng(7)
    coef = rng.uniform(-1, 1, size=4)

    def f(t, x):
        y = x - math.log(100.0)
        return (1 + coef[0] * t + coef[1] * y[:, 0] * y[:, -1]
                + coef[2] * t * y[:, 0] ** 2 + coef[3] * y[:, -1] ** 3)

    def grad(t, x):
        y = x - math.log(100.0)
        g = np.zeros_like(y)
        g[:, 0] += coef[1] * y[:, -1] + 2 * coef[2] * t * y[:, 0]
        g[:, -1] += coef[1] * y[:, 0] + 3 * coef[3] * y[:, -1] ** 2
        return g

    with Problem(cfg) as P:
        pts = P.points()
        P.fit_values(f(pts[:, 0], pts[:, 1:]), 0)
        tq = rng.uniform(0.0, 1.0, size=9)
        xq = math.log(100.0) + rng.uniform(-0.3, 0.3, size=(9, d))
        price, delta = P.price_delta(tq, np.exp(xq))
    np.testing.assert_allclose(price, f(tq, xq), rtol=0, atol=1e-9)
    np.testing.assert_allclose(delta * np.exp(xq), grad(tq, xq), rtol=0,
                               atol=1e-8)


def test_rank_deficient_grids_are_rejected():
    from paper_1102_4666_amd import BsdeError, Problem
    # two spatial values cannot determine the degree-2 and 3 terms in x
    with pytest.raises(BsdeError) as e:
        Problem(problem(d=1, n_t=5, n_x=2, eta=3))
    assert e.value.status == 3, str(e.value)
    # fewer points than basis functions
    with pytest.raises(BsdeError) as e:
        Problem(problem(d=2, n_t=2, n_x=2, eta=3))
    assert e.value.status == 3, str(e.value)
    # a basis too large for the on-device factorisation (p = 84): the host
    # Cholesky applies the same test
    with pytest.raises(BsdeError) as e:
        Problem(problem(d=5, vol_level=0.2, S0=100.0, n_t=5, n_x=2, eta=3))
    assert e.value.status == 3, str(e.value)
    # both paths still accept a well-posed grid afterwards
    with Problem(problem(d=1, n_t=5, n_x=8, eta=3)) as P:
        assert P.n == 40


def test_redraw_resumes_and_is_solve_only():
    from paper_1102_4666_amd import BsdeError, Problem, Server, solve_batch
    cfg = dict(CASES["d2_redraw"], precision="fp64", K_it=4)
    a = run_gpu(cfg)
    with Problem(cfg) as P:
        np.testing.assert_allclose(P.points(), oracle.points(cfg, 0), rtol=1e-15)
        P.set_coefficients(a["alpha"][2], 2)
        P.solve()
        np.testing.assert_array_equal(P.coefficients(4), a["alpha"][4])
        np.testing.assert_array_equal(P.corrections(3)[0], a["c"][3])
        np.testing.assert_allclose(P.points(), oracle.points(cfg, 3), rtol=1e-15)
    with Problem(cfg) as P:
        with pytest.raises(BsdeError) as e:
            solve_batch([P])
        assert e.value.status == 6
    with Server(1 << 30) as S:
        with pytest.raises(BsdeError) as e:
            S.submit(cfg)
        assert e.value.status == 6
    with pytest.raises(BsdeError) as e:   # redraw needs a random grid
        Problem(dict(cfg, grid="tensor", n_x=6))
    assert e.value.status == 1


def test_hyperbolic_index_set_kernel():
    # q = 0.6 at d = 10, eta = 5 runs on a kernel of the hyperbolic set
    # itself (p = 221, eq. hyper_set); d = 2, eta = 4, q = 0.6 has none and
    # runs the total-degree kernel with the other coefficients held at zero
    from paper_1102_4666_amd import Problem
    with Problem(dict(CASES["d10_hyperbolic"], precision="fp32")) as P:
        assert P.p == len(oracle.index_set(11, 5, 0.6)) == 221
    cfg = problem(d=2, n_t=6, n_x=8, eta=4, q=0.6, M=64, N=4, K_it=2)
    with Problem(cfg) as P:
        assert P.p == 35                      # binom(3 + 4, 4)
        P.solve()
        alpha = P.coefficients()
    assert np.count_nonzero(alpha) == len(oracle.index_set(3, 4, 0.6))
