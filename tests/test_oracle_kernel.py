"""Pins of the oracle's kernel operator (Section 3.2, "A kernel operator",
the first version of the method), in its normalised form
h = sum_i y_i k_i / sum_i k_i with Gaussian k_i of bandwidth b in the mapped
coordinates z.  Checked against what the mathematics fixes: constants are
reproduced with vanishing derivatives, the derivative channels are the
derivatives of the value channel (central differences), a bandwidth far
below the point spacing interpolates the point values, and on a uniform
grid a function linear in z is reproduced exactly at interior nodes
(symmetry of the weights)."""
import numpy as np
import pytest

import oracle
from workloads import problem

pytestmark = pytest.mark.filterwarnings("ignore")


def _z_to_x(cfg, z):
    lo, hi = oracle.domain(cfg)
    return lo + (np.asarray(z) + 1.0) * (hi - lo) / 2.0


def _cfg(d, **kw):
    base = dict(d=d, vol_level=[0.2, 0.3][:d], S0=[100.0, 110.0][:d],
                rho=0.3 if d > 1 else 0.0, grid="random", n_t=5,
                n_x=40 if d > 1 else 12, eta=2, M=8, N=4, K_it=1,
                kernel_bw=0.35)
    base.update(kw)
    return problem(**base)


@pytest.mark.parametrize("d", [1, 2])
def test_constants_are_reproduced_with_zero_derivatives(d):
    cfg = _cfg(d)
    n = len(oracle.points(cfg))
    y = np.full(n, 3.7)
    rng = np.random.default_rng(1)
    for _ in range(5):
        t = rng.uniform(0.0, 1.0)
        x = _z_to_x(cfg, rng.uniform(-1.3, 1.3, d))   # also outside D
        u, ut, ux, uxx = oracle.kernel_eval(cfg, y, t, x)
        assert abs(u - 3.7) < 1e-12
        assert abs(ut) < 1e-10 and np.all(np.abs(ux) < 1e-10)
        assert np.all(np.abs(uxx) < 1e-8)


@pytest.mark.parametrize("d", [1, 2])
def test_derivative_channels_are_derivatives_of_the_value(d):
    cfg = _cfg(d)
    n = len(oracle.points(cfg))
    rng = np.random.default_rng(2)
    y = rng.normal(size=n)
    h = 1e-4
    for _ in range(4):
        t = rng.uniform(0.2, 0.8)
        x = _z_to_x(cfg, rng.uniform(-0.6, 0.6, d))
        u, ut, ux, uxx = oracle.kernel_eval(cfg, y, t, x)
        val = lambda tt, xx: oracle.kernel_eval(cfg, y, tt, xx)[0]
        fd_t = (val(t + h, x) - val(t - h, x)) / (2 * h)
        assert abs(ut - fd_t) <= 1e-5 * (1 + abs(ut))
        for j in range(d):
            e = np.zeros(d)
            e[j] = h
            fd = (val(t, x + e) - val(t, x - e)) / (2 * h)
            assert abs(ux[j] - fd) <= 1e-5 * (1 + abs(ux[j]))
            fd2 = (val(t, x + e) - 2 * u + val(t, x - e)) / h ** 2
            assert abs(uxx[j, j] - fd2) <= 2e-3 * (1 + abs(uxx[j, j]))
            for k in range(j + 1, d):
                f = np.zeros(d)
                f[k] = h
                fdm = (val(t, x + e + f) - val(t, x + e - f) - val(t, x - e + f)
                       + val(t, x - e - f)) / (4 * h * h)
                assert abs(uxx[j, k] - fdm) <= 2e-3 * (1 + abs(uxx[j, k]))
                assert uxx[j, k] == pytest.approx(uxx[k, j], rel=1e-12, abs=1e-12)


def test_small_bandwidth_interpolates_the_point_values():
    # tensor grid: z spacings 2/(n_x - 1) and 2/(n_t - 1); b a tenth of the
    # smaller one, so that a neighbour weighs e^{-50} of the node itself
    cfg = _cfg(1, grid="tensor", n_t=5, n_x=9, kernel_bw=0.025)
    pts = oracle.points(cfg)
    y = np.random.default_rng(3).normal(size=len(pts))
    for i in range(0, len(pts), 7):
        u = oracle.kernel_eval(cfg, y, pts[i, 0], pts[i, 1:])[0]
        assert abs(u - y[i]) < 1e-12


def test_linear_in_z_is_exact_at_interior_nodes_of_a_uniform_grid():
    # 101 spatial nodes (spacing 0.02 in z), b = 0.04: an interior node has
    # its neighbours placed symmetrically out to >= 20 b, so the weighted
    # mean of z_1 is z_1 of the node up to e^{-200}
    cfg = _cfg(1, grid="tensor", n_t=3, n_x=101, kernel_bw=0.04)
    pts = oracle.points(cfg)
    lo, hi = oracle.domain(cfg)
    z1 = 2.0 * (pts[:, 1] - lo[0]) / (hi[0] - lo[0]) - 1.0
    y = 2.0 + 0.5 * z1
    for node in (40, 50, 63):
        x = pts[node, 1:]
        zx = 2.0 * (x[0] - lo[0]) / (hi[0] - lo[0]) - 1.0
        u, ut, ux, uxx = oracle.kernel_eval(cfg, y, 0.5, x)
        assert abs(u - (2.0 + 0.5 * zx)) < 1e-12
        # slope: d/dx of 0.5 z_1 = 0.5 * 2/(hi - lo), curvature zero
        assert ux[0] == pytest.approx(0.5 * 2.0 / (hi[0] - lo[0]), rel=1e-9)
        assert abs(uxx[0, 0]) < 1e-8


def test_kernel_loop_starts_from_zero_and_adds_the_corrections():
    # y^0 = c^0 (u^0 = 0) and y^1 = u^1(points) + c^1 with u^1 = h[y^0]
    cfg = _cfg(1, grid="tensor", n_t=3, n_x=6, M=16, N=3, K_it=2,
               vol_kind="bump", bump_a=0.25, omega=1.0)
    res = oracle.solve(cfg)
    assert np.all(res["alpha"][0] == 0.0) and np.all(res["u"][0] == 0.0)
    np.testing.assert_array_equal(res["alpha"][1], res["c"][0])
    np.testing.assert_allclose(res["alpha"][2], res["u"][1] + res["c"][1],
                               rtol=0, atol=1e-14)
    pts = oracle.points(cfg)
    u1 = [oracle.kernel_eval(cfg, res["alpha"][1], p[0], p[1:])[0] for p in pts]
    np.testing.assert_allclose(res["u"][1], u1, rtol=0, atol=1e-13)
    # the corrections of iteration 1 use u^1 = h[y^0]
    c1, _ = oracle.corrections(cfg, res["alpha"][1], 1, 0, len(pts))
    np.testing.assert_array_equal(c1, res["c"][1])
