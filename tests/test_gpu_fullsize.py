"""Full-size GPU parity: the benchmark workloads at their real sizes, in the
launch configuration the benchmark uses, against the stored FP64 oracle
results of tests/golden (written by tests/golden/make_golden.py, which calls
only the oracle).

Every per-point correction of every iteration is compared element by
element with the oracle's (``<name>.c.npz``).  The tolerance of point i is
scaled by the size of the terms the correction is computed from,
1 + |c_i| + sd_i + |u_i| with sd_i the oracle's sample standard deviation of
the path terms a_m at that point and u_i = u^k(t_i, x_i) the iterate there:
a rounding difference in the path arithmetic is relative to the terms
summed, not to their mean, which can be small by cancellation, and a
rounding-level difference of the two sides' least-squares coefficients
moves every a_m by that relative amount of u^k.  To that per-point bound
is added the least-squares solves' own rounding: a solve's backward error
is relative to the whole data vector, so u^k at any point carries an
absolute error up to about kappa(B) 2^-52 max_j |u^k_j| per solve, with
kappa(B) the condition number of the oracle's basis matrix; after k solves
(the non-contracting penalty-100 map carries earlier differences along)
the bound is 4 (k + 1) kappa(B) 2^-52 max_j |u^k_j|.  It matters only where
the iterates are large (penalty 100); at penalty 1, max |u| is about the
price.  The oracle's iterates u^k at the points are rebuilt from the stored
corrections with the oracle's own least-squares step, in the order of its
loop (the rebuilt final price must equal the stored one).

Price and delta gates are those of the method's accuracy target:
|d price| <= 1e-4 max(K, |price|) and |d delta| <= 1e-4 max(1, |delta|) for
FP64 paths, 5e-4 and 5e-3 for FP32 paths.

Penalty 100 (the workloads as stated) is "Picard not converged": the
penalised driver has Lipschitz constant r + omega and the Picard map of
Section 3 contracts only when that constant times T is small (Section 5.4),
so at omega T = 100 the projected iterates grow by about an order of
magnitude per iteration.  Those cases assert the divergence of the oracle's
iterates, per-point parity of every correction, and the same price gate.
With FP32 paths the non-contracting map amplifies each iteration's FP32
rounding by about its growth factor per iteration, so the two trajectories
part after a few iterations; there the per-point parity is that of the
iteration map itself: for every k the library is started from the oracle's
own iterate u^k (its values at the points, fitted in the library's basis)
and runs iteration k alone, and its corrections are compared with the
oracle's c^k.  FP32 paths evaluate u^k and its derivative channels as
p-term FP32 sums whose terms are of the size of the iterate, U_k = max_j
|u^k_j| (Chebyshev functions are bounded by 1 on the domain), so the map's
per-point bound adds the standard bound of such a sum, p 2^-24 U_k: it
matters only where U_k is far above the price (penalty 100, U_k up to
1e10).  Where the FP32-path price of the whole run misses the gate, the
miss is reported as an expected failure (the same amplification) rather
than hidden by a wider tolerance."""
import json
import os

import numpy as np
import pytest

from gpu_util import run_gpu

pytestmark = pytest.mark.gpu
HERE = os.path.dirname(os.path.abspath(__file__))

TOL = {"fp64": dict(c=1e-8, price=1e-4, delta=1e-4),
       "fp32": dict(c=2e-3, price=5e-4, delta=5e-3)}


def _golden(name):
    path = os.path.join(HERE, "golden", name + ".json")
    cpath = os.path.join(HERE, "golden", name + ".c.npz")
    if not (os.path.exists(path) and os.path.exists(cpath)):
        pytest.skip("stored oracle result %s not generated" % name)
    with open(path) as f:
        g = json.load(f)
    with np.load(cpath) as z:
        g["c_all"] = np.array(z["c"])
        g["var_all"] = np.array(z["var"], dtype=np.float64)
    return g


def _point_scale(c_ref, var_ref, u_ref):
    return 1.0 + np.abs(c_ref) + np.sqrt(np.maximum(var_ref, 0.0)) + np.abs(u_ref)


def _oracle_iterates(g, cfg):
    """u^k at the points of iteration k, k = 0..K_it-1, from the stored
    corrections: alpha^0 = 0, u^k = B_k alpha^k, alpha^{k+1} = argmin
    |u^k + c^k - B_k alpha| -- the oracle's loop (oracle.solve_parallel)
    with its own basis matrices and least-squares solver; and the largest
    condition number of those basis matrices."""
    import oracle
    redraw = bool(cfg.get("redraw", 0)) and cfg.get("grid") in ("random", "uniform")
    B = oracle.basis_matrix(cfg)
    kappa = np.linalg.cond(B)
    alpha = np.zeros(B.shape[1])
    us = []
    for k in range(cfg["K_it"]):
        if redraw:
            B = oracle.basis_matrix(cfg, k)
            kappa = max(kappa, np.linalg.cond(B))
        u = oracle._rowdot(B, alpha)
        us.append(u)
        alpha = oracle.lstsq(B, u + g["c_all"][k])
    pr, _ = oracle.price_delta(cfg, alpha, [0.0], [cfg["S0"]])
    ref = g["price"][-1]
    assert abs(pr[0] - ref) <= 1e-9 * max(1.0, abs(ref)), (pr[0], ref)
    return np.array(us), kappa


CASES = [
    ("eur_put_d1", "fp64"), ("eur_put_d1", "fp32"),
    ("amer_put_d1_w1", "fp64"), ("amer_put_d1_w1", "fp32"),
    ("amer_put_d1_w100", "fp64"), ("amer_put_d1_w100", "fp32"),
    ("amer_basket_d2_w1", "fp64"), ("amer_basket_d2_w1", "fp32"),
    ("amer_basket_d2_w100", "fp64"), ("amer_basket_d2_w100", "fp32"),
    ("geo_basket_d5_w1", "fp64"), ("geo_basket_d5_w1", "fp32"),
    ("geo_basket_d5_w100", "fp64"), ("geo_basket_d5_w100", "fp32"),
    # points redrawn at every iteration (Algorithm 1)
    ("geo_basket_d5_redraw_w1", "fp64"), ("geo_basket_d5_redraw_w1", "fp32"),
]


@pytest.mark.parametrize("name,prec", CASES)
def test_full_size_against_stored_oracle(name, prec):
    g = _golden(name)
    cfg = dict(g["cfg"], precision=prec)
    print("full-size case", name, prec, flush=True)
    K = cfg["K"]
    diverging = cfg["omega"] >= 100
    if diverging:
        # Picard not converged: the oracle's own iterates grow
        prices = np.abs(np.array(g["price"]))
        cmax = np.abs(g["c_all"]).max(axis=1)
        assert prices[-1] > 1e3 * K and cmax[-1] > 1e3 * cmax[0], (prices, cmax)
    got = run_gpu(cfg)
    tol = TOL[prec]
    c_ref, var_ref = g["c_all"], g["var_all"]
    u_ref, kappa = _oracle_iterates(g, dict(cfg, precision="fp64"))
    assert got["c"].shape == c_ref.shape
    c_cmp = got["c"]
    p_basis = got["alpha"].shape[1]
    if diverging and prec == "fp32":
        # parity of the iteration map: iteration k alone from the oracle's u^k
        from paper_1102_4666_amd import Problem
        c_cmp = np.empty_like(got["c"])
        for k in range(cfg["K_it"]):
            with Problem(dict(cfg, K_it=k + 1)) as P:
                P.fit_values(u_ref[k], k)
                P.solve()
                c_cmp[k] = P.corrections(k)[0]
    for k in range(cfg["K_it"]):
        U = float(np.abs(u_ref[k]).max())
        ls_abs = 4.0 * (k + 1) * kappa * 2.0 ** -52 * U
        if diverging and prec == "fp32":
            ls_abs += p_basis * 2.0 ** -24 * U
        bound = tol["c"] * _point_scale(c_ref[k], var_ref[k], u_ref[k]) + ls_abs
        diff = np.abs(c_cmp[k] - c_ref[k])
        worst = int(np.argmax(diff / bound))
        print("  k=%d max |dc_i| / bound_i = %.3g at point %d (gpu %.17g oracle %.17g; "
              "absolute term %.3g)" % (k, diff[worst] / bound[worst], worst,
                                            c_cmp[k][worst], c_ref[k][worst], ls_abs))
        assert diff[worst] <= bound[worst], (k, worst, diff[worst], bound[worst])
    big = var_ref > 1e-12 * var_ref.max()
    vrel = np.abs(got["var"] - var_ref)[big] / var_ref[big]
    print("  sample variances: max relative difference %.3g" % vrel.max())
    if prec == "fp64" and not diverging:
        # the sample variance of every point and iteration, to the
        # single-precision rounding of the stored values
        np.testing.assert_allclose(got["var"], var_ref, rtol=2e-6, atol=1e-12)
    pref, dref = g["price"][-1], np.array(g["delta"][-1])
    dp = abs(got["price"] - pref)
    dd = float(np.abs(got["delta"] - dref).max())
    print("  price gpu %.10g oracle %.10g (|d|/K %.3g); delta gpu %s oracle %s "
          "(max |d| %.3g)" % (got["price"], pref, dp / K, got["delta"], dref, dd))
    price_ok = dp <= tol["price"] * max(K, abs(pref))
    delta_ok = dd <= tol["delta"] * max(1.0, float(np.abs(dref).max()))
    if diverging and prec == "fp32" and not (price_ok and delta_ok):
        pytest.xfail("Picard not converged (omega = 100): FP32-path price gate "
                     "missed, |d price| = %.3g = %.3g max(K, |price|)"
                     % (dp, dp / max(K, abs(pref))))
    assert price_ok, (dp, pref)
    assert delta_ok, (dd, dref)
