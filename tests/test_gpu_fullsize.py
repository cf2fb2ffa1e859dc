"""Full-size GPU parity: the benchmark workloads at their real sizes, in the
launch configuration the benchmark uses, against the stored FP64 oracle
results of tests/golden (written by tests/golden/make_golden.py, which calls
only the oracle).

Every per-point correction of every iteration is compared element by
element with the oracle's (``<name>.c.npz``).  The tolerance of point i is
scaled by the size of the path terms a_m it averages,
1 + |c_i| + sd_i with sd_i the oracle's sample standard deviation of a_m at
that point: a rounding difference in the path arithmetic is relative to the
terms summed, not to their mean, which can be small by cancellation.

Price and delta gates are those of the method's accuracy target:
|d price| <= 1e-4 max(K, |price|) and |d delta| <= 1e-4 max(1, |delta|) for
FP64 paths, 5e-4 and 5e-3 for FP32 paths.

Penalty 100 (the workloads as stated) is "Picard not converged": the
penalised driver has Lipschitz constant r + omega and the Picard map of
Section 3 contracts only when that constant times T is small (Section 5.4),
so at omega T = 100 the projected iterates grow by about an order of
magnitude per iteration.  Those cases assert the divergence of the oracle's
iterates, per-point parity of every correction, and the same price gate;
where an FP32-path price misses that gate the miss is reported as an
expected failure (the cause: FP32 rounding of each iteration's corrections
amplified by the non-contracting map) rather than hidden by a wider
tolerance."""
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


def _point_scale(c_ref, var_ref):
    return 1.0 + np.abs(c_ref) + np.sqrt(np.maximum(var_ref, 0.0))


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
    assert got["c"].shape == c_ref.shape
    for k in range(cfg["K_it"]):
        scale = _point_scale(c_ref[k], var_ref[k])
        err = np.abs(got["c"][k] - c_ref[k]) / scale
        worst = int(np.argmax(err))
        print("  k=%d max |dc_i| / (1 + |c_i| + sd_i) = %.3g at point %d "
              "(gpu %.17g oracle %.17g)" % (k, err[worst], worst,
                                             got["c"][k][worst], c_ref[k][worst]))
        assert err[worst] <= tol["c"], (k, worst, err[worst])
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
