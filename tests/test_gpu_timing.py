"""Timing levels of bsde_solve: what each level measures, and that the
results do not depend on it."""
import numpy as np
import pytest

import paper_1102_4666_amd as bsde
from workloads import problem

pytestmark = pytest.mark.gpu


def _solve(cfg, level):
    with bsde.Problem(cfg) as P:
        P.set_timing(level)
        P.solve()
        price, delta = P.price_delta()
        return price[0], delta[0], P.timings()


def test_timing_levels():
    cfg = problem(d=1, vol_kind="bump", bump_a=0.25, n_t=6, n_x=24, eta=4,
                  M=512, N=12, K_it=3, omega=1.0, precision="fp32", seed=7)
    out = {lvl: _solve(cfg, lvl) for lvl in (0, 1, 2)}
    for lvl in (1, 2):
        assert out[lvl][0] == out[0][0]
        np.testing.assert_array_equal(out[lvl][1], out[0][1])
    t0, t1, t2 = out[0][2], out[1][2], out[2][2]
    assert np.all(t0[:4] == 0) and t0[4] > 0
    assert t1[0] > 0 and t1[1] > 0 and t1[2] == 0 and t1[3] == 0 and t1[4] > 0
    assert np.all(t2 > 0)
    # level 1 folds reduction, projection and update into [1]
    assert t1[0] < t1[4] and t2[0] < t2[4]
    with bsde.Problem(cfg) as P:
        with pytest.raises(bsde.BsdeError) as e:
            P.set_timing(3)
        assert e.value.status == 1
