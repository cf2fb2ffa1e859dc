"""Batched solves: many problems of uneven d, grid, M, N, iteration count
and precision in persistent launches (optionally one captured hipGraph)
give, problem by problem, exactly the results of solving each alone."""
import numpy as np
import pytest

import paper_1102_4666_amd as bsde
from workloads import problem

pytestmark = pytest.mark.gpu


def _mix():
    return [
        problem(d=1, vol_kind="bump", bump_a=0.25, n_t=6, n_x=20, eta=4,
                M=700, N=11, K_it=3, omega=1.0, precision="fp32", seed=3),
        problem(d=1, n_t=5, n_x=12, eta=4, M=300, N=7, K_it=2,
                precision="fp64", seed=4),
        problem(d=2, vol_kind="bump", vol_level=[0.2, 0.3], bump_a=0.25,
                rho=0.3, S0=[100.0, 95.0], n_t=4, n_x=6, eta=3, M=260, N=6,
                K_it=4, omega=100.0, precision="fp32", seed=5),
        problem(d=5, vol_kind="bump", vol_level=[0.15, 0.2, 0.25, 0.3, 0.35],
                bump_a=0.25, rho=0.2, payoff="put_geom", S0=100.0,
                grid="random", n_t=3, n_x=40, eta=2, M=100, N=4, K_it=2,
                omega=100.0, precision="fp32", seed=6),
        problem(d=1, vol_kind="bump", bump_a=0.25, n_t=6, n_x=20, eta=4,
                M=1500, N=9, K_it=3, omega=1.0, precision="fp32", seed=7),
        # the Dupire-type volatility: a kernel signature of its own
        problem(d=5, vol_kind="dupire", vol_level=0.3, div=0.1, S0=100.0,
                grid="random", n_t=3, n_x=40, eta=2, M=100, N=4, K_it=2,
                omega=1.0, precision="fp32", seed=8),
    ]


def _collect(P):
    K = P.cfg["K_it"]
    return (np.array([P.coefficients(k) for k in range(K + 1)]),
            np.array([P.corrections(k)[0] for k in range(K)]))


def _alone(cfgs, tilings):
    out = []
    for cfg, t in zip(cfgs, tilings):
        with bsde.Problem(cfg) as P:
            if t:
                P.set_tiling(*t)
            P.solve()
            out.append(_collect(P))
    return out


@pytest.mark.parametrize("graph", [False, True])
def test_batch_equals_alone(graph):
    cfgs = _mix()
    tilings = [None, (2, 1), None, None, (1, 6)]
    ref = _alone(cfgs, tilings)
    probs = [bsde.Problem(c) for c in cfgs]
    try:
        for P, t in zip(probs, tilings):
            if t:
                P.set_tiling(*t)
        for rep in range(3):            # the schedule runs several times
            for P in probs:
                P.set_coefficients(np.zeros(P.p), 0)
            ms = bsde.solve_batch(probs, graph=graph)
            assert ms > 0
            for P, (a_ref, c_ref) in zip(probs, ref):
                a, c = _collect(P)
                np.testing.assert_array_equal(a, a_ref)
                np.testing.assert_array_equal(c, c_ref)
    finally:
        for P in probs:
            P.close()


def test_batch_resumes_problems_at_different_iterations():
    cfgs = _mix()[:3]
    ref = _alone(cfgs, [None] * 3)
    probs = [bsde.Problem(c) for c in cfgs]
    try:
        # problem 0 starts from its own iteration-1 coefficients
        probs[0].set_coefficients(ref[0][0][1], 1)
        bsde.solve_batch(probs)
        for P, (a_ref, c_ref) in zip(probs, ref):
            np.testing.assert_array_equal(P.coefficients(), a_ref[-1])
    finally:
        for P in probs:
            P.close()


def test_autotune_records_tiling_for_later_problems():
    from gpu_util import run_gpu
    cfg = problem(d=1, vol_kind="bump", bump_a=0.25, n_t=5, n_x=12, eta=4,
                  M=1100, N=9, K_it=2, precision="fp32", seed=11)
    with bsde.Problem(cfg) as P:
        groups, ppl, ms = P.autotune()
    assert groups * ppl * 256 >= 1100 and ms > 0
    # problems of the same signature created afterwards start with the
    # recorded tiling: bitwise equal to setting it explicitly
    a = run_gpu(cfg)
    b = run_gpu(cfg, tiling=(groups, ppl))
    np.testing.assert_array_equal(a["c"], b["c"])
    np.testing.assert_array_equal(a["alpha"], b["alpha"])
