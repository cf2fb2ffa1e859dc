"""Batched and served results against the FP64 oracle.

The batched entry point (persistent launches over many problems, the
schedule captured as a hipGraph) and the request server are checked here
against ``oracle.solve`` on the same Philox streams -- per-point corrections
of every iteration, price and dollar deltas -- at the accuracy target's
tolerances: FP64 paths |d price| <= 1e-4 K, |d delta| <= 1e-4, corrections
within 1e-8 (1 + |c| + sd); FP32 paths 5e-4 K, 5e-3 and 2e-3.  (The
bitwise alone-versus-batch and alone-versus-mix checks live in
test_gpu_batch.py and test_gpu_server.py.)"""
import numpy as np
import pytest

import oracle
import paper_1102_4666_amd as bsde
from workloads import problem

pytestmark = pytest.mark.gpu
GIB = 1 << 30

TOL = {"fp64": dict(c=1e-8, price=1e-4, delta=1e-4),
       "fp32": dict(c=2e-3, price=5e-4, delta=5e-3)}


def _mix(prec):
    """Problems of d = 1, 2 and 5 with different grids, M, N, iteration
    counts and penalties (0 or 1)."""
    return [
        problem(d=1, vol_kind="bump", bump_a=0.25, n_t=6, n_x=20, eta=4,
                M=700, N=11, K_it=3, omega=1.0, precision=prec, seed=21),
        problem(d=2, vol_kind="bump", vol_level=[0.2, 0.3], bump_a=0.25,
                rho=0.3, S0=[100.0, 95.0], n_t=4, n_x=6, eta=3, M=260, N=6,
                K_it=4, omega=1.0, K=97.0, precision=prec, seed=22),
        problem(d=5, vol_kind="bump", vol_level=[0.15, 0.2, 0.25, 0.3, 0.35],
                bump_a=0.25, rho=0.2, payoff="put_geom", S0=100.0,
                grid="random", n_t=3, n_x=40, eta=2, M=100, N=4, K_it=2,
                omega=1.0, precision=prec, seed=23),
        problem(d=1, n_t=5, n_x=12, eta=4, M=300, N=7, K_it=2,
                precision=prec, seed=24),
    ]


def _oracle(cfg, t=0.0, S=None):
    res = oracle.solve(cfg)
    S = cfg["S0"] if S is None else S
    pr, de = oracle.price_delta(cfg, res["alpha"][-1], [t], [S])
    return res, pr[0], de[0]


def _check(cfg, c, price, delta, ref, what):
    res, rp, rd = ref
    tol = TOL[cfg["precision"]]
    scale = 1.0 + np.abs(res["c"]) + np.sqrt(np.maximum(res["var"], 0.0))
    if c is not None:
        err = np.abs(c - res["c"]) / scale
        assert err.max() <= tol["c"], (what, float(err.max()))
    assert abs(price - rp) <= tol["price"] * cfg["K"], (what, price, rp)
    assert np.abs(np.asarray(delta) - rd).max() <= tol["delta"], (what, delta, rd)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_batch_graph_matches_oracle(prec):
    cfgs = _mix(prec)
    refs = [_oracle(c) for c in cfgs]
    probs = [bsde.Problem(c) for c in cfgs]
    try:
        for rep in range(2):            # the captured schedule, twice
            for P in probs:
                P.set_coefficients(np.zeros(P.p), 0)
            bsde.solve_batch(probs, graph=True)
            for j, (P, cfg, ref) in enumerate(zip(probs, cfgs, refs)):
                c = np.array([P.corrections(k)[0] for k in range(cfg["K_it"])])
                pr, de = P.price_delta()
                print("batch %s rep %d problem %d (d=%d): price gpu %.10g "
                      "oracle %.10g" % (prec, rep, j, cfg["d"], pr[0], ref[1]),
                      flush=True)
                _check(cfg, c, pr[0], de[0], ref, "batch problem %d" % j)
    finally:
        for P in probs:
            P.close()


def test_served_requests_match_oracle():
    # three requests of different d and precision, served together, each
    # priced at its own query point
    cfgs = [_mix("fp32")[0], _mix("fp64")[1], _mix("fp32")[2]]
    queries = [(0.0, [104.0]), (0.25, [98.0, 103.0]), (0.0, [100.0] * 5)]
    refs = [_oracle(c, t, S) for c, (t, S) in zip(cfgs, queries)]
    with bsde.Server(4 * GIB, max_inflight=8) as S:
        tickets = [S.submit(c, t, q) for c, (t, q) in zip(cfgs, queries)]
        res = [S.poll(t) for t in tickets]
    for j, (cfg, r, ref) in enumerate(zip(cfgs, res, refs)):
        assert r["status"] == 0
        print("served request %d (d=%d, %s): price gpu %.10g oracle %.10g" %
              (j, cfg["d"], cfg["precision"], r["price"], ref[1]), flush=True)
        _check(cfg, None, r["price"], r["delta"][:cfg["d"]], ref,
               "served request %d" % j)
