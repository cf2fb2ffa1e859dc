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


def test_recorded_tilings_persist_by_architecture(tmp_path):
    # signatures no other test tunes (N = 13 to 16): records for this
    # device's architecture are taken by problems created after the load,
    # records of another architecture are skipped, a malformed file changes
    # nothing, and save writes back what was loaded
    from gpu_util import run_gpu

    def cfg_n(N):
        return problem(d=1, vol_kind="bump", bump_a=0.25, n_t=5, n_x=12, eta=4,
                       M=1100, N=N, K_it=2, precision="fp32", seed=11)

    # the architecture the library keys its records by: the first field of
    # a saved record
    with bsde.Problem(cfg_n(16)) as P:
        P.autotune()
    first = tmp_path / "first.txt"
    assert bsde.bsde_autotune_save(str(first)) >= 1
    rows = [ln.split() for ln in first.read_text().splitlines() if not ln.startswith("#")]
    arch = rows[0][0]
    assert arch.startswith("gfx") and all(r[0] == arch for r in rows)

    with bsde.Problem(cfg_n(13)) as P:
        n = P.n
        assert P.tiling() == (0, 0)
    size_class = int(np.ceil(np.log2(n)))

    def rec(a, N, groups, ppl):
        return "%s 1 4 10 %d %d 1100 %d %d %d %d" % (
            a, bsde.PRECISIONS["fp32"], bsde.VOL_KINDS["bump"], N, size_class, groups, ppl)

    f = tmp_path / "tilings.txt"
    f.write_text("# recorded tilings\n" + rec(arch, 13, 3, 2) + "\n" +
                 rec("gfx000", 14, 5, 1) + "\n")
    assert bsde.bsde_autotune_load(str(f)) == 1
    with bsde.Problem(cfg_n(13)) as P:
        assert P.tiling() == (3, 2)
    with bsde.Problem(cfg_n(14)) as P:
        assert P.tiling() == (0, 0)
    # the loaded tiling is the one the solve runs: bitwise equal to setting it
    a = run_gpu(cfg_n(13))
    b = run_gpu(cfg_n(13), tiling=(3, 2))
    np.testing.assert_array_equal(a["c"], b["c"])
    # a tiling that does not cover M (1 x 2 x 256 < 1100) rejects the file
    bad = tmp_path / "bad.txt"
    bad.write_text(rec(arch, 15, 4, 1) + "\n" + rec(arch, 15, 1, 2) + "\n")
    with pytest.raises(bsde.BsdeError):
        bsde.bsde_autotune_load(str(bad))
    with bsde.Problem(cfg_n(15)) as P:
        assert P.tiling() == (0, 0)
    out = tmp_path / "saved.txt"
    assert bsde.bsde_autotune_save(str(out)) >= 1
    assert rec(arch, 13, 3, 2) in out.read_text().splitlines()
