"""The no-allocation batched solve (bsde_solve_batch_noalloc) against the
allocating one (bsde_solve_batch): the same problems give the same
coefficients and corrections bit for bit, on two calls in a row, the second
with a smaller batch; a batch whose tables exceed the fixed workspace is
rejected with BSDE_EINVAL."""
import numpy as np
import pytest

import paper_1102_4666_amd as bsde
from workloads import problem

pytestmark = pytest.mark.gpu


def _mix(scale=1):
    return [
        problem(d=1, vol_kind="bump", bump_a=0.25, n_t=6, n_x=20, eta=4,
                M=700 * scale, N=11, K_it=3, omega=1.0, precision="fp32", seed=31),
        problem(d=2, vol_kind="bump", vol_level=[0.2, 0.3], bump_a=0.25,
                rho=0.3, S0=[100.0, 95.0], n_t=4, n_x=6, eta=3, M=260, N=6,
                K_it=4, omega=1.0, precision="fp64", seed=32),
        problem(d=5, vol_kind="bump", vol_level=[0.15, 0.2, 0.25, 0.3, 0.35],
                bump_a=0.25, rho=0.2, payoff="put_geom", S0=100.0,
                grid="random", n_t=3, n_x=40, eta=2, M=100, N=4, K_it=2,
                omega=1.0, precision="fp32", seed=33),
    ]


def _collect(P):
    K = P.cfg["K_it"]
    return (np.array([P.coefficients(k) for k in range(K + 1)]),
            np.array([P.corrections(k)[0] for k in range(K)]))


def _run(cfgs, noalloc):
    probs = [bsde.Problem(c) for c in cfgs]
    try:
        if noalloc:
            bsde.solve_batch_noalloc(probs)
        else:
            bsde.solve_batch(probs)
        return [_collect(P) for P in probs]
    finally:
        for P in probs:
            P.close()


def test_noalloc_batch_equals_allocating_batch_twice():
    first = _mix(scale=2)
    second = _mix(scale=1)[:2]          # a smaller batch next
    for cfgs in (first, second):
        print("no-allocation batch of %d problems" % len(cfgs), flush=True)
        ref = _run(cfgs, noalloc=False)
        got = _run(cfgs, noalloc=True)
        for (a_ref, c_ref), (a, c) in zip(ref, got):
            np.testing.assert_array_equal(a, a_ref)
            np.testing.assert_array_equal(c, c_ref)


def test_noalloc_rejects_tables_beyond_the_workspace():
    # about 2.4 KB of tables per problem and iteration step: 40 problems x
    # 60 iterations need more than the 4 MiB workspace
    cfgs = [problem(d=1, n_t=4, n_x=6, eta=2, M=64, N=2, K_it=60, seed=40 + j)
            for j in range(40)]
    probs = [bsde.Problem(c) for c in cfgs]
    try:
        with pytest.raises(bsde.BsdeError) as e:
            bsde.solve_batch_noalloc(probs)
        assert e.value.status == 1
        assert "workspace" in str(e.value)
    finally:
        for P in probs:
            P.close()
