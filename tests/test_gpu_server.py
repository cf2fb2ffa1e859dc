"""The request server: continuous batching, admission by device memory,
and results that are the same whether a request runs alone or in a mix."""
import threading
import time

import numpy as np
import pytest

import paper_1102_4666_amd as bsde
from workloads import problem

pytestmark = pytest.mark.gpu
GIB = 1 << 30


def _requests():
    out = []
    for j in range(10):
        if j % 3 == 0:
            cfg = problem(d=1, vol_kind="bump", bump_a=0.25, n_t=6, n_x=20,
                          eta=4, M=300 + 100 * j, N=10, K_it=2 + j % 3,
                          omega=float(j % 2), K=90.0 + 3 * j,
                          precision="fp32", seed=100 + j)
        elif j % 3 == 1:
            cfg = problem(d=2, vol_kind="bump", vol_level=[0.2, 0.3],
                          bump_a=0.25, rho=0.3, S0=[100.0, 100.0], n_t=4,
                          n_x=6, eta=3, M=256, N=6, K_it=3, K=95.0 + j,
                          precision="fp32", seed=100 + j)
        else:
            cfg = problem(d=5, vol_kind="bump",
                          vol_level=[0.15, 0.2, 0.25, 0.3, 0.35], bump_a=0.25,
                          rho=0.2, payoff="put_geom", S0=100.0, grid="random",
                          n_t=3, n_x=40, eta=2, M=128, N=4, K_it=2,
                          omega=1.0, precision="fp64", seed=100 + j)
        out.append(cfg)
    return out


def test_alone_equals_mix_equals_plain_solve():
    reqs = _requests()
    probe = 4
    with bsde.Server(4 * GIB) as S:
        alone = S.poll(S.submit(reqs[probe], 0.0, [105.0] * reqs[probe]["d"]))
    assert alone["status"] == 0
    with bsde.Problem(reqs[probe]) as P:
        P.solve()
        pr, de = P.price_delta(0.0, [105.0] * reqs[probe]["d"])
    assert alone["price"] == pr[0]
    np.testing.assert_array_equal(alone["delta"][:reqs[probe]["d"]], de[0])

    with bsde.Server(4 * GIB, max_inflight=6) as S:
        tickets = {}
        for j, cfg in enumerate(reqs):          # staggered arrivals
            tickets[j] = S.submit(cfg, 0.0, [105.0] * cfg["d"])
            time.sleep(0.002 * (j % 3))
        res = {j: S.poll(t) for j, t in tickets.items()}
        st = S.stats()
    assert all(r["status"] == 0 for r in res.values())
    assert res[probe]["price"] == alone["price"]
    np.testing.assert_array_equal(res[probe]["delta"], alone["delta"])
    assert st["completed"] == len(reqs) and st["p99_ms"] >= st["p50_ms"] > 0


def test_arrivals_join_a_running_batch():
    # a long request is on the GPU when short ones arrive: they join its
    # engine steps and finish first (continuous batching, not a queue)
    long_cfg = problem(d=1, vol_kind="bump", bump_a=0.25, n_t=16, n_x=128,
                       eta=4, M=4000, N=200, K_it=30, omega=1.0,
                       precision="fp32", seed=900)
    short = _requests()[:6]
    with bsde.Server(4 * GIB) as S:
        t_long = S.submit(long_cfg)
        time.sleep(0.01)
        t_short = [S.submit(c) for c in short]
        r_short = [S.poll(t) for t in t_short]
        r_long = S.poll(t_long)
        st = S.stats()
    assert r_long["status"] == 0 and all(r["status"] == 0 for r in r_short)
    assert max(r["latency_ms"] for r in r_short) < r_long["latency_ms"]
    assert st["engine_steps"] < long_cfg["K_it"] + sum(c["K_it"] for c in short)


def test_admission_by_device_memory():
    reqs = _requests()[:6]
    # a budget of ~1 MiB admits one small problem at a time
    with bsde.Server(1 << 20, max_inflight=64) as S:
        tickets = [S.submit(c) for c in reqs]
        res = [S.poll(t) for t in tickets]
        st = S.stats()
    assert all(r["status"] == 0 for r in res)
    assert st["reserved_bytes"] == 0 and st["in_flight"] == 0
    with bsde.Server(4 * GIB) as S:
        ref = [S.poll(S.submit(c)) for c in reqs]
    for a, b in zip(res, ref):
        assert a["price"] == b["price"]


def test_unsupported_and_concurrent_clients():
    good = _requests()[0]
    bad = problem(d=4, vol_level=0.2, S0=100.0, eta=3)   # no kernel for d=4
    with bsde.Server(4 * GIB) as S:
        assert S.poll(S.submit(bad))["status"] == 6
        results = []

        def client(k):
            results.append(S.poll(S.submit(dict(good, seed=500 + k))))
        threads = [threading.Thread(target=client, args=(k,)) for k in range(4)]
        for t in threads:
            t.start()
        for t in threads:
            t.join()
        assert len(results) == 4 and all(r["status"] == 0 for r in results)
        t = S.submit(good)
        r = S.poll(t, wait=False)
        assert r is None or r["status"] == 0
        if r is None:
            assert S.poll(t)["status"] == 0


def test_cheap_requests_chain_iterations_beside_a_heavy_one():
    # an engine step lasts about one iteration of the heaviest problem, so
    # a cheap request in flight beside it runs several of its iterations
    # per step -- and its result is still the one it gets alone
    heavy = problem(d=1, vol_kind="bump", bump_a=0.25, n_t=16, n_x=128,
                    eta=4, M=4000, N=200, K_it=40, omega=1.0,
                    precision="fp32", seed=901)   # ~2 ms per iteration
    cheap = problem(d=1, vol_kind="bump", bump_a=0.25, n_t=6, n_x=20, eta=4,
                    M=256, N=10, K_it=8, omega=1.0, precision="fp32",
                    seed=902)
    with bsde.Server(4 * GIB) as S:
        alone = S.poll(S.submit(cheap))
    with bsde.Server(4 * GIB) as S:
        th = S.submit(heavy)
        time.sleep(0.02)        # the heavy request is on the GPU by now
        tc = S.submit(cheap)
        rc, rh = S.poll(tc), S.poll(th)
    assert rh["status"] == 0 and rc["status"] == 0
    assert rh["engine_steps"] == heavy["K_it"]
    assert rc["engine_steps"] <= 2, rc["engine_steps"]
    assert rc["price"] == alone["price"]
    np.testing.assert_array_equal(rc["delta"], alone["delta"])


def test_light_requests_do_not_wait_for_heavy_steps():
    # iterations of a few milliseconds go to the light engine lane, so a
    # cheap request arriving beside a heavy problem (d = 5, ~10 ms per
    # iteration) finishes long before it, with the result it gets alone
    heavy = problem(d=5, vol_kind="bump", vol_level=[0.15, 0.2, 0.25, 0.3, 0.35],
                    bump_a=0.25, rho=0.2, payoff="put_geom", S0=100.0,
                    grid="random", n_t=10, n_x=4096, eta=3, M=1000, N=50,
                    K_it=10, omega=1.0, precision="fp32", seed=903)
    cheap = problem(d=1, vol_kind="bump", bump_a=0.25, n_t=6, n_x=20, eta=4,
                    M=256, N=10, K_it=8, omega=1.0, precision="fp32", seed=904)
    with bsde.Server(4 * GIB) as S:
        alone = S.poll(S.submit(cheap))
    with bsde.Server(4 * GIB) as S:
        th = S.submit(heavy)
        time.sleep(0.03)        # the heavy request is on the GPU by now
        tc = S.submit(cheap)
        rc, rh = S.poll(tc), S.poll(th)
    assert rh["status"] == 0 and rc["status"] == 0
    assert rc["latency_ms"] < 0.5 * rh["latency_ms"], (rc["latency_ms"], rh["latency_ms"])
    assert rc["price"] == alone["price"]
    np.testing.assert_array_equal(rc["delta"], alone["delta"])
