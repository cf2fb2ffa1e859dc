"""Host-side checks of bench.py: the one-GPU guard and the roofline model's
constants (no GPU needed)."""
import importlib.util
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _bench():
    spec = importlib.util.spec_from_file_location("bench", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_issue_cycle_model_uses_measured_costs():
    b = _bench()
    c = b.ISSUE_COST
    assert (c["f32v"], c["intv"], c["four"], c["trans"]) == (3.2, 2.25, 4.1, 8.3)
    m = b.ISSUE_CYCLES_D1_FP32
    philox_block = 16 * 4.1 + 3 * 4.1 + 15 * 2.25
    assert m["normal_philox"] == pytest.approx(philox_block / 4)
    assert m["normal_box_muller"] == pytest.approx((2 * 4.1 + 4 * 8.3 + 4 * 3.2) / 2)
    assert m["local_vol"] == pytest.approx(2 * 3.2 + 8.3)
    assert b.SIMD_ISSUE_CYCLES_PEAK == pytest.approx(1024 * 2.4e9)


def test_flop_count_of_the_path_kernel():
    b = _bench()
    # index sets: binom(d + 1 + eta, eta) functions at total degree; the
    # paper's d = 10 hyperbolic set eta = 5, q = 0.6 has 221
    assert [len(b.index_set(d, e)) for d, e in ((1, 4), (5, 3), (10, 3))] == [15, 84, 364]
    assert len(b.index_set(10, 5, 0.6)) == 221
    # live entries of the channel table: all p for u, then for each of the
    # d + 1 first derivatives the functions one degree lower (binom(d + eta,
    # eta - 1) of them) and for each of the d (d + 1) / 2 second
    # derivatives those two degrees lower (binom(d - 1 + eta, eta - 2))
    from math import comb
    for d, e in ((1, 4), (2, 5), (5, 3), (10, 3)):
        p, live = b.live_channel_entries(d, e)
        assert live == p + (d + 1) * comb(d + e, e - 1) + d * (d + 1) // 2 * comb(d - 1 + e, e - 2)
    assert b.live_channel_entries(5, 3) == (84, 357)
    assert b.live_channel_entries(10, 3) == (364, 1882)
    # d = 1, eta = 4 (p = 15, C = 4, 41 live entries), N = 50, arithmetic
    # put: 16 FLOP per asset-step plus the per-path work over 50 steps
    tot, mf = b.flop_per_path_step(1, 15, 4, 41, 50, "bump", "put")
    per_path = 4 + 24 + 24 + 3 * (2 + 3 * 3) + 28 + 2 * 41 + 30 + 6 + 2 + 10 + 12
    assert tot == pytest.approx(16 + per_path / 50)
    assert mf == pytest.approx(2 * 41 / 50)
    # d = 5, eta = 3 (p = 84, C = 22), geometric put: 20 per asset-step
    tot, mf = b.flop_per_path_step(5, 84, 22, 357, 50, "bump", "put_geom")
    assert mf == pytest.approx(2 * 357 / 50)
    assert 120 < tot < 135
    # d = 10, eta = 3 (p = 364, C = 67)
    tot, mf = b.flop_per_path_step(10, 364, 67, 1882, 50, "bump", "put")
    assert mf == pytest.approx(2 * 1882 / 50)
    assert 310 < tot < 330


def test_traffic_is_null_unless_measured_for_these_sources():
    b = _bench()
    saved = b.TRAFFIC
    try:
        b.TRAFFIC = None
        assert b.traffic_bytes([1, 4]) is None
        rec = {"sources_sha16": b.kernel_sources_sha16(), "tiling": [1, 4],
               "fetch_kib": 100.0, "write_kib": 50.0}
        b.TRAFFIC = [rec, dict(rec, tiling=[4, 1], fetch_kib=300.0)]
        assert b.traffic_bytes([1, 4]) == (100.0 * 2.0 + 50.0 * 1.0) * 1024
        assert b.traffic_bytes([4, 1]) == (300.0 * 2.0 + 50.0 * 1.0) * 1024
        assert b.traffic_bytes([2, 2]) is None
        b.TRAFFIC = [dict(rec, sources_sha16="0" * 16)]
        assert b.traffic_bytes([1, 4]) is None
    finally:
        b.TRAFFIC = saved


def test_counter_figures_follow_the_recorded_profile():
    b = _bench()
    saved = b.COUNTERS
    try:
        rec = dict(saved[0], sources_sha16=b.kernel_sources_sha16(), tiling=[4, 1])
        b.COUNTERS = [rec]
        c = b.counter_figures([4, 1], 36.9)
        assert 0 < c["valu_issue"] <= 1 and 0 <= c["mfma_busy"] <= 1
        assert c["fp64_vector_tflops_issued"] == pytest.approx(
            rec["fp64_vector_flop_per_launch"] / 36.9e-3 / 1e12)
        assert b.counter_figures([2, 2], 36.9) is None
        b.COUNTERS = [dict(rec, sources_sha16="0" * 16)]
        assert b.counter_figures([4, 1], 36.9) is None
    finally:
        b.COUNTERS = saved
    # the recorded profiles are of the current kernel sources
    assert all(r["sources_sha16"] == b.kernel_sources_sha16() for r in b.COUNTERS + b.TRAFFIC)


def test_gate_labels_the_diverging_penalty():
    b = _bench()
    ok = b.gate("fp64", 6.8, [0.1], 6.8 + 5e-4, [0.1 + 5e-5], 100.0, 1.0)
    assert ok["gate_pass"] and "label" not in ok
    bad = b.gate("fp32", -5.2e8, [1.0], -5.2e8 + 77.7, [80.5], 100.0, 100.0)
    assert not bad["gate_pass"] and bad["label"] == "Picard not converged"


def test_single_launch_overrides():
    b = _bench()
    assert b._overrides("") == {}
    assert b._overrides("eta=2,q=1.0,vol_kind=const") == {"eta": 2, "q": 1.0,
                                                          "vol_kind": "const"}
