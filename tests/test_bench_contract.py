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


def test_issue_cycle_model():
    b = _bench()
    fp32 = b.ISSUE_CYCLES_PER_WAVE_STEP["fp32"]
    # the per-term counts of the operation-by-operation derivation
    assert fp32["normal_philox"] == pytest.approx(106 / 4)
    assert fp32["normal_box_muller"] == pytest.approx(24.0)
    assert fp32["per_path"] == pytest.approx(572 / 50)
    assert sum(fp32.values()) == pytest.approx(81.94)
    assert sum(b.ISSUE_CYCLES_PER_WAVE_STEP["fp64"].values()) == pytest.approx(655.2)
    assert b.SIMD_ISSUE_CYCLES_PEAK == pytest.approx(1024 * 2.4e9)


def test_traffic_table():
    b = _bench()
    # measured tilings report calibrated bytes; others report null
    assert b.traffic_bytes("fp32", 8) == (305 * 2.0 + 512 * 1.0) * 1024
    assert b.traffic_bytes("fp32", 3) is None
    assert b.traffic_bytes("bf16", 8) is None


def test_single_launch_overrides():
    b = _bench()
    assert b._overrides("") == {}
    assert b._overrides("eta=2,q=1.0,vol_kind=const") == {"eta": 2, "q": 1.0,
                                                          "vol_kind": "const"}
