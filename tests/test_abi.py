"""The C ABI without a GPU: the library loads, exports every entry point
that include/bsde.h declares, and rejects invalid arguments with the
documented status codes before touching the device."""
import ctypes
import os
import re

import numpy as np
import pytest

import paper_1102_4666_amd as bsde
from workloads import problem

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "bsde.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(bsde_[a-z_]+)\s*\(", src)))


def test_every_declared_symbol_is_exported():
    lib = bsde.lib()
    names = _declared()
    assert len(names) >= 14
    for name in names:
        assert hasattr(lib, name), name
        assert isinstance(getattr(lib, name), ctypes._CFuncPtr)
    assert set(names) == set(bsde.EXPORTS)


def test_status_strings():
    lib = bsde.lib()
    for s in range(7):
        assert lib.bsde_status_string(s)


@pytest.mark.parametrize("bad,status", [
    (dict(d=0), 1), (dict(d=11), 1), (dict(M=0), 1), (dict(N=0), 1),
    (dict(K_it=0), 1), (dict(omega=-1.0), 1), (dict(n_t=1), 1),
    (dict(q=0.0), 1), (dict(q=1.5), 1), (dict(T=0.0), 1),
    (dict(d=3, rho=-0.6, vol_level=0.2, S0=100.0, eta=3), 1),
    (dict(eta=7), 6), (dict(d=4, vol_level=0.2, S0=100.0, eta=3), 6),
    (dict(n_t=2, n_x=3, eta=4), 3),  # 6 points < 15 basis functions
    # the kernel operator: bandwidth > 0, d <= 2, no redraw, no Dupire vol
    (dict(kernel_bw=-0.1), 1), (dict(kernel_bw=float("inf")), 1),
    (dict(d=3, vol_level=0.2, S0=100.0, eta=2, kernel_bw=0.3), 6),
    (dict(grid="random", redraw=1, kernel_bw=0.3), 6),
    (dict(vol_kind="dupire", kernel_bw=0.3), 6),
])
def test_invalid_arguments(bad, status):
    cfg = problem(**bad)
    with pytest.raises(bsde.BsdeError) as e:
        bsde.Problem(cfg)
    assert e.value.status == status, str(e.value)


def test_valid_problem_without_gpu_reports_device_error():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    with pytest.raises(bsde.BsdeError) as e:
        bsde.Problem(problem(eta=4))
    assert e.value.status == 4


def test_set_timing_rejects_a_null_handle():
    assert bsde.lib().bsde_set_timing(None, 1) == 1
