"""No Monte Carlo path kernel spills to scratch memory (the compiler's
kernel-resource-usage report written by the build): a spill puts per-lane
scratch traffic into the innermost loops of the path simulation."""
import os

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
RES = os.path.join(ROOT, "paper_1102_4666_amd", "_build", "resources.txt")


def test_path_kernels_do_not_spill():
    if not os.path.exists(RES):
        pytest.skip("library not built in this tree")
    rows = [ln.split() for ln in open(RES) if "path_kernel" in ln]
    assert rows, "no path kernels in the resource report"
    for name, vgprs, scratch in rows:
        assert int(scratch.split("=")[1]) == 0, (name, vgprs, scratch)
