"""Helpers for the GPU tests: run a problem through the C ABI and collect
the per-iteration corrections, the price and the deltas."""
import numpy as np

from paper_1102_4666_amd import Problem


def run_gpu(cfg, tiling=None, stream=None):
    with Problem(cfg) as P:
        if tiling:
            P.set_tiling(*tiling)
        P.solve(stream)
        out = {
            "c": np.array([P.corrections(k)[0] for k in range(cfg["K_it"])]),
            "var": np.array([P.corrections(k)[1] for k in range(cfg["K_it"])]),
            "pts": P.points(),
            "alpha": np.array([P.coefficients(k) for k in range(cfg["K_it"] + 1)]),
            "timings": P.timings(),
        }
        pr, de = P.price_delta()
        out["price"] = pr[0]
        out["delta"] = de[0]
    return out


def assert_close_c(c_gpu, c_ref, rel, what=""):
    """|c_gpu - c_ref| <= rel * (1 + |c_ref|) elementwise, with a readable
    report of the worst element."""
    err = np.abs(c_gpu - c_ref) / (1.0 + np.abs(c_ref))
    worst = np.unravel_index(np.argmax(err), err.shape)
    assert err.max() <= rel, "%s worst %s: gpu %.17g ref %.17g (scaled err %.3g)" % (
        what, worst, c_gpu[worst], c_ref[worst], err.max())
