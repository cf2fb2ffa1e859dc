"""The parallel driver of the oracle (used to write stored full-size
results) gives exactly the results of the serial oracle loop."""
import numpy as np

import oracle
from workloads import problem


def test_parallel_driver_is_bitwise_equal_to_serial_loop():
    cfg = problem(d=2, vol_kind="bump", vol_level=[0.2, 0.25], bump_a=0.25,
                  rho=0.3, S0=[100.0, 100.0], n_t=4, n_x=5, eta=3, M=40, N=5,
                  K_it=3, omega=100.0)
    a = oracle.solve(cfg)
    b = oracle.solve_parallel(cfg, workers=2, chunk=7)
    for key in ("alpha", "c", "var", "u"):
        np.testing.assert_array_equal(a[key], b[key])
