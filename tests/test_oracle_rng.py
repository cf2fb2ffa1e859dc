"""Pins of the oracle's random numbers: Philox4x32-10 against its published
known-answer vectors and against rocRAND's independent implementation, the
Box-Muller normals against the normal law, and the split of U into the Euler
step j* and the fraction theta."""
import os
import shutil
import subprocess

import numpy as np
import pytest
from scipy import stats

import oracle

HERE = os.path.dirname(os.path.abspath(__file__))


# Known-answer vectors of Philox4x32-10 published with the generator
# (Salmon, Moraes, Dror, Shaw, SC'11, Random123 distribution).
KAT = [
    ((0, 0, 0, 0), (0, 0), (0x6627E8D5, 0xE169C58D, 0xBC57AC4C, 0x9B00DBD8)),
    ((0xFFFFFFFF,) * 4, (0xFFFFFFFF,) * 2,
     (0x408F276D, 0x41C83B0E, 0xA20BC7C6, 0x6D5451FD)),
    ((0x243F6A88, 0x85A308D3, 0x13198A2E, 0x03707344),
     (0xA4093822, 0x299F31D0),
     (0xD16CFE09, 0x94FDCCEB, 0x5001E420, 0x24126EA1)),
]


@pytest.mark.parametrize("ctr,key,expect", KAT)
def test_philox_known_answers(ctr, key, expect):
    assert tuple(int(x) for x in oracle.philox4x32_10(ctr, key)) == expect


def test_philox_matches_rocrand(tmp_path):
    hdr = "/opt/rocm/include/rocrand/rocrand_philox4x32_10.h"
    if not (shutil.which("g++") and os.path.exists(hdr)):
        pytest.skip("rocRAND headers or g++ not available")
    exe = str(tmp_path / "philox_rocrand")
    subprocess.check_call(["g++", "-std=c++17", "-O1", "-D__HIP_PLATFORM_AMD__",
                           "-I/opt/rocm/include",
                           os.path.join(HERE, "philox_rocrand.cpp"), "-o", exe])
    rng = np.random.default_rng(7)
    rows = []
    for _ in range(500):
        seed = int(rng.integers(0, 2 ** 63))
        c = [int(v) for v in rng.integers(0, 2 ** 32, size=4)]
        c[1] >>= 2   # rocRAND's 64-bit word offset holds 4 * (c1 << 32 | c0)
        rows.append((seed, c))
    rows.append((0, [0, 0, 0, (1 << 24) | 0]))
    inp = "\n".join("%d %d %d %d %d" % (s, *c) for s, c in rows)
    out = subprocess.run([exe], input=inp, capture_output=True, text=True,
                         check=True).stdout.split("\n")
    for (seed, c), line in zip(rows, out):
        key = (seed & 0xFFFFFFFF, seed >> 32)
        got = [int(x) for x in oracle.philox4x32_10(c, key)]
        assert got == [int(x) for x in line.split()]


def test_normals_are_standard_normal():
    # 32,000 normals from 1,000 paths x 32 normals each
    z = np.concatenate([oracle.normals(3, m, 11, 2, 0, 0, 32)
                        for m in range(1000)])
    n = len(z)
    assert abs(z.mean()) < 4 / np.sqrt(n)
    assert abs(z.var() - 1) < 4 * np.sqrt(2 / n)
    assert abs(stats.skew(z)) < 4 * np.sqrt(6 / n)
    assert abs(stats.kurtosis(z)) < 4 * np.sqrt(24 / n)
    assert stats.kstest(z, "norm").pvalue > 1e-4
    # the two members of a Box-Muller pair are uncorrelated
    pairs = z.reshape(-1, 2)
    assert abs(np.corrcoef(pairs[:, 0], pairs[:, 1])[0, 1]) < 4 / np.sqrt(len(pairs))


def test_normal_streams_differ_by_every_counter_word():
    base = oracle.normals(0, 1, 2, 3, 0, 0, 8)
    for args in [(1, 1, 2, 3, 0), (0, 2, 2, 3, 0), (0, 1, 3, 3, 0),
                 (0, 1, 2, 4, 0), (0, 1, 2, 3, 1)]:
        other = oracle.normals(*args, 0, 8)
        assert not np.allclose(base, other)
    # blocks are consecutive: normals 4..7 of block 0 == normals 0..3 of block 1
    np.testing.assert_array_equal(base[4:8], oracle.normals(0, 1, 2, 3, 0, 1, 4))


def test_uniform_time_split():
    cfg = {"d": 1, "vol_level": [0.2], "S0": [100.0], "r": 0.05, "K": 100.0,
           "T": 1.0, "n_t": 4, "n_x": 4, "eta": 2, "M": 1, "N": 50,
           "K_it": 1}
    Us = []
    for m in range(2000):
        P = oracle.path(cfg, 0.25, [4.6], 3, m, 1)
        U, js, th = P["U"], P["jstar"], P["theta"]
        assert 0 < U < 1 and 0 <= js < 50 and 0 <= th < 1
        assert abs(U * 50 - (js + th)) < 1e-12
        assert abs(P["tau"] - (0.25 + 0.75 * U)) < 1e-15
        Us.append(U)
    assert stats.kstest(Us, "uniform").pvalue > 1e-4
