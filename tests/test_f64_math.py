"""The FP64 elementary functions of the FP64 path kernels
(paper_1102_4666_amd/csrc/bsde_f64_math.h), compiled for the host with g++
and checked against 120-bit references (mpmath): the logarithm and the
quarter-turn sine/cosine of the Box-Muller words, the square root of the
Box-Muller radius, and the exponential of non-positive arguments of the
local volatility -- the series forms and the forms from the kernels'
tables (1024 sectors of the turn, 256 powers 2^(j/256)).  The host build
refines seeds of single-precision accuracy, no better than the device's
hardware seeds.  No GPU needed."""
import os
import subprocess
import tempfile

import numpy as np
import pytest

mpmath = pytest.importorskip("mpmath")

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1102_4666_amd", "csrc")

DRIVER = r"""
#include "bsde_f64_math.h"
#include <cstdio>
int main() {
    static bsde::f64::Tables T;
    bsde::f64::fill_tables(T, 0, 1);
    char kind[8];
    while (std::scanf("%7s", kind) == 1) {
        if (kind[0] == 'l') {
            unsigned w; if (std::scanf("%u", &w) != 1) return 1;
            std::printf("%.17g\n", bsde::f64::log_word(w));
        } else if (kind[0] == 'q') {
            double x; if (std::scanf("%lf", &x) != 1) return 1;
            std::printf("%.17g\n", bsde::f64::sqrt_nonneg(x));
        } else if (kind[0] == 'X') {
            double t; if (std::scanf("%lf", &t) != 1) return 1;
            std::printf("%.17g\n", bsde::f64::exp2_neg_tab(t, T));
        } else if (kind[0] == 'E') {
            double x; if (std::scanf("%lf", &x) != 1) return 1;
            std::printf("%.17g\n", bsde::f64::exp_nonpos_tab(x, T));
        } else if (kind[0] == 'S') {
            unsigned w; if (std::scanf("%u", &w) != 1) return 1;
            double s, c; bsde::f64::sincos_turn_tab(w, T, s, c);
            std::printf("%.17g %.17g\n", s, c);
        } else if (kind[0] == 'e') {
            double x; if (std::scanf("%lf", &x) != 1) return 1;
            std::printf("%.17g\n", bsde::f64::exp_nonpos(x));
        } else {
            unsigned w; if (std::scanf("%u", &w) != 1) return 1;
            double s, c; bsde::f64::sincos_turn(w, s, c);
            std::printf("%.17g %.17g\n", s, c);
        }
    }
    return 0;
}
"""


@pytest.fixture(scope="module")
def driver():
    d = tempfile.mkdtemp()
    src = os.path.join(d, "f64.cpp")
    exe = os.path.join(d, "f64")
    with open(src, "w") as f:
        f.write(DRIVER)
    subprocess.check_call(["g++", "-O2", "-std=c++17", "-I", CSRC, src, "-o", exe])
    return exe


def _run(exe, lines):
    out = subprocess.run([exe], input="\n".join(lines), capture_output=True,
                         text=True, check=True).stdout.split("\n")
    return out[:len(lines)]


def _words():
    rng = np.random.default_rng(3)
    w = [int(x) for x in rng.integers(0, 2 ** 32, 4000, dtype=np.uint64)]
    # ends of the range, quarter-turn boundaries and the mantissa split
    # point sqrt(2) of the logarithm
    w += [0, 1, 2, 3, 2 ** 31, 2 ** 32 - 1, 2 ** 32 - 2]
    w += [q * 2 ** 29 + o for q in range(8) for o in (-1, 0, 1) if 0 <= q * 2 ** 29 + o < 2 ** 32]
    w += [int(np.sqrt(2) * 2 ** k) + o for k in range(1, 31) for o in (-1, 0, 1)]
    return w


def _ulps(got, ref):
    r = float(ref)
    return float(abs(mpmath.mpf(got) - ref)) / np.spacing(abs(r)) if r != 0 else abs(got)


def test_log_of_the_box_muller_word(driver):
    mpmath.mp.prec = 120
    ws = _words()
    out = _run(driver, ["l %d" % w for w in ws])
    worst = max(_ulps(float(v), mpmath.log((mpmath.mpf(w) + mpmath.mpf(0.5)) / 2 ** 32))
                for w, v in zip(ws, out))
    assert worst <= 2.0, worst


def test_quarter_turn_sine_and_cosine(driver):
    mpmath.mp.prec = 120
    ws = _words()
    out = _run(driver, ["s %d" % w for w in ws])
    worst = 0.0
    for w, ln in zip(ws, out):
        s, c = map(float, ln.split())
        a = 2 * mpmath.pi * (mpmath.mpf(w) + mpmath.mpf(0.5)) / 2 ** 32
        worst = max(worst, _ulps(s, mpmath.sin(a)), _ulps(c, mpmath.cos(a)))
        assert abs(s * s + c * c - 1.0) < 1e-15
    assert worst <= 2.0, worst


@pytest.mark.parametrize("form", ["s", "S"])
def test_sector_sine_and_cosine(driver, form):
    # "s": quarter turns and series; "S": 1024 sectors from the LDS table
    mpmath.mp.prec = 120
    ws = _words() + [(j * 2 ** 22 + o) % 2 ** 32 for j in range(1025)
                     for o in (-2 ** 21 - 1, -2 ** 21, -1, 0, 1, 2 ** 21 - 1)]
    out = _run(driver, ["%s %d" % (form, w) for w in ws])
    worst = 0.0
    for w, ln in zip(ws, out):
        s, c = map(float, ln.split())
        a = 2 * mpmath.pi * (mpmath.mpf(w) + mpmath.mpf(0.5)) / 2 ** 32
        worst = max(worst, _ulps(s, mpmath.sin(a)), _ulps(c, mpmath.cos(a)))
    assert worst <= 2.0, worst


@pytest.mark.parametrize("form", ["e", "E"])
def test_exp_of_non_positive_arguments(driver, form):
    mpmath.mp.prec = 120
    rng = np.random.default_rng(4)
    xs = list(-rng.uniform(0, 1, 2000) ** 2 * 40) + list(-rng.uniform(0, 708, 1000))
    xs += [0.0, -0.0, -1e-300, -1e-20, -0.3465735902799726, -0.34657359027997264,
           -707.9, -708.0]
    # half-way points of the exponential table's bins, where |r| is largest
    xs += [-(k + 0.5) * float(mpmath.log(2)) / 256 * (1 + e) for k in range(0, 4096, 37)
           for e in (-1e-15, 0.0, 1e-15)]
    out = _run(driver, ["%s %.17g" % (form, x) for x in xs])
    worst = max(_ulps(float(v), mpmath.exp(mpmath.mpf(x))) for x, v in zip(xs, out))
    assert worst <= 1.5, worst
    # below the clamp the value is e^-708, far under the volatility's rounding
    tail = _run(driver, ["%s -709" % form, "%s -1e10" % form])
    for v in tail:
        assert float(v) == pytest.approx(float(mpmath.exp(-708)), rel=1e-15)


def test_power_of_two_of_the_scaled_square(driver):
    # 2^(-t/256), t = y^2 with the FP64 bump state y = kappa (x - log c),
    # kappa^2 = 256 log2 e (the d = 10 kernels): random squares below the
    # clamp, half-integers (f = +-1/2, the largest series argument), the
    # table's period 256, and the clamp
    mpmath.mp.prec = 120
    rng = np.random.default_rng(6)
    ts = list((rng.uniform(0, 26, 2000) * 19.2) ** 2) + list(rng.uniform(0, 261485, 1000))
    ts += [0.0, 0.5, 1.5, 255.5, 256.0, 256.5, 511.49999999999994, 1e-300, 1e-12,
           261484.5, 261485.0]
    ts += [k + 0.5 * (1 + e) for k in range(0, 5000, 41) for e in (-1e-15, 0.0)]
    out = _run(driver, ["X %.17g" % t for t in ts])
    worst = max(_ulps(float(v), mpmath.power(2, -mpmath.mpf(t) / 256)) for t, v in zip(ts, out))
    assert worst <= 1.5, worst
    # beyond the clamp the value stays 2^(-261485/256), a normal number
    for v in _run(driver, ["X 261486", "X 1e12"]):
        assert float(v) == pytest.approx(float(mpmath.power(2, -mpmath.mpf(261485) / 256)),
                                         rel=1e-15)


def test_square_root_of_the_radius(driver):
    mpmath.mp.prec = 120
    rng = np.random.default_rng(5)
    # -2 v ln u for the step and bridge scales and every u: from 1e-25 to ~50,
    # plus other magnitudes and exact squares
    xs = list(10.0 ** rng.uniform(-12, 2, 3000)) + list(rng.uniform(0, 50, 1000))
    xs += [2.0 ** -899, 1e-100, 1e-25, 1e-30, 0.25, 1.0, 2.0, 4.0, 49.0, 1e30]
    out = _run(driver, ["q %.17g" % x for x in xs])
    worst = max(_ulps(float(v), mpmath.sqrt(mpmath.mpf(x))) for x, v in zip(xs, out))
    assert worst <= 1.0, worst
    assert float(_run(driver, ["q 0"])[0]) == 0.0
