"""The FFT twiddle table of the differential-filter path (csrc/gd_twiddle.h),
evaluated at compile time by the C++ compiler, against the C library's sin
and cos.  CPU only: the header is plain C++, compiled here with g++."""
import math
import os
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HDR_DIR = os.path.join(ROOT, "paper_1707_09177_amd", "csrc")

PROG = r"""
#include <cstdio>
#include "gd_twiddle.h"
constexpr gdtw::Table kTable = gdtw::make_table();
int main() {
    std::printf("%d\n", gdtw::kTwN);
    for (int k = 0; k < gdtw::kTwN / 2; ++k) std::printf("%.17g %.17g\n", kTable.v[k].re, kTable.v[k].im);
    return 0;
}
"""


@pytest.fixture(scope="module")
def table(tmp_path_factory):
    d = tmp_path_factory.mktemp("tw")
    src, exe = d / "tw.cpp", d / "tw"
    src.write_text(PROG)
    subprocess.check_call(["g++", "-std=c++20", "-O1", "-fconstexpr-ops-limit=1000000000", "-I", HDR_DIR,
                           str(src), "-o", str(exe)])
    out = subprocess.check_output([str(exe)], text=True).split("\n")
    n = int(out[0])
    vals = np.array([[float(t) for t in line.split()] for line in out[1:] if line.strip()])
    return n, vals


def test_table_size(table):
    n, vals = table
    assert n == 4096 and vals.shape == (n // 2, 2)


def test_table_matches_libm(table):
    # exp(-2 pi i k / N): cos and -sin of the angle.  The reference is the C
    # library's long double sin and cos (64-bit mantissa) of the angle formed
    # in long double, so its own error (~1e-19) is far below the bound; the
    # same functions in double carry the rounding of the double angle
    # 2 pi k / N (up to 4.4e-16 here), which the table's exact integer
    # reduction avoids.
    n, vals = table
    if np.finfo(np.longdouble).nmant < 60:
        pytest.skip("no extended-precision long double on this host")
    k = np.arange(n // 2, dtype=np.longdouble)
    ang = 2 * np.arccos(np.longdouble(-1)) * k / n
    want = np.stack([np.cos(ang), -np.sin(ang)], axis=1)
    assert float(np.max(np.abs(vals.astype(np.longdouble) - want))) <= 3e-16
    # and against the double-precision library functions, whose angle rounds
    dbl = np.stack([[math.cos(2.0 * math.pi * i / n) for i in range(n // 2)],
                    [-math.sin(2.0 * math.pi * i / n) for i in range(n // 2)]], axis=1)
    assert np.max(np.abs(vals - dbl)) <= 5e-16


def test_table_exact_points(table):
    # the quadrant and octant points are exact by symmetry
    n, vals = table
    assert tuple(vals[0]) == (1.0, 0.0) or tuple(vals[0]) == (1.0, -0.0)
    assert vals[n // 4][0] == 0.0 and vals[n // 4][1] == -1.0
    assert abs(vals[n // 8][0] - math.sqrt(0.5)) <= 1.2e-16 and abs(vals[n // 8][1] + math.sqrt(0.5)) <= 1.2e-16
    # unit modulus everywhere
    assert np.max(np.abs(np.hypot(vals[:, 0], vals[:, 1]) - 1.0)) <= 4e-16
