"""Failure detection at readouts, on the CPU: the host-side checks behind
LB_ENONFINITE and the Mach guard (paper_1504_06123_amd/csrc/lbmax_checks.h)
compiled alone with g++ and driven with planted values, and the C entry
points' handling of a NULL handle.  The GPU side (a diverging run returning
LB_ENONFINITE, a fast run raising the guard) is in test_gpu_checks.py."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1504_06123_amd", "csrc")

HARNESS = r"""
#include "lbmax_checks.h"
#include <cmath>
#include <cstdio>
#include <limits>
using namespace lbmax;
int main() {
    int bad = 0;
    const double nan = std::numeric_limits<double>::quiet_NaN();
    const double inf = std::numeric_limits<double>::infinity();
    double clean[4] = {1e-3, -2e-3, 0.0, 5e-4};
    ValueScan a = scan_values(clean, 4);
    bad += a.nonfinite != 0 || a.max_abs != 2e-3;
    double dirty[5] = {1e-3, nan, -inf, 3.0, inf};
    ValueScan b = scan_values(dirty, 5);
    bad += b.nonfinite != 3 || b.max_abs != 3.0;
    bad += scan_values(dirty, 1).nonfinite != 0;   // only the first entry
    double ux[3] = {0.05, -0.08, 0.06}, uy[3] = {0.0, 0.06, -0.05};
    // |u| = 0.05, 0.1, 0.078: exactly at the guard does not trip it
    bad += std::fabs(max_speed(ux, uy, 3) - 0.1) > 1e-15;
    bad += mach_guard_trips(max_speed(ux, uy, 3));
    uy[1] = 0.0601;
    bad += !mach_guard_trips(max_speed(ux, uy, 3));
    double ux2[2] = {0.01, nan};
    bad += !mach_guard_trips(max_speed(ux2, nullptr, 2));   // a NaN speed trips it
    bad += mach_guard_trips(max_speed(ux2, nullptr, 1));
    std::printf(bad ? "FAILED %d\n" : "checks ok\n", bad);
    return bad;
}
"""


def test_readout_checks_on_planted_values(tmp_path):
    if shutil.which("g++") is None:
        pytest.skip("g++ not available")
    src = tmp_path / "harness.cpp"
    src.write_text(HARNESS)
    exe = str(tmp_path / "harness")
    build = subprocess.run(["g++", "-std=c++17", "-O1", "-Wall", "-Werror", "-I", CSRC,
                            "-o", exe, str(src)], capture_output=True, text=True)
    assert build.returncode == 0, build.stderr
    run = subprocess.run([exe], capture_output=True, text=True, timeout=60)
    assert run.returncode == 0 and "checks ok" in run.stdout, run.stdout + run.stderr


def test_check_entry_points_with_null_handle():
    from paper_1504_06123_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        from paper_1504_06123_amd import build
        build.build()
    lib = _lib.load()
    assert lib.lb_set_checks(None, _lib.LB_CHECK_FINITE) == _lib.LB_EINVAL
    assert lib.lb_warnings(None) == 0
