"""The FP64 oracle under AddressSanitizer and UndefinedBehaviorSanitizer.

oracle/sanitize_main.c steps the oracle through every mode it implements
(the integral nlM law, its UCM limit, the quasi-logarithmic grid, the full
Finger tensor, the paper's coupling, the accumulated-strain damping, the
instantaneous law), a state round trip, the grid on its own and the matrix
exponential; built with -fsanitize=address,undefined and no recovery, any
out-of-bounds access, leak, use after free or undefined operation ends the
program with a non-zero status.  CPU only.
"""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ORACLE = os.path.join(os.path.dirname(HERE), "oracle")


def test_oracle_clean_under_asan_and_ubsan(tmp_path):
    if shutil.which("gcc") is None:
        pytest.skip("gcc not available")
    exe = str(tmp_path / "orc_san")
    cmd = ["gcc", "-O1", "-g", "-std=c11", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-ffp-contract=off",
           "-o", exe, os.path.join(ORACLE, "lb_oracle.c"),
           os.path.join(ORACLE, "sanitize_main.c"), "-lm"]
    build = subprocess.run(cmd, capture_output=True, text=True)
    if build.returncode != 0 and "asan" in (build.stderr or "").lower():
        pytest.skip("sanitizer runtime not available: " + build.stderr[-300:])
    assert build.returncode == 0, build.stderr
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1")
    run = subprocess.run([exe], capture_output=True, text=True, timeout=300, env=env)
    assert run.returncode == 0, run.stdout + run.stderr
    assert "all modes ok" in run.stdout
