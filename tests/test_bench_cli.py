"""Command-line contract of bench.py that holds without a GPU."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused_before_any_device_work():
    res = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                         capture_output=True, text=True, timeout=120, cwd=ROOT)
    assert res.returncode == 2
    msg = json.loads(res.stdout.strip().splitlines()[-1])
    assert "--gpus must be 1" in msg["error"]


def test_counter_run_rejects_unknown_legs_before_any_device_work():
    res = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--counter-run",
                          "nonesuch"], capture_output=True, text=True, timeout=120, cwd=ROOT)
    assert res.returncode == 2
    assert "invalid choice" in res.stderr
