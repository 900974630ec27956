"""Write the stored expected values of the long parity runs.

Every number written here comes from the FP64 oracle (``oracle/``) run on the
seeded inputs of ``workloads``; nothing is read from the GPU path.  Usage:

    python tests/golden/make_golden.py NAME [NAME ...]     (or "all")

Names and the runs they store (sampled u_x, u_y, sigma_xy, N1, rho):
  startup_cessation   1 x 256, window 8192, 20000 steps on + 20000 off,
                      every 1000 steps
  large_2d_64x32      the large 2D channel recipe on a 64 x 32 grid with the
                      full window 4096, 5000 steps, every 500
  large_2d_column     one column (lx = 1, ly = 512, window 4096) of the
                      unperturbed large 2D channel, 5000 steps, every 500;
                      an x-invariant 1024 x 512 run must reproduce it in
                      every column
  batched_cheap8      the 8 batched channels of smallest ly*window, full
                      10000 steps, every 1000
  batched_all_1000    all 64 batched channels, 1000 steps, every 100
"""
from __future__ import annotations

import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import workloads  # noqa: E402


def cheap8_indices(wl):
    order = sorted(range(len(wl.channels)),
                   key=lambda i: wl.channels[i].ly * wl.channels[i].n_hist)
    return sorted(order[:8])


def runs():
    return {
        "startup_cessation": lambda: (workloads.startup_cessation(), None, None, None),
        "large_2d_64x32": lambda: (workloads.large_2d(lx=64, ly=32), None, None, None),
        "large_2d_column": lambda: (workloads.large_2d(lx=1, perturb=False), None, None, None),
        "batched_cheap8": lambda: (workloads.batched(), None, None,
                                   cheap8_indices(workloads.batched())),
        "batched_all_1000": lambda: (workloads.batched(), 1000, 100, None),
    }


def make(name):
    wl, steps, every, chans = runs()[name]()
    t0 = time.time()
    res = oracle.run_workload(wl, steps=steps, sample_every=every, channels=chans)
    idx = chans if chans is not None else list(range(len(wl.channels)))
    out = {"channels": np.array(idx), "steps": wl.steps if steps is None else steps,
           "sample_every": wl.sample_every if every is None else every,
           "steps_on": wl.steps_on}
    for j, r in enumerate(res):
        for k, v in r.items():
            out[f"c{idx[j]}_{k}"] = v
    path = os.path.join(HERE, f"{name}.npz")
    np.savez_compressed(path, **out)
    print(f"{name}: {time.time() - t0:.0f} s -> {path}", flush=True)


if __name__ == "__main__":
    names = sys.argv[1:] or ["all"]
    if names == ["all"]:
        names = list(runs())
    for n in names:
        make(n)
