"""Throughput benchmark: lattice node-steps/s of the hybrid LB / integral
nonlinear-Maxwell step at history window N_h, with the HBM roofline of the
history kernel and the FP64 oracle timed on the host beside it.

Workload: the large 2D channel, 1024 x 512 nodes, window N_h = 4096, FP32
populations and history (Kahan sums, FP64 strain), tau = 1000, g = 5e-6,
1 % seeded velocity perturbation.  One step = the whole path for every node:
pull-stream + collide with the stress-divergence force, velocity gradient,
history push and the N_h-entry history integral.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W]
Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0   # MI355X HBM3E, 8 TB/s


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def hist_bytes_per_entry(ch) -> int:
    """Algorithmic bytes per history entry-update: the FP32 shear rate and,
    for channels that are not unidirectional, the FP32 |gamma_dot|."""
    uni = ch.lx == 1 and ch.gy == 0.0 and (ch.u0 is None)
    return 4 if uni else 8


def cpu_baseline(seconds: float = 12.0):
    """The FP64 oracle on a bounded sample of the same workload: a 16 x 512
    strip of the channel with the full 4096-entry window (seeded synthetic
    history, so every entry is live), stepped until `seconds` have passed."""
    import numpy as np
    import oracle
    import workloads

    ch = workloads.large_2d(lx=16, ly=512, n_hist=4096).channels[0]
    oc = oracle.OracleChannel(ch)
    rng = np.random.default_rng(workloads.BASE_SEED + 10)
    s, r = workloads.random_history(rng, ch.n_hist, ch.nodes, dtype=np.float64)
    st = oc.get_state()
    oc.set_state(t=2 * ch.n_hist, n=st["n"], ring_s=s, ring_r=r)
    del s, r
    steps = 0
    t0 = time.perf_counter()
    while True:
        oc.step(1)
        steps += 1
        el = time.perf_counter() - t0
        if el >= seconds:
            break
    oc.close()
    return {"value": ch.nodes * steps / el, "unit": "node-steps/s", "cores": 1,
            "kind": "oracle",
            "sample": f"16x512 strip of the 1024x512 channel, N_h=4096 full window, "
                      f"{steps} steps in {el:.1f} s, single thread"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; --gpus must be 1 "
                                   "(multi-GPU sharding is a design note only)"}))
        sys.exit(2)

    import torch
    import workloads
    from paper_1504_06123_amd import Solver, _lib

    if not os.path.exists(_lib.LIB_PATH):
        import __graft_entry__
        __graft_entry__.build()

    wl = workloads.large_2d()
    ch = wl.channels[0]
    nodes, H = ch.nodes, ch.n_hist
    log(f"bench: {wl.name} nodes={nodes} N_h={H} precision=f32")
    s = Solver(wl.channels, precision="f32", device="cuda:0")
    s.step(args.warmup)
    torch.cuda.synchronize()
    s.profile(True)  # HIP events around every launch on the solver's stream
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s.step(args.steps)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    hist_ms, hist_n = s.kernel_time(0)
    lb_ms, lb_n = s.kernel_time(1)
    s.profile(False)
    # the run must still be physical: finite, near-unit density
    rho, ux, _ = s.fields(0)
    import numpy as np
    assert np.isfinite(ux).all() and abs(rho.mean() - 1) < 1e-3
    s.close()

    node_steps = nodes * args.steps / el
    entries = nodes * H
    hist_avg_s = hist_ms / hist_n / 1e3
    alg_bytes = entries * hist_bytes_per_entry(ch)
    achieved = alg_bytes / hist_avg_s / 1e9
    log(f"bench: {args.steps} steps in {el:.3f} s; history kernel {hist_avg_s*1e3:.3f} ms avg, "
        f"lattice kernel {lb_ms/lb_n:.3f} ms avg")

    cpu = None
    if not args.no_cpu_baseline:
        log("bench: timing the FP64 oracle on the host")
        cpu = cpu_baseline(args.cpu_seconds)

    line = {
        "metric": "lattice node-steps/sec at history length N_h; achieved HBM GB/s vs peak",
        "value": node_steps,
        "unit": "node-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": el / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "large 2D channel 1024x512, N_h=4096, tau=1000 steps, "
                               "g=5e-6, 1% seeded velocity perturbation",
                   "lx": ch.lx, "ly": ch.ly, "n_hist": H, "nodes": nodes,
                   "history_entries_per_step": entries},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                     "kernel": "k_hist<float>",
                     "kernel_avg_ms": hist_avg_s * 1e3,
                     "alg_bytes_per_launch": alg_bytes},
        "entry_updates_per_s": entries * args.steps / el,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
