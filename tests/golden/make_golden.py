"""Write the stored expected values of the long parity runs.

Every number written here comes from the FP64 oracle (``oracle/``) run on the
seeded inputs of ``workloads``; nothing is read from the GPU path.  Usage:

    python tests/golden/make_golden.py NAME [NAME ...]     (or "all")

Names and the runs they store (sampled u_x, sigma_xy, N1; u_y and rho as
well for the 2D runs):
  startup_cessation   1 x 256, window 8192, 20000 steps on + 20000 off,
                      every 1000 steps
  large_2d_64x32      the large 2D channel recipe on a 64 x 32 grid with the
                      full window 4096, 5000 steps, every 500
  large_2d_column     one column (lx = 1, ly = 512, window 4096) of the
                      unperturbed large 2D channel, 5000 steps, every 500;
                      an x-invariant 1024 x 512 run must reproduce it in
                      every column
  startup_cessation_grid  the startup/cessation channel on the
                      quasi-logarithmic grid of Sec. III with C = 128 and
                      B = 7 (reach 16256 steps), same run and sampling
  batched_cheap8      the 8 batched channels of smallest ly*window, full
                      10000 steps, every 1000
  batched_all_1000    all 64 batched channels, 1000 steps, every 250
  large_2d_first96    the full 1024 x 512 perturbed channel (the benchmark's
                      workload) over its first 96 steps, sampled at steps 32,
                      64 and 96 on 4096 seeded nodes (u_x, u_y, rho, sigma_xy,
                      N1).  The ring starts zero-filled, so before step
                      n_hist - 1 every entry past the pushed ones is zero and
                      contributes nothing: the oracle runs it with a 128-entry
                      window, identical to the 4096-entry one up to step 126
                      (tests/test_oracle_pins.py checks this identity)
  variants_first96    the same channel, nodes and identity for the variants
                      the benchmark times beside it: the full Finger tensor,
                      the accumulated-strain damping law, the paper's coupling
                      (each with a 128-entry window, sampled at steps 32, 64
                      and 96), the instantaneous law (no history, same steps)
                      and the quasi-logarithmic grid with B = 6, C = 128
                      (steps 32 and 64; all grid blocks combine within them);
                      u_x, u_y, sigma_xy, N1
  differentiation     the 1 x 128 differentiation run: u_x samples (every 200
                      steps) at the true parameters (the target) and at the
                      evaluation point p0, the loss
                      L = sum over samples and nodes of (u_x(p0) - u_x(true))^2,
                      and dL/dp by central differences with relative step
                      1e-6 for p = (G_inf, tau, gamma_c, g_x)
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
        "startup_cessation_grid": lambda: (workloads.startup_cessation(grid=(7, 128)), None,
                                           None, None),
        "large_2d_64x32": lambda: (workloads.large_2d(lx=64, ly=32), None, None, None),
        "large_2d_column": lambda: (workloads.large_2d(lx=1, perturb=False), None, None, None),
        "batched_cheap8": lambda: (workloads.batched(), None, None,
                                   cheap8_indices(workloads.batched())),
        "batched_all_1000": lambda: (workloads.batched(), 1000, 250, None),
    }


def differentiation_fd(h_rel: float = 1e-6):
    wl = workloads.differentiation()
    ch0 = wl.channels[0]
    true = workloads.true_channel(ch0)

    def samples(ch):
        r = oracle.run_workload(workloads.Workload("d", [ch], "f64", steps_on=wl.steps_on,
                                                   sample_every=wl.sample_every))[0]
        return r["t"], r["ux"][:, :, 0]

    t, target = samples(true)
    _, u0 = samples(ch0)
    loss0 = float(np.sum((u0 - target) ** 2))
    grad = np.zeros(4)
    for i, name in enumerate(workloads.ADJOINT_PARAMS):
        p = getattr(ch0, name)
        hp = h_rel * p
        lp = float(np.sum((samples(ch0.replace(**{name: p + hp}))[1] - target) ** 2))
        lm = float(np.sum((samples(ch0.replace(**{name: p - hp}))[1] - target) ** 2))
        grad[i] = (lp - lm) / (2 * hp)
        print(f"differentiation: dL/d{name} = {grad[i]:.10e}", flush=True)
    return {"t": t, "target": target, "u_p0": u0, "loss": loss0, "grad_fd": grad,
            "params": np.array([getattr(ch0, n) for n in workloads.ADJOINT_PARAMS]),
            "h_rel": h_rel}


FIRST96_NODES = 4096
FIRST96_SAMPLES = (32, 64, 96)


def large_2d_first96():
    ch = workloads.large_2d().channels[0]
    assert max(FIRST96_SAMPLES) < 127
    rng = np.random.default_rng(workloads.BASE_SEED + 20)
    idx = np.sort(rng.choice(ch.nodes, size=FIRST96_NODES, replace=False))
    oc = oracle.OracleChannel(ch.replace(n_hist=128))
    out = {"nodes": idx, "t": np.array(FIRST96_SAMPLES), "n_hist_run": 128}
    cols = {k: [] for k in ("ux", "uy", "rho", "sxy", "n1")}
    done = 0
    for t in FIRST96_SAMPLES:
        oc.step(t - done)
        done = t
        rho, ux, uy = oc.fields()
        sxy, n1 = oc.stress()
        for k, v in (("ux", ux), ("uy", uy), ("rho", rho), ("sxy", sxy), ("n1", n1)):
            cols[k].append(v.ravel()[idx])
    oc.close()
    for k, v in cols.items():
        out[k] = np.array(v)
    return out


def _sample_full_size(ch, samples):
    """u_x, u_y, rho, sigma_xy, N1 of a full-size channel at the given steps
    on the FIRST96 nodes."""
    rng = np.random.default_rng(workloads.BASE_SEED + 20)
    idx = np.sort(rng.choice(ch.nodes, size=FIRST96_NODES, replace=False))
    oc = oracle.OracleChannel(ch)
    cols = {k: [] for k in ("ux", "uy", "rho", "sxy", "n1")}
    done = 0
    for t in samples:
        oc.step(t - done)
        done = t
        rho, ux, uy = oc.fields()
        sxy, n1 = oc.stress()
        for k, v in (("ux", ux), ("uy", uy), ("rho", rho), ("sxy", sxy), ("n1", n1)):
            cols[k].append(v.ravel()[idx])
    oc.close()
    return idx, {k: np.array(v) for k, v in cols.items()}


def variants_first96():
    base = workloads.large_2d().channels[0]
    short = base.replace(n_hist=128)
    cases = {"full_tensor": (short.replace(finger=True), FIRST96_SAMPLES),
             "strain_damping": (short.replace(law="strain_damping"), FIRST96_SAMPLES),
             "paper_coupling": (short.replace(paper_coupling=True), FIRST96_SAMPLES),
             "instantaneous": (base.replace(law="instantaneous"), FIRST96_SAMPLES),
             "grid": (base.replace(hist_blocks=6, hist_block_len=128), (32, 64))}
    out = {}
    for name, (ch, samples) in cases.items():
        t0 = time.time()
        idx, cols = _sample_full_size(ch, samples)
        out["nodes"] = idx
        out[f"{name}_t"] = np.array(samples)
        for k, v in cols.items():
            if k != "rho":
                out[f"{name}_{k}"] = v
        print(f"variants_first96: {name} {time.time() - t0:.0f} s", flush=True)
    return out


def make(name):
    if name == "variants_first96":
        t0 = time.time()
        out = variants_first96()
        path = os.path.join(HERE, f"{name}.npz")
        np.savez_compressed(path, **out)
        print(f"{name}: {time.time() - t0:.0f} s -> {path}", flush=True)
        return
    if name == "large_2d_first96":
        t0 = time.time()
        out = large_2d_first96()
        path = os.path.join(HERE, f"{name}.npz")
        np.savez_compressed(path, **out)
        print(f"{name}: {time.time() - t0:.0f} s -> {path}", flush=True)
        return
    if name == "differentiation":
        t0 = time.time()
        out = differentiation_fd()
        path = os.path.join(HERE, f"{name}.npz")
        np.savez_compressed(path, **out)
        print(f"{name}: {time.time() - t0:.0f} s -> {path}", flush=True)
        return
    wl, steps, every, chans = runs()[name]()
    t0 = time.time()
    res = oracle.run_workload(wl, steps=steps, sample_every=every, channels=chans)
    idx = chans if chans is not None else list(range(len(wl.channels)))
    out = {"channels": np.array(idx), "steps": wl.steps if steps is None else steps,
           "sample_every": wl.sample_every if every is None else every,
           "steps_on": wl.steps_on}
    keep = ("t", "ux", "sxy", "n1") + (("uy", "rho") if wl.channels[0].lx > 1 else ())
    for j, r in enumerate(res):
        for k in keep:
            out[f"c{idx[j]}_{k}"] = r[k]
    path = os.path.join(HERE, f"{name}.npz")
    np.savez_compressed(path, **out)
    print(f"{name}: {time.time() - t0:.0f} s -> {path}", flush=True)


if __name__ == "__main__":
    names = sys.argv[1:] or ["all"]
    if names == ["all"]:
        names = list(runs()) + ["large_2d_first96", "variants_first96", "differentiation"]
    for n in names:
        make(n)
