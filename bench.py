"""Throughput benchmark: lattice node-steps/s of the hybrid LB / integral
nonlinear-Maxwell step at history window N_h, with the roofline of the
history kernel and the FP64 oracle timed on the host beside it.

Workload: the large 2D channel, 1024 x 512 nodes, window N_h = 4096, tau =
1000, g = 5e-6, 1 % seeded velocity perturbation.  Precision of the headline
number: FP32 populations in split storage (FP32 remainders against the
equilibrium of FP64 moments), FP32 history ring whose window sums are FP32
partial sums added into Kahan-compensated FP32 totals, FP64 accumulated
strain; the mode with FP64 populations is timed beside it.  One step = the whole path for every node:
pull-stream + collide with the stress-divergence force, velocity gradient,
history push and the N_h-entry history integral.  The launch shape (steps
per history pass, lanes, chunks, persistent pass) is chosen by the
autotuner before the timed region.  The timed region is sustained: the
workload's own run length (5000 steps) rounded up to whole blocks, or
--steps if that is longer; the first block alone is reported beside it.

Beside it ("grid"): the same channel on the quasi-logarithmic history grid
of Sec. III; ("full_tensor"): the same channel with the full Finger tensor
instead of its simple-shear reduction; ("laws"): the same channel with the
accumulated-strain damping variant and with the instantaneous law; and
("batched"): the 64-channel batched workload (uneven widths and
windows, FP32, one launch per phase) against the plain per-channel FP64
path (one handle per channel, no blocking, no graphs) on the same GPU.

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

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E
# MI355X published FP32 vector peak: 256 CUs x 4 SIMDs x 64 flops per cycle x
# 2.4 GHz.  (The library is built without packed FP32 instructions; a plain FP32
# FMA loop still issues a wave64 FMA every 2.4 to 3.3 cycles per SIMD with 8 to 2
# waves per SIMD, so this peak, not half of it, bounds the vector arithmetic.)
FP32_PEAK_TFLOPS = 157.3
# the large 2D channel's own run length
LARGE_2D_RUN_STEPS = 5000
# replay length of the step graphs the legs use or tune over; --no-graphs sets it to 0
GRAPH_LEN = 64

KERNEL_SOURCE = os.path.join(ROOT, "paper_1504_06123_amd", "csrc", "lbmax_kernels.hip")
# rocprofv3 counter results for the history pass on this workload (see
# profiles/history_pass_large_2d_1024x512_nh4096.md), keyed by
# (precision, steps per pass, nodes per lane).  Valid only for the kernel source they
# were taken from; otherwise reported as null.
MEASURED = {
    "source_sha256": "4420735c938cc4f3a0b522dceeec0453bbaa654f000d4af98829c3c55b44b196",
    # HBM bytes per launch: FETCH_SIZE x 2.000 + WRITE_SIZE x 1.000 (copy-calibrated),
    # from `bench.py --counter-run <leg>` under rocprofv3 --pmc
    "traffic_bytes": {("f32", 32, 1): 8395456.6 * 1024 * 2 + 266560.0 * 1024,
                      ("f32", 1, 4): 8411893.1 * 1024 * 2 + 41231.2 * 1024,
                      ("f32p64", 32, 1): 8394923.6 * 1024 * 2 + 266560.0 * 1024,
                      ("f32p64", 1, 4): 8411801.9 * 1024 * 2 + 41233.6 * 1024},
    # SQ_INSTS_VALU x 64 / history entries (both modes run the same pass kernels)
    "valu_instr_per_entry": {("f32", 32, 1): 90.77, ("f32p64", 32, 1): 90.77,
                             ("f32", 1, 4): 9.53, ("f32p64", 1, 4): 9.53},
    # the side legs' dominant kernels, keyed by (leg, steps per pass), same calibration
    "leg_traffic_bytes": {("grid", 16): 1602534.0 * 1024 * 2 + 211968.0 * 1024,
                          ("full_tensor", 16): 33557838.6 * 1024 * 2 + 213072.0 * 1024,
                          ("strain_damping", 32): 8395973.2 * 1024 * 2 + 266240.0 * 1024},
}


def measured(kind: str, key):
    import hashlib
    with open(KERNEL_SOURCE, "rb") as f:
        if hashlib.sha256(f.read()).hexdigest() != MEASURED["source_sha256"]:
            return None
    return MEASURED[kind].get(key)


def graph_lens():
    """Graph replay lengths the autotuner tries (0: plain launches)."""
    return (0, GRAPH_LEN) if GRAPH_LEN else (0,)


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def unidirectional(ch) -> bool:
    return ch.lx == 1 and ch.gy == 0.0 and ch.u0 is None


def hist_bytes_per_entry(ch) -> int:
    """Algorithmic bytes per history entry read by a pass: the FP32 shear
    rate and, unless the channel is unidirectional, the FP32 |gamma_dot|."""
    return 4 if unidirectional(ch) else 8


def pass_flops_per_entry(block: int) -> int:
    """Algorithmic FP32 operations per history entry of one pass serving
    `block` steps: decay rate (fma 2), exponent (1), two exponentials (2),
    s*E (1), FP64 strain add (1), 2*strain (1); per step of the block: decay
    factor (1), sigma_xy add (1), sigma_xx fma (2)."""
    return 8 + 4 * block


def time_steps(solver, steps: int):
    """Per-kernel times from `steps` plain launches bracketed by HIP events,
    then the wall time of `steps` more in the configured launch (graph replay
    included; event timing turns graphs off)."""
    import torch
    torch.cuda.synchronize()
    solver.profile(True)
    solver.step(steps)
    kt = {w: solver.kernel_time(w) for w in (0, 1, 2)}
    solver.profile(False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    solver.step(steps)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    return el, kt


def bench_large_2d(wl, args, precision: str):
    """Tune and time the large 2D channel in one precision; roofline of the
    history pass."""
    import numpy as np
    import torch
    from paper_1504_06123_amd import Solver, autotune

    ch = wl.channels[0]
    nodes, H = ch.nodes, ch.n_hist
    log(f"bench: {wl.name} nodes={nodes} N_h={H} precision={precision}")
    s = Solver(wl.channels, precision=precision, device="cuda:0")
    s.step(args.warmup)
    # The pass in the default launch shape, one window reduction per step (no
    # temporal blocking): the HBM-bound form of the history kernel, timed with
    # HIP events over 8 steps (its time includes the chunk combine).
    one_step = None
    if s.block == 1:
        s.profile(True)
        s.step(8)
        ms1, n1 = s.kernel_time(0)
        s.profile(False)
        vec1 = s.tiling(0)[1]
        one_s = ms1 / n1 / 1e3
        gbs1 = ch.nodes * ch.n_hist * hist_bytes_per_entry(ch) / one_s / 1e9
        one_step = {"bound": "hbm", "achieved": gbs1, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": gbs1 / HBM_PEAK_GBS,
                    "traffic": measured("traffic_bytes", (precision, 1, vec1)),
                    "kernel": f"k_hist_pass (one step per pass, {vec1} nodes per lane, "
                              f"{s.tiling(0)[0]} age chunks; with the chunk combine)",
                    "kernel_avg_ms": one_s * 1e3}
        log(f"bench: {precision}: one-step pass {one_s*1e3:.3f} ms ({gbs1:.0f} GB/s)")
    if args.no_tune:
        cfg = dict(block=args.block, vec=1, chunk_len=1 << 30, persistent=args.persistent,
                   graph=args.graph if GRAPH_LEN else 0)
        autotune.apply(s, cfg)
    else:
        best = autotune.tune(s, autotune.candidates(s, blocks=(1, 8, 16, 32),
                                                    chunk_lens=(1024, 1 << 30),
                                                    graphs=graph_lens()),
                             min_steps=64)
        cfg = {k: best[k] for k in ("block", "vec", "chunk_len", "persistent", "graph")}
        log(f"bench: tuned {cfg} ({best['ms_per_step']:.4f} ms/step in tuning)")
    M = cfg["block"]
    # sustained: the run length rounded up to whole blocks (or --steps if longer)
    steps = -(-max(args.steps, LARGE_2D_RUN_STEPS) // M) * M
    s.step(2 * M)
    # one block alone, in the tuned launch
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s.step(M)
    torch.cuda.synchronize()
    burst_s = time.perf_counter() - t0
    el, kt = time_steps(s, steps)
    rho, ux, _ = s.fields(0)
    assert np.isfinite(ux).all() and abs(rho.mean() - 1) < 1e-3
    s.close()
    del s
    torch.cuda.empty_cache()

    pass_ms, n_pass = kt[0]
    pass_s = pass_ms / n_pass / 1e3
    entries = nodes * H
    alg_bytes = entries * hist_bytes_per_entry(ch)
    alg_flops = entries * pass_flops_per_entry(M)
    gbs = alg_bytes / pass_s / 1e9
    tflops = alg_flops / pass_s / 1e12
    hbm_frac = gbs / HBM_PEAK_GBS
    log(f"bench: {precision}: {steps} steps in {el:.3f} s ({el/steps*1e3:.4f} ms/step); "
        f"history pass {pass_s*1e3:.3f} ms x {n_pass} ({gbs:.0f} GB/s, {tflops:.1f} TFLOP/s); "
        f"lattice {kt[1][0]/max(kt[1][1],1):.4f} ms; block step "
        f"{(kt[2][0]/kt[2][1]) if kt[2][1] else 0:.4f} ms")
    key = (precision, M, cfg["vec"])
    traffic = measured("traffic_bytes", key)
    vpe = measured("valu_instr_per_entry", key)
    vpe_src = "rocprofv3 SQ_INSTS_VALU" if vpe else "model"
    if not vpe:
        # Instruction model.  M >= 16: one FMA (or add) per sum and step plus
        # the seven low and 2 M/8 high powers and the per-entry decay, strain
        # and compensated-total work (the counted 32-step pass has 91).  Shorter
        # blocks carry the decay factor along the steps: three instructions per
        # step.
        vpe = 2.25 * M + 19 if M >= 16 else 3.5 * M + 10
    # Cycles each SIMD spends per wave-level VALU instruction, counted at the
    # nominal 2.4 GHz engine clock.  Under this load the engine runs below
    # 2.4 GHz (rocprofv3 GRBM_GUI_ACTIVE counts about 3.7 real cycles per
    # instruction for the 32-step pass, which holds 2 waves per SIMD).
    wave_instr = vpe * entries / 64
    cycles_per_instr = 1024 * 2.4e9 * pass_s / wave_instr
    # The binding published roof: the longer of the algorithmic bytes at the
    # HBM peak and the algorithmic FP32 operations at the FP32 peak.
    hbm_bound = alg_bytes / (HBM_PEAK_GBS * 1e9) >= alg_flops / (FP32_PEAK_TFLOPS * 1e12)
    if hbm_bound:
        roof = {"bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": hbm_frac}
    else:
        roof = {"bound": "alu", "achieved": tflops, "peak": FP32_PEAK_TFLOPS,
                "unit": "TFLOP/s", "frac": tflops / FP32_PEAK_TFLOPS}
    roof.update({"traffic": traffic,
                 "kernel": f"k_hist_pass ({precision}, {M} steps per pass)",
                 "kernel_avg_ms": pass_s * 1e3, "alg_bytes_per_launch": alg_bytes,
                 "alg_flops_per_launch": alg_flops, "hbm_GBs": gbs, "hbm_frac": hbm_frac,
                 "fp32_TFLOPs": tflops, "fp32_frac": tflops / FP32_PEAK_TFLOPS,
                 "valu_instr_per_entry": vpe, "valu_instr_source": vpe_src,
                 "valu_cycles_per_instr_at_2p4ghz": cycles_per_instr})
    return {"el": el, "steps": steps, "cfg": cfg, "roof": roof, "one_step": one_step,
            "node_steps_per_s": nodes * steps / el, "ms_per_step": el / steps * 1e3,
            "burst": {"steps": M, "ms_per_step": burst_s / M * 1e3,
                      "value": nodes * M / burst_s}}


def oracle_strip(seconds: float, seed_offset: int = 10):
    """Step the FP64 oracle on a 16 x 512 strip of the channel with the full
    4096-entry window (seeded synthetic history, so every entry is live) until
    `seconds` have passed; returns (node-steps, seconds, steps)."""
    import numpy as np
    import oracle
    import workloads

    ch = workloads.large_2d(lx=16, ly=512, n_hist=4096).channels[0]
    oc = oracle.OracleChannel(ch)
    rng = np.random.default_rng(workloads.BASE_SEED + seed_offset)
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
    return ch.nodes * steps, el, steps


def _cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(seconds: float = 12.0, max_procs: int = 16):
    """The FP64 oracle on a bounded sample of the same workload: one 16 x 512
    strip in this process (single thread: `value`), then one strip per host
    core in worker processes, each its own seeded strip (`all_cores`; at most
    16 workers, the CPU share of one GPU)."""
    import multiprocessing as mp

    ns, el, steps = oracle_strip(seconds)
    out = {"value": ns / el, "unit": "node-steps/s", "cores": 1, "kind": "oracle",
           "sample": f"16x512 strip of the 1024x512 channel, N_h=4096 full window, "
                     f"{steps} steps in {el:.1f} s, single thread",
           "cpu_model": _cpu_model(), "host_cores": os.cpu_count()}
    procs = max(1, min(max_procs, len(os.sched_getaffinity(0))))
    if procs > 1:
        # fresh interpreters (spawn): the workers touch no GPU state
        with mp.get_context("spawn").Pool(procs) as pool:
            res = pool.starmap(oracle_strip, [(seconds, 10 + i) for i in range(procs)])
        rate = sum(n / e for n, e, _ in res)
        out["all_cores"] = {"value": rate, "unit": "node-steps/s", "cores": procs,
                            "sample": f"{procs} processes, one 16x512 strip each, "
                                      f"{sum(r[2] for r in res)} steps in total"}
    return out


def bench_grid(steps: int = 256, B: int = 6, C: int = 128, block: int = 16):
    """The large 2D channel on the quasi-logarithmic history grid of Sec. III
    (B blocks of C entries; reach C (2^B - 1) = 8064 steps), FP64 lattice and
    FP32 history, `block` steps per grid pass, 64-step graphs."""
    import torch
    import workloads
    from paper_1504_06123_amd import Solver

    ch = workloads.large_2d().channels[0].replace(hist_blocks=B, hist_block_len=C)
    s = Solver([ch], precision="f32p64")
    s.set_block(block)
    s.set_graph(GRAPH_LEN)
    s.step(2 * C)
    el, kt = time_steps(s, steps)
    s.close()
    del s
    torch.cuda.empty_cache()
    pass_s = kt[0][0] / kt[0][1] / 1e3
    edge_s = kt[2][0] / kt[2][1] / 1e3 if kt[2][1] else 0.0
    # each grid block alternates between C - 1 and C live entries; the pass
    # reads every live entry once, 8 B each (FP32 averaged shear rate + FP32
    # |gamma_dot|)
    alg_bytes = ch.nodes * B * (C - 0.5) * 8
    gbs = alg_bytes / pass_s / 1e9
    log(f"bench: grid B={B} C={C} block {block}: {el/steps*1e3:.4f} ms/step; grid pass "
        f"{pass_s*1e3:.4f} ms ({gbs:.0f} GB/s), in-block grid step {edge_s*1e3:.4f} ms, "
        f"lattice {kt[1][0]/max(kt[1][1],1):.4f} ms")
    return {"workload": f"large 2D channel 1024x512 on the quasi-logarithmic history grid, "
                        f"B={B} blocks of C={C} (reach {C * (2 ** B - 1)} steps)",
            "value": ch.nodes * steps / el, "unit": "node-steps/s", "ms_per_step": el / steps * 1e3,
            "dtype": "f32 history + f64 lattice", "steps_per_pass": block,
            "roofline": {"bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": gbs / HBM_PEAK_GBS,
                         "traffic": measured("leg_traffic_bytes", ("grid", block)),
                         "kernel": f"k_grid_pass ({block} steps per pass)",
                         "kernel_avg_ms": pass_s * 1e3, "alg_bytes_per_launch": alg_bytes,
                         "in_block_step_avg_ms": edge_s * 1e3}}


def bench_finger(steps: int = 128):
    """The perturbed large 2D channel with the full Finger tensor (the exact
    model for non-unidirectional flow), FP64 lattice and FP32 history,
    16 steps per pass, persistent pass."""
    import torch
    import workloads
    from paper_1504_06123_amd import Solver, autotune

    ch = workloads.large_2d().channels[0].replace(finger=True)
    s = Solver([ch], precision="f32p64")
    s.step(16)
    cfg = dict(block=16, vec=1, chunk_len=1 << 30, persistent=True, graph=0)
    autotune.apply(s, cfg)
    s.step(32)
    el, kt = time_steps(s, steps)
    s.close()
    del s
    torch.cuda.empty_cache()
    pass_s = kt[0][0] / kt[0][1] / 1e3
    # 32 B per entry: kappa (4 x FP32) and exp(kappa dt) - I (4 x FP32)
    alg_bytes = ch.nodes * ch.n_hist * 32
    gbs = alg_bytes / pass_s / 1e9
    log(f"bench: full tensor: {el/steps*1e3:.4f} ms/step, pass {pass_s*1e3:.3f} ms "
        f"({gbs:.0f} GB/s)")
    return {"workload": "large 2D channel 1024x512, N_h=4096, full Finger tensor",
            "value": ch.nodes * steps / el, "unit": "node-steps/s",
            "ms_per_step": el / steps * 1e3, "dtype": "f32 history + f64 lattice",
            "config": cfg,
            "roofline": {"bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": gbs / HBM_PEAK_GBS,
                         "traffic": measured("leg_traffic_bytes", ("full_tensor", 16)),
                         "kernel": "k_finger_pass_persistent (16 steps per pass)",
                         "kernel_avg_ms": pass_s * 1e3, "alg_bytes_per_launch": alg_bytes}}


def bench_laws(steps: int = 256):
    """The large 2D channel with the accumulated-strain damping variant
    (32-step passes, one bulk sum per entry), with the instantaneous law (no
    history), and with the integral law coupled through the paper's forcing
    term; FP64 lattice and FP32 history."""
    import torch
    import workloads
    from paper_1504_06123_amd import Solver, autotune

    base = workloads.large_2d().channels[0]
    out = {}
    for law, block, coupled in (("strain_damping", 32, False), ("instantaneous", 1, False),
                                ("nlm", 32, True)):
        ch = base.replace(law=law, paper_coupling=coupled)
        s = Solver([ch], precision="f32p64")
        s.step(32)
        autotune.apply(s, dict(block=block, vec=1, chunk_len=1 << 30, persistent=False,
                               graph=0))
        s.step(2 * block)
        el, kt = time_steps(s, steps)
        s.close()
        del s
        torch.cuda.empty_cache()
        rec = {"value": ch.nodes * steps / el, "unit": "node-steps/s",
               "ms_per_step": el / steps * 1e3, "steps_per_pass": block,
               "lattice_kernel_ms": kt[1][0] / max(kt[1][1], 1)}
        if law == "strain_damping":
            pass_s = kt[0][0] / kt[0][1] / 1e3
            alg = ch.nodes * ch.n_hist * 8
            rec["roofline"] = {"bound": "hbm", "achieved": alg / pass_s / 1e9,
                               "peak": HBM_PEAK_GBS, "unit": "GB/s",
                               "frac": alg / pass_s / 1e9 / HBM_PEAK_GBS,
                               "traffic": measured("leg_traffic_bytes",
                                                   ("strain_damping", block)),
                               "kernel": "k_wm_pass (32 steps per pass)",
                               "kernel_avg_ms": pass_s * 1e3, "alg_bytes_per_launch": alg}
        name = "nlm_paper_coupling" if coupled else law
        log(f"bench: {name}: {rec['ms_per_step']:.4f} ms/step")
        out[name] = rec
    return out


def bench_batched(steps: int = 2000):
    """64 uneven channels: tuned FP32 batched path vs plain per-channel FP64."""
    import torch
    import workloads
    from paper_1504_06123_amd import Solver, autotune

    wl = workloads.batched()
    nodes = wl.nodes
    s = Solver(wl.channels, precision="f32")
    s.step(64)
    best = autotune.tune(s, autotune.candidates(s, blocks=(8, 16, 32),
                                                chunk_lens=(256, 512, 1024, 2048, 4096),
                                                graphs=graph_lens()), min_steps=64)
    M = best["block"]
    s.step(64)
    el, kt = time_steps(s, max(M, steps // M * M))
    steps = max(M, steps // M * M)
    s.close()
    batched = nodes * steps / el
    # the history pass (with its chunk combine) over the 64 windows
    pass_s = kt[0][0] / kt[0][1] / 1e3
    entries = wl.entries_per_step
    tflops = entries * pass_flops_per_entry(M) / pass_s / 1e12
    gbs = entries * 4 / pass_s / 1e9  # unidirectional: FP32 shear rate only
    # plain per-channel FP64: one handle per channel, one step at a time
    handles = [Solver([c], precision="f64") for c in wl.channels]
    for h in handles:
        h.step(2)
    base_steps = 20
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(base_steps):
        for h in handles:
            h.step(1)
    torch.cuda.synchronize()
    el64 = time.perf_counter() - t0
    for h in handles:
        h.close()
    plain = nodes * base_steps / el64
    cfg = {k: best[k] for k in ("block", "vec", "chunk_len", "persistent", "graph")}
    return {"workload": "64 channels, lx=1, ly log-uniform [16,1024], tau U[50,2000], "
                        "window 10*tau rounded to a power of two",
            "nodes": nodes, "history_entries_per_step": wl.entries_per_step,
            "value": batched, "unit": "node-steps/s", "dtype": "f32", "config": cfg,
            "ms_per_step": el / steps * 1e3,
            "roofline": {"bound": "alu", "achieved": tflops, "peak": FP32_PEAK_TFLOPS,
                         "unit": "TFLOP/s", "frac": tflops / FP32_PEAK_TFLOPS, "traffic": None,
                         "kernel": f"k_hist_pass + k_combine ({M} steps per pass)",
                         "kernel_avg_ms": pass_s * 1e3, "hbm_GBs": gbs,
                         "hbm_frac": gbs / HBM_PEAK_GBS},
            "plain_per_channel_f64": plain, "speedup_vs_plain_f64": batched / plain}


def bench_adjoint(repeats: int = 3, oracle_steps: int = 200):
    """Gradients of the differentiation run (1 x 128 channel, window 2048,
    4000 steps, u_x sampled every 200, checkpoints every 256; LB_F32, 32-step
    blocks): the forward run with its snapshots, then the adjoint sweep
    (segment replay and the discrete adjoint), for dL/d(G_inf, tau, gamma_c,
    g_x) of L = sum (u - u_target)^2 with the target from the true
    parameters; forward steps and replays in 64-step graphs.  The oracle's central differences need 8 forward runs; their
    cost is extrapolated from `oracle_steps` timed oracle steps."""
    import numpy as np
    import torch
    import oracle
    import workloads
    from paper_1504_06123_amd import Solver, adjoint

    wl = workloads.differentiation()
    ch = wl.channels[0]
    steps, every, seg = wl.steps, wl.sample_every, 256
    prec, block = wl.precision, 32
    with Solver([workloads.true_channel(ch)], precision=prec) as s:
        s.set_block(block)
        target, _ = adjoint.forward(s, steps, every, seg)
    fw, bw = [], []
    with Solver([ch], precision=prec) as s:
        s.set_block(block)
        s.set_graph(GRAPH_LEN)
        init = s.save_state()
        for _ in range(repeats + 1):      # the first round warms up
            s.load_state(init)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            u, ckpts = adjoint.forward(s, steps, every, seg)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            g = adjoint.backward(s, ckpts, steps, every, seg, 2 * (u - target),
                                 t_start=int(ckpts[0][0]))
            torch.cuda.synchronize()
            t2 = time.perf_counter()
            fw.append(t1 - t0)
            bw.append(t2 - t1)
            del ckpts
    f_s, b_s = min(fw[1:]), min(bw[1:])
    # the adjoint history transpose reads the FP64 adjoint ring once per
    # node and step: n_hist x 8 B
    alg = ch.nodes * ch.n_hist * 8 * steps
    gbs = alg / b_s / 1e9
    oc = oracle.OracleChannel(ch)
    t0 = time.perf_counter()
    oc.step(oracle_steps)
    per_step = (time.perf_counter() - t0) / oracle_steps
    oc.close()
    fd_s = 8 * steps * per_step
    log(f"bench: adjoint 1x{ch.ly} N_h={ch.n_hist} {steps} steps: forward {f_s*1e3:.1f} ms, "
        f"sweep {b_s*1e3:.1f} ms ({b_s/steps*1e6:.1f} us per step); oracle FD ~{fd_s:.0f} s")
    return {"workload": f"differentiation run, 1x{ch.ly} channel, N_h={ch.n_hist}, {steps} steps, "
                        f"u_x sampled every {every}, checkpoints every {seg}",
            "value": 1.0 / (f_s + b_s), "unit": "gradients/s", "dtype": prec,
            "steps_per_pass": block,
            "forward_ms": f_s * 1e3, "sweep_ms": b_s * 1e3,
            "sweep_us_per_step": b_s / steps * 1e6,
            "gradient": [float(x) for x in np.asarray(g)[0]],
            "roofline": {"bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": gbs / HBM_PEAK_GBS, "traffic": None,
                         "kernel": "adjoint sweep (history transpose over the FP64 adjoint ring)",
                         "alg_bytes": alg,
                         "note": "128 nodes: a handful of wavefronts per launch, latency-bound"},
            "oracle_fd": {"seconds_per_gradient": fd_s, "kind": "oracle",
                          "sample": f"{oracle_steps} oracle steps timed, x 8 runs x {steps} steps",
                          "cores": 1},
            "speedup_vs_oracle_fd": fd_s / (f_s + b_s)}


def counter_run(leg: str, copy_mib: int = 4096):
    """A short plain-launch run for hardware-counter collection (no HIP
    events, no graphs): `copy` copies `copy_mib` MiB device to device (the
    calibration of FETCH_SIZE and WRITE_SIZE); the other legs build the
    channel as their timed leg does, take 32 warm-up steps in the default
    launch shape (one-step passes), then 4 blocks in the leg's shape."""
    import numpy as np
    import torch
    import workloads
    from paper_1504_06123_amd import Solver, autotune

    if leg == "copy":
        n = copy_mib << 18
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        return {"counter_run": leg, "bytes": n * 4}
    base = workloads.large_2d().channels[0]
    prec, block, persistent = "f32p64", 32, True
    if leg in ("f32", "f32p64"):
        ch, prec = base, leg
    elif leg == "grid":
        ch, block = base.replace(hist_blocks=6, hist_block_len=128), 16
    elif leg == "full_tensor":
        ch, block = base.replace(finger=True), 16
    elif leg == "strain_damping":
        ch, persistent = base.replace(law="strain_damping"), False
    else:
        raise ValueError(f"unknown counter-run leg {leg}")
    s = Solver([ch], precision=prec)
    if leg == "grid":
        s.set_block(block)
        s.step(2 * 128)
    else:
        s.step(32)
        autotune.apply(s, dict(block=block, vec=1, chunk_len=1 << 30,
                               persistent=persistent, graph=0))
    s.step(4 * block)
    torch.cuda.synchronize()
    _, ux, _ = s.fields(0)
    assert np.isfinite(ux).all()
    steps = s.t
    s.close()
    return {"counter_run": leg, "precision": prec, "steps_per_pass": block, "steps": steps}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=800)
    ap.add_argument("--warmup", type=int, default=32)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--no-grid", action="store_true")
    ap.add_argument("--no-finger", action="store_true")
    ap.add_argument("--no-laws", action="store_true")
    ap.add_argument("--no-adjoint", action="store_true")
    ap.add_argument("--only", choices=("grid", "full_tensor", "laws", "batched", "adjoint"),
                    help="run one side leg alone and print its record")
    ap.add_argument("--no-tune", action="store_true")
    ap.add_argument("--block", type=int, default=32, help="steps per pass without tuning")
    ap.add_argument("--persistent", action="store_true", help="persistent pass without tuning")
    ap.add_argument("--graph", type=int, default=0, help="graph replay length without tuning")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--side-f32p64", dest="side", action="store_true", default=True,
                    help="also time the mode with FP64 populations (default)")
    ap.add_argument("--no-side-f32p64", dest="side", action="store_false")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="first copy this many MiB device-to-device (counter calibration)")
    ap.add_argument("--counter-run", choices=("copy", "f32", "f32p64", "grid", "full_tensor",
                                              "strain_damping"),
                    help="a short plain-launch run of one leg for rocprofv3 --pmc")
    ap.add_argument("--no-graphs", action="store_true",
                    help="plain launches only, in every leg (for rocprofv3 counter runs, "
                         "which have ended with a host segfault inside stream capture)")
    args = ap.parse_args()
    if args.no_graphs:
        global GRAPH_LEN
        GRAPH_LEN = 0
    if args.gpus != 1:
        print(json.dumps({"error": "liblbmax runs on one GPU per process and bench.py "
                                   "measures one GPU; --gpus must be 1 (sharding across "
                                   "GPUs is described, not implemented)"}))
        sys.exit(2)

    import numpy as np
    import torch
    import workloads
    from paper_1504_06123_amd import Solver, _lib, autotune

    if not os.path.exists(_lib.LIB_PATH):
        import __graft_entry__
        __graft_entry__.build()

    if args.counter_run:
        print(json.dumps(counter_run(args.counter_run, args.copy_probe_mib or 4096)),
              flush=True)
        return

    if args.copy_probe_mib:
        n = args.copy_probe_mib << 18  # float32 elements
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        log(f"bench: copy probe of {args.copy_probe_mib} MiB done")
        del src, dst

    if args.only:
        # one side leg alone (for profiling); prints that leg's record
        legs = {"grid": bench_grid, "full_tensor": bench_finger, "laws": bench_laws,
                "batched": bench_batched, "adjoint": bench_adjoint}
        print(json.dumps({args.only: legs[args.only]()}), flush=True)
        return

    wl = workloads.large_2d()
    ch = wl.channels[0]
    nodes, H = ch.nodes, ch.n_hist
    main = bench_large_2d(wl, args, "f32")
    side = bench_large_2d(wl, args, "f32p64") if args.side else None
    el, steps, cfg, roof = main["el"], main["steps"], main["cfg"], main["roof"]
    node_steps = nodes * steps / el
    entries = nodes * H

    grid = None
    if not args.no_grid:
        log("bench: large 2D channel on the quasi-logarithmic grid")
        grid = bench_grid()
    finger = None
    if not args.no_finger:
        log("bench: large 2D channel with the full Finger tensor")
        finger = bench_finger()
    laws = None
    if not args.no_laws:
        log("bench: alternative constitutive laws on the large 2D channel")
        laws = bench_laws()
    adj = None
    if not args.no_adjoint:
        log("bench: gradients of the differentiation run (adjoint)")
        adj = bench_adjoint()
    batched = None
    if not args.no_batched:
        log("bench: batched 64-channel workload")
        batched = bench_batched()
        log(f"bench: batched {batched['value']:.3e} node-steps/s, plain per-channel FP64 "
            f"{batched['plain_per_channel_f64']:.3e}")
    cpu = None
    if not args.no_cpu_baseline:
        log("bench: timing the FP64 oracle on the host")
        cpu = cpu_baseline(args.cpu_seconds)

    line = {
        "metric": "lattice node-steps/sec at history length N_h; achieved HBM GB/s vs peak",
        "value": node_steps,
        "unit": "node-steps/s",
        "n_gpus": 1,
        "steps": steps,
        "steps_requested": args.steps,
        "warmup": args.warmup,
        "ms_per_step": el / steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 (populations: FP32 remainders on FP64 moments; history: FP32 ring, "
                 "FP32 partial sums into Kahan-compensated FP32 totals; FP64 strain)",
        "data": "synthetic",
        "config": {"workload": "large 2D channel 1024x512, N_h=4096, tau=1000 steps, "
                               "g=5e-6, 1% seeded velocity perturbation",
                   "lx": ch.lx, "ly": ch.ly, "n_hist": H, "nodes": nodes,
                   "history_entries_per_step": entries, "launch": cfg,
                   "precision": "f32"},
        "roofline": roof,
        # the same history kernel run once per step (the shape the blocked
        # pass replaces): HBM-bound
        "history_pass_one_step": main["one_step"],
        "entry_updates_per_s": entries * steps / el,
        # the first block alone (one history pass and its in-block steps)
        "burst": main["burst"],
        "f32p64": side and {"value": side["node_steps_per_s"],
                            "ms_per_step": side["ms_per_step"], "steps": side["steps"],
                            "launch": side["cfg"], "roofline": side["roof"],
                            "burst": side["burst"]},
        "grid": grid,
        "full_tensor": finger,
        "laws": laws,
        "batched": batched,
        "adjoint": adj,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
