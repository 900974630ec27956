"""GPU parity: the HIP path (through the C interface) against the FP64 oracle
on identical seeded inputs.

Error metric per output X: max over samples and nodes of |X_gpu - X_ref|,
divided by max over samples and nodes of |X_ref| (normalised max-norm; it
stays meaningful through zero crossings of the velocity during cessation).
Both velocity components are divided by the speed scale max |u| of the
reference.
Tolerances: FP32 path 1e-5 for velocity and 1e-4 for sigma_xy and N1.  FP64
path 1e-11: the oracle keeps whole populations (about 0.44, rounding unit
5.6e-17) while the GPU keeps deviations from the weights, so the two differ
by the oracle's own rounding floor, about 1e-16 absolute per step; for
velocities of 1e-4 that random-walks to a few 1e-12 over 10^3 steps (the
largest seen is 3.1e-12).
"""
import math
import os

import numpy as np
import pytest

import oracle
import workloads

pytestmark = pytest.mark.gpu

TOL64 = 1e-11
TOL32 = {"ux": 1e-5, "uy": 1e-5, "sxy": 1e-4, "n1": 1e-4}


@pytest.fixture(scope="module")
def Solver():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1504_06123_amd import Solver as S, _lib
    assert os.path.exists(_lib.LIB_PATH), "liblbmax.so not built"
    return S


def say(msg):
    print(msg, flush=True)


def nerr(a, b):
    a, b = np.asarray(a), np.asarray(b)
    den = np.abs(b).max()
    return float(np.abs(a - b).max() / den) if den > 0 else float(np.abs(a).max())


def run_gpu(Solver, chans, precision, steps, every, steps_on=None, chunks=None, graph=0,
            vec=None, block=1, persistent=False):
    """Advance all channels together; sample every `every` steps.  The force
    goes to zero after steps_on steps (cessation)."""
    steps_on = steps if steps_on is None else steps_on
    out = [{k: [] for k in ("ux", "uy", "rho", "sxy", "n1")} for _ in chans]
    with Solver(chans, precision=precision) as s:
        for ci in range(len(chans)):
            nc = s.tiling(ci)[0] if chunks is None else chunks[ci]
            v = s.tiling(ci)[1] if vec is None else vec[ci]
            s.set_tiling(ci, nc, v)
        if block != 1:
            s.set_block(block)
        if persistent:
            s.set_persistent(True)
        if graph:
            s.set_graph(graph)
        marks = sorted({m for m in list(range(every, steps + 1, every)) + [steps_on, steps]
                        if 0 < m <= steps})
        done = 0
        for m in marks:
            if done >= steps_on:
                for ci in range(len(chans)):
                    s.set_force(ci, 0.0, 0.0)
            s.step(m - done)
            done = m
            if done % every == 0:
                for ci in range(len(chans)):
                    rho, ux, uy = s.fields(ci)
                    sxy, n1 = s.stress(ci)
                    for k, v in (("ux", ux), ("uy", uy), ("rho", rho), ("sxy", sxy), ("n1", n1)):
                        out[ci][k].append(v)
    return [{k: np.array(v) for k, v in o.items()} for o in out]


def run_oracle(chans, steps, every, steps_on=None):
    wl = workloads.Workload("t", list(chans), "f64", steps_on=steps if steps_on is None else steps_on,
                            steps_off=0 if steps_on is None else steps - steps_on,
                            sample_every=every)
    return oracle.run_workload(wl, steps=steps, sample_every=every)


def compare(gpu, ref, tol, keys=("ux", "sxy", "n1"), label=""):
    """Velocity components are normalised by the speed scale max(|u_x|, |u_y|)
    of the reference: in a unidirectional channel u_y is rounding noise on
    both sides and has no scale of its own."""
    vscale = max(np.abs(ref["ux"]).max(), np.abs(ref["uy"]).max())
    errs = {}
    for k in keys:
        if k in ("ux", "uy"):
            errs[k] = float(np.abs(gpu[k] - ref[k]).max() / vscale)
        else:
            errs[k] = nerr(gpu[k], ref[k])
    say(f"  {label} errors: " + ", ".join(f"{k}={v:.2e}" for k, v in errs.items()))
    for k, v in errs.items():
        t = tol[k] if isinstance(tol, dict) else tol
        assert v <= t, f"{label} {k}: {v:.3e} > {t:.1e}"
    return errs


# ---------------------------------------------------------------------------
# FP64 path
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("chunks", [None, 1])
def test_plain_f64_channel(Solver, chunks):
    """4 x 16 channel, FP64, tau = 100, window 1000, startup, 2000 steps."""
    wl = workloads.plain_f64()
    say(f"case plain_f64 chunks={chunks}")
    gpu = run_gpu(Solver, wl.channels, "f64", 2000, 100,
                  chunks=None if chunks is None else [chunks])[0]
    ref = run_oracle(wl.channels, 2000, 100)[0]
    compare(gpu, ref, TOL64, keys=("ux", "uy", "rho", "sxy", "n1"), label="plain_f64")


def test_f64_gradient_readout(Solver):
    ch = workloads.large_2d(lx=6, ly=9, n_hist=64).channels[0]
    say("case f64 gradient 6x9")
    with Solver([ch], precision="f64") as s:
        s.step(37)
        k = s.grad(0)
    oc = oracle.OracleChannel(ch)
    oc.step(37)
    kr = oc.grad()
    _, uxr, uyr = oc.fields()
    # kappa is a difference of velocities (stencil weights summing to at most
    # 4/3 + 1 in magnitude): its error is bounded by that of the velocity, so
    # it is measured on the velocity scale
    vscale = max(np.abs(uxr).max(), np.abs(uyr).max())
    for i in range(4):
        err = float(np.abs(k[i] - kr[i]).max() / vscale)
        say(f"  kappa[{i}] error on the velocity scale {err:.2e}")
        assert err < 3 * TOL64


@pytest.mark.parametrize("name,kw", [
    ("min_width_ly3", dict(lx=1, ly=3, n_hist=2)),
    ("ragged_3x37", dict(lx=3, ly=37, n_hist=300)),
    ("newtonian", dict(lx=2, ly=20, g_inf=0.0, n_hist=50)),
    ("ucm", dict(lx=1, ly=24, gamma_c=math.inf, n_hist=400, tau_m=60.0)),
    ("ragged_window_1000", dict(lx=5, ly=70, n_hist=1000, tau_m=80.0)),
])
def test_f64_edge_cases(Solver, name, kw):
    ch = workloads.plain_f64().channels[0].replace(gx=2e-5, **kw)
    say(f"case f64 edge {name}")
    gpu = run_gpu(Solver, [ch], "f64", 700, 100, steps_on=450)[0]
    ref = run_oracle([ch], 700, 100, steps_on=450)[0]
    keys = ("ux", "uy", "rho") if ch.g_inf == 0 else ("ux", "uy", "rho", "sxy", "n1")
    compare(gpu, ref, TOL64, keys=keys, label=name)


def test_f64_2d_perturbed(Solver):
    ch = workloads.large_2d(lx=24, ly=16, n_hist=256).channels[0].replace(tau_m=60.0)
    say("case f64 2d perturbed 24x16")
    gpu = run_gpu(Solver, [ch], "f64", 600, 100)[0]
    ref = run_oracle([ch], 600, 100)[0]
    compare(gpu, ref, TOL64, keys=("ux", "uy", "rho", "sxy", "n1"), label="f64_2d")


# ---------------------------------------------------------------------------
# FP32 paths: split FP32 population storage ("f32") or FP64 populations
# ("f32p64"); FP32 history, FP32 partial sums into Kahan-compensated FP32
# totals; FP64 strain
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("precision", ["f32", "f32p64"])
def test_f32_startup_cessation_reduced(Solver, precision):
    """Quasi-1D startup then cessation, FP32 history vs FP64 oracle."""
    ch = workloads.startup_cessation().channels[0].replace(ly=64, n_hist=1024, tau_m=250.0, gx=5e-6)
    say(f"case {precision} startup/cessation 1x64")
    gpu = run_gpu(Solver, [ch], precision, 3000, 100, steps_on=1500)[0]
    ref = run_oracle([ch], 3000, 100, steps_on=1500)[0]
    compare(gpu, ref, TOL32, label="f32_startcess")


@pytest.mark.parametrize("precision", ["f32", "f32p64"])
def test_f32_2d_perturbed(Solver, precision):
    ch = workloads.large_2d(lx=32, ly=24, n_hist=512).channels[0].replace(tau_m=100.0)
    say(f"case {precision} 2d perturbed 32x24")
    gpu = run_gpu(Solver, [ch], precision, 800, 100)[0]
    ref = run_oracle([ch], 800, 100)[0]
    compare(gpu, ref, TOL32, keys=("ux", "uy", "sxy", "n1"), label="f32_2d")


def test_f32_batched_uneven_channels(Solver):
    """Several channels of uneven width and window in one handle: each must
    match its own oracle run."""
    wl = workloads.batched()
    chans = [c.replace(n_hist=min(c.n_hist, 2048), tau_m=min(c.tau_m, 200.0))
             for c in sorted(wl.channels, key=lambda c: c.ly)[::9]]
    say(f"case f32 batched {[c.ly for c in chans]}")
    gpu = run_gpu(Solver, chans, "f32", 600, 200)
    ref = run_oracle(chans, 600, 200)
    for ci in range(len(chans)):
        compare(gpu[ci], ref[ci], TOL32, label=f"batched ch{ci} ly={chans[ci].ly}")


# ---------------------------------------------------------------------------
# Launch-shape invariance, determinism, graphs, state
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("block", [1, 32])
def test_chunk_split_invariance(Solver, block):
    """A window split into 2, 7 or 16 age chunks (combined in FP64) equals the
    unsplit window to rounding order, past the first window fill (2048-entry
    window, 2600 steps with cessation at 1800), so the window-end terms of
    non-final chunks carry real entries; each run also matches the oracle."""
    ch = workloads.startup_cessation().channels[0].replace(ly=40, n_hist=2048, tau_m=300.0,
                                                            gx=5e-6)
    steps, on = 2600, 1800
    say(f"case chunk invariance, block {block}")
    a = run_gpu(Solver, [ch], "f64", steps, 200, steps_on=on, chunks=[1], block=block)[0]
    ref = run_oracle([ch], steps, 200, steps_on=on)[0]
    compare(a, ref, TOL64, label="chunks=1")
    for nc in (2, 7, 16):
        b = run_gpu(Solver, [ch], "f64", steps, 200, steps_on=on, chunks=[nc], block=block)[0]
        for k in ("ux", "sxy", "n1"):
            assert nerr(b[k], a[k]) < 1e-12, (nc, k)
        compare(b, ref, TOL64, label=f"chunks={nc}")


def test_lane_width_invariance(Solver):
    """Nodes per lane only changes which lane owns which node.  Widths 1 and 2
    group the same number of rows per partial sum, so they agree bit for bit;
    width 4 groups fewer rows and agrees to rounding."""
    ch = workloads.large_2d(lx=40, ly=30, n_hist=700).channels[0].replace(tau_m=90.0)
    say("case lane width invariance")
    for prec, tol in (("f32", 1e-6), ("f64", 1e-13)):
        a = run_gpu(Solver, [ch], prec, 300, 100, chunks=[3], vec=[1])[0]
        b = run_gpu(Solver, [ch], prec, 300, 100, chunks=[3], vec=[2])[0]
        c = run_gpu(Solver, [ch], prec, 300, 100, chunks=[3], vec=[4])[0]
        for k in a:
            assert np.array_equal(a[k], b[k]), (prec, k)
        for k in ("ux", "sxy", "n1"):
            assert nerr(c[k], a[k]) < tol, (prec, k)


@pytest.mark.parametrize("name,kw,chunks", [
    ("2d", dict(lx=6, ly=11, n_hist=300, tau_m=40.0, u0="perturb"), None),
    ("uni_chunked", dict(lx=1, ly=40, n_hist=1500, tau_m=120.0), [9]),
    ("window2", dict(lx=2, ly=9, n_hist=2, tau_m=5.0), None),
    ("window5", dict(lx=1, ly=7, n_hist=5, tau_m=3.0), None),
    ("window9_ucm", dict(lx=3, ly=8, n_hist=9, tau_m=4.0, gamma_c=math.inf), None),
])
def test_temporal_blocking_f64(Solver, name, kw, chunks):
    """One history pass per block of M steps: FP64 results match the oracle
    and the unblocked path (rounding order only), including windows shorter
    than the block and split windows."""
    u0 = kw.pop("u0", None)
    ch = workloads.plain_f64().channels[0].replace(gx=3e-5, **kw)
    if u0 == "perturb":
        ch = ch.replace(u0=workloads.large_2d(lx=ch.lx, ly=ch.ly, n_hist=2).channels[0].u0)
    say(f"case blocking f64 {name}")
    ref = run_oracle([ch], 420, 35, steps_on=300)[0]
    base = run_gpu(Solver, [ch], "f64", 420, 35, steps_on=300, chunks=chunks)[0]
    for M in (2, 4, 8, 16, 32):
        got = run_gpu(Solver, [ch], "f64", 420, 35, steps_on=300, chunks=chunks, block=M)[0]
        compare(got, ref, TOL64, keys=("ux", "uy", "sxy", "n1"), label=f"{name} M={M}")
        for k in ("ux", "sxy", "n1"):
            assert nerr(got[k], base[k]) < 1e-12, (M, k)


def test_temporal_blocking_f32_2d(Solver):
    ch = workloads.large_2d(lx=32, ly=24, n_hist=512).channels[0].replace(tau_m=100.0)
    say("case blocking f32 2d")
    ref = run_oracle([ch], 800, 100)[0]
    for M in (4, 8, 16, 32):
        got = run_gpu(Solver, [ch], "f32", 800, 100, block=M)[0]
        compare(got, ref, TOL32, keys=("ux", "uy", "sxy", "n1"), label=f"f32_2d M={M}")


def test_blocking_save_load_mid_block_and_graph(Solver):
    ch = workloads.large_2d(lx=8, ly=12, n_hist=200).channels[0].replace(tau_m=40.0)
    say("case blocking save/load + graph")
    with Solver([ch], precision="f32") as s:
        s.set_block(4)
        s.step(150)                 # 150 = 37 blocks + 2 steps: inside a block
        buf = s.save_state()
        s.step(77)
        want = s.fields(0), s.stress(0)
        s.step(5)
        s.load_state(buf)
        s.step(77)
        got = s.fields(0), s.stress(0)
    for a, b in zip(want, got):
        for x, y in zip(a, b):
            assert np.array_equal(x, y)
    a = run_gpu(Solver, [ch], "f32", 400, 100, block=4)[0]
    b = run_gpu(Solver, [ch], "f32", 400, 100, block=4, graph=32)[0]
    for k in a:
        assert np.array_equal(a[k], b[k]), k


def test_persistent_pass_bitwise(Solver):
    """The persistent pass computes the same tiles as the plain launch, only
    scheduled differently: identical bits, also for many uneven channels."""
    wl = workloads.batched()
    chans = [c.replace(n_hist=min(c.n_hist, 1024)) for c in wl.channels[:12]]
    say("case persistent pass")
    for block in (1, 4):
        a = run_gpu(Solver, chans, "f32", 200, 100, block=block)
        b = run_gpu(Solver, chans, "f32", 200, 100, block=block, persistent=True)
        for ca, cb in zip(a, b):
            for k in ca:
                assert np.array_equal(ca[k], cb[k]), (block, k)


def test_autotune_restores_state(Solver):
    from paper_1504_06123_amd import autotune
    ch = workloads.large_2d(lx=16, ly=40, n_hist=512).channels[0].replace(tau_m=60.0)
    say("case autotune")
    with Solver([ch], precision="f32") as s:
        s.step(123)
        before = s.fields(0), s.stress(0)
        best = autotune.tune(s, autotune.candidates(s, blocks=(1, 8), chunk_lens=(128, 1 << 30)),
                             min_steps=16)
        assert s.t == 123 and best["ms_per_step"] > 0
        after = s.fields(0), s.stress(0)
        for a, b in zip(before, after):
            for x, y in zip(a, b):
                assert np.array_equal(x, y)
        s.step(200)
        _, ux, _ = s.fields(0)
    oc = oracle.OracleChannel(ch)
    oc.step(323)
    _, rux, _ = oc.fields()
    assert nerr(ux, rux) < TOL32["ux"]


def test_bitwise_determinism_and_graph_replay(Solver):
    ch = workloads.large_2d(lx=16, ly=20, n_hist=300).channels[0].replace(tau_m=50.0)
    say("case determinism + graph")
    a = run_gpu(Solver, [ch], "f32", 400, 100)[0]
    b = run_gpu(Solver, [ch], "f32", 400, 100)[0]
    c = run_gpu(Solver, [ch], "f32", 400, 100, graph=32)[0]
    for k in a:
        assert np.array_equal(a[k], b[k]), k
        assert np.array_equal(a[k], c[k]), k


@pytest.mark.parametrize("precision", ["f32", "f32p64", "f64"])
def test_save_load_resume_bitwise(Solver, precision):
    ch = workloads.large_2d(lx=8, ly=12, n_hist=200).channels[0].replace(tau_m=40.0)
    say(f"case save/load {precision}")
    with Solver([ch], precision=precision) as s:
        s.step(150)
        buf = s.save_state()
        s.step(77)
        want = s.fields(0), s.stress(0)
        s.step(5)
        s.load_state(buf)
        assert s.t == 150
        s.step(77)
        got = s.fields(0), s.stress(0)
    for a, b in zip(want, got):
        for x, y in zip(a, b):
            assert np.array_equal(x, y)


@pytest.mark.parametrize("block,graph", [(1, 0), (32, 64)])
def test_zero_and_negative_step_counts(Solver, block, graph):
    """lb_step(0) is a no-op (state bit for bit, step counter and block
    position unchanged, also in the middle of a block with graphs on);
    lb_step(-1) fails with LB_EINVAL and leaves the handle usable."""
    import torch
    from paper_1504_06123_amd import LBError, _lib
    ch = workloads.large_2d(lx=8, ly=12, n_hist=64).channels[0].replace(tau_m=30.0)
    say(f"case zero and negative step counts, block {block}, graph {graph}")
    with Solver([ch], precision="f32") as s:
        s.set_block(block)
        if graph:
            s.set_graph(graph)
        s.step(45)  # mid-block for block 32
        before = s.save_state().clone()
        s.step(0)
        assert s.t == 45
        assert torch.equal(s.save_state(), before)
        with pytest.raises(LBError) as ei:
            s.step(-1)
        assert ei.value.status == _lib.LB_EINVAL
        assert s.t == 45
        assert torch.equal(s.save_state(), before)
        s.step(19)
        got = s.fields(0), s.stress(0)
    with Solver([ch], precision="f32") as s:
        s.set_block(block)
        if graph:
            s.set_graph(graph)
        s.step(45)
        s.step(19)
        want = s.fields(0), s.stress(0)
    for a, b in zip(want, got):
        for x, y in zip(a, b):
            assert np.array_equal(x, y)


def test_readout_before_first_step_is_state_error(Solver):
    from paper_1504_06123_amd import LBError
    ch = workloads.plain_f64().channels[0]
    with Solver([ch], precision="f64") as s:
        with pytest.raises(LBError) as ei:
            s.fields(0)
        assert ei.value.status == -4
        with pytest.raises(LBError):
            s.set_force(3, 0.0)


# ---------------------------------------------------------------------------
# Full-size 2D channel 1024 x 512, window 4096, in the benchmark's launch
# configuration
# ---------------------------------------------------------------------------

def test_large_2d_full_size_first_steps(Solver):
    """First 12 steps of the full-size perturbed channel, every node."""
    wl = workloads.large_2d()
    ch = wl.channels[0]
    say("case large_2d full size, 12 steps")
    with Solver([ch], precision="f32") as s:
        s.step(12)
        _, ux, uy = s.fields(0)
        sxy, n1 = s.stress(0)
    oc = oracle.OracleChannel(ch)
    oc.step(12)
    _, rux, ruy = oc.fields()
    rsxy, rn1 = oc.stress()
    errs = dict(ux=nerr(ux, rux), uy=nerr(uy, ruy), sxy=nerr(sxy, rsxy), n1=nerr(n1, rn1))
    say(f"  errors {errs}")
    for k, v in errs.items():
        assert v <= TOL32[k], (k, v)


@pytest.mark.parametrize("block", [1, 32])
def test_fp32_longest_window(Solver, block):
    """The longest window FP32 histories take, 2^24 entries (ages stay exact
    in FP32), on a 1 x 32 channel (a 4 GiB ring split into 64 age chunks):
    the zero-filled ring makes its first 40 steps equal to the oracle's with
    a 64-entry window, unblocked and with 32 steps per pass."""
    ch = workloads.startup_cessation().channels[0].replace(ly=32, n_hist=1 << 24,
                                                            tau_m=200.0, gx=2e-5)
    steps = 40
    say(f"case longest FP32 window 2^24, 1 x 32, {steps} steps, block {block}")
    with Solver([ch], precision="f32p64") as s:
        assert s.max_chunks(0) == 64
        s.set_block(block)
        s.step(steps)
        _, ux, _ = s.fields(0)
        sxy, n1 = s.stress(0)
    oc = oracle.OracleChannel(ch.replace(n_hist=64))
    oc.step(steps)
    _, rux, _ = oc.fields()
    rsxy, rn1 = oc.stress()
    errs = dict(ux=nerr(ux, rux), sxy=nerr(sxy, rsxy), n1=nerr(n1, rn1))
    say(f"  errors {errs}")
    for k, v in errs.items():
        assert v <= TOL32[k], (k, v)


def test_large_2d_full_size_synthetic_window(Solver):
    """Full-size ring with seeded random history at an arbitrary step (the
    window wraps): sigma at sampled nodes against the oracle's history sum
    of the same inputs.  Fluid at rest, so the pushed entry is zero."""
    import torch
    from paper_1504_06123_amd import pack_state_header, state_layout
    ch = workloads.large_2d(perturb=False).channels[0].replace(gx=0.0)
    H, N = ch.n_hist, ch.nodes
    t_now = 3 * H + 1234
    say("case large_2d full size synthetic window")
    secs, total = state_layout([ch], "f32")
    sec = secs[0]
    gen = torch.Generator(device="cuda").manual_seed(1504)
    with Solver([ch], precision="f32") as s:
        assert s.state_bytes() == total
        st = torch.zeros(total, dtype=torch.uint8, device="cuda")
        hdr = pack_state_header(t_now, 1, "f32", total)
        st[:256] = torch.frombuffer(bytearray(hdr), dtype=torch.uint8).cuda()
        off, rows, n = sec["ring_s"]
        ring_s = st[off:off + rows * n * 4].view(torch.float32).view(rows, n)
        ring_s.uniform_(-1e-3, 1e-3, generator=gen)
        off, rows, n = sec["ring_r"]
        ring_r = st[off:off + rows * n * 4].view(torch.float32).view(rows, n)
        ring_r.uniform_(0.0, 2e-3, generator=gen)
        s.load_state(st)
        s.step(1)
        sxy, n1 = s.stress(0)
        rng = np.random.default_rng(7)
        nodes = rng.choice(N, size=24, replace=False)
        cols_s = ring_s[:, torch.from_numpy(nodes).cuda()].double().cpu().numpy()
        cols_r = ring_r[:, torch.from_numpy(nodes).cuda()].double().cpu().numpy()
    t = t_now  # the step just taken
    got_xy, got_n1, ref_xy, ref_n1 = [], [], [], []
    for j, node in enumerate(nodes):
        s_age = np.zeros(H)
        r_age = np.zeros(H)
        for k in range(1, H):
            slot = (t - k) % H
            s_age[k] = cols_s[slot, j]
            r_age[k] = cols_r[slot, j]
        rxy, rxx = oracle.history_sum_ages(s_age, r_age, ch.g_inf, ch.tau_m, ch.gamma_c)
        y, x = divmod(int(node), ch.lx)
        # per node: relative 1e-4 (the stress bar) above an absolute floor
        assert abs(sxy[y, x] - rxy) <= 1e-4 * abs(rxy) + 1e-12 * ch.g_inf, (node, sxy[y, x], rxy)
        assert abs(n1[y, x] - rxx) <= 1e-4 * abs(rxx) + 1e-12 * ch.g_inf, (node, n1[y, x], rxx)
        got_xy.append(sxy[y, x])
        got_n1.append(n1[y, x])
        ref_xy.append(rxy)
        ref_n1.append(rxx)
    e_xy, e_n1 = nerr(got_xy, ref_xy), nerr(got_n1, ref_n1)
    say(f"  synthetic window errors: sxy={e_xy:.2e}, n1={e_n1:.2e}")
    assert e_xy <= TOL32["sxy"] and e_n1 <= TOL32["n1"]


@pytest.mark.parametrize("precision,block,persistent", [
    ("f64", 1, False), ("f64", 32, True), ("f32", 32, True)])
def test_maximum_node_count(Solver, precision, block, persistent):
    """The largest channels the library takes (lx * ly <= 2^26 - 64): 8192 x
    8191 nodes, a 48-entry window that wraps twice in 100 steps.  Every
    index of a node plane, a history row or a block-sum plane is at its
    largest here; in FP64 one history row is 512 MiB, and the pass reads
    groups of 4 rows (2 GiB) through 32-bit buffer offsets.  The start is
    x-invariant (a seeded velocity profile in y, no force), so every column
    must equal the oracle's 1 x 8191 column."""
    import torch
    lx, ly, steps = 8192, 8191, 100
    rng = np.random.default_rng(workloads.BASE_SEED + 26)
    prof = 1e-3 * rng.uniform(-1.0, 1.0, size=ly)
    base = workloads.plain_f64().channels[0].replace(n_hist=48, tau_m=20.0, gx=0.0)
    col = np.zeros((2, ly, 1))
    col[0, :, 0] = prof
    say(f"case maximum node count {lx}x{ly} ({lx * ly} nodes), {precision}, "
        f"block {block}, persistent {persistent}")
    u0 = np.zeros((2, ly, lx))
    u0[0] = prof[:, None]
    ch = base.replace(lx=lx, ly=ly, u0=u0)
    del u0
    with Solver([ch], precision=precision) as s:
        if block != 1:
            s.set_block(block)
        if persistent:
            s.set_persistent(True)
        s.step(steps)
        _, ux, uy = s.fields(0)
        sxy, n1 = s.stress(0)
    del ch
    torch.cuda.empty_cache()
    oc = oracle.OracleChannel(base.replace(lx=1, ly=ly, u0=col))
    oc.step(steps)
    _, rux, ruy = oc.fields()
    rsxy, rn1 = oc.stress()
    vscale = np.abs(rux).max()
    errs = dict(ux=float(np.abs(ux - rux).max() / vscale),
                sxy=nerr(sxy, np.broadcast_to(rsxy, sxy.shape)),
                n1=nerr(n1, np.broadcast_to(rn1, n1.shape)))
    # u_y is zero up to rounding on both sides (the oracle's whole
    # populations leave about 1e-15, FP32 remainders about 1e-8 of the speed
    # scale): a bound, not a comparison
    uy_max = float(np.abs(uy).max() / vscale)
    say(f"  errors {errs}, max |u_y| / max |u_x| = {uy_max:.1e}")
    tol = TOL32 if precision == "f32" else {k: TOL64 for k in errs}
    for k, v in errs.items():
        assert v <= tol[k], (k, v)
    assert uy_max <= (TOL32["uy"] if precision == "f32" else 1e-9), uy_max
