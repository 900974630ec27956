"""GPU adjoint (lb_adjoint_*) against central finite differences of the FP64
oracle's loss, at the same parameters and with the same target.

Loss: L = sum over sampled steps and nodes of (u_x - u_x_target)^2.
Gradients with respect to (G_inf, tau, gamma_c, g_x).  Tolerances: FP32
adjoint 1e-4 relative per component (the stated bar); FP64 adjoint 1e-5,
set by the finite differences themselves: with a relative step of 1e-6 the
oracle's loss changes by ~1e-7 of itself for the least sensitive parameter,
and the rounding pattern of the whole FP64 trajectory changes with the
parameter, which leaves ~1e-6 of noise in that difference.
"""
import math
import os

import numpy as np
import pytest

import oracle
import workloads

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


@pytest.fixture(scope="module")
def lb():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1504_06123_amd as lb
    from paper_1504_06123_amd import _lib
    assert os.path.exists(_lib.LIB_PATH), "liblbmax.so not built"
    return lb


def say(msg):
    print(msg, flush=True)


def oracle_samples(ch, steps, every):
    wl = workloads.Workload("a", [ch], "f64", steps_on=steps, sample_every=every)
    return oracle.run_workload(wl)[0]["ux"][:, :, 0]


def oracle_fd(ch, target, steps, every, h_rel=1e-6):
    grad = []
    for name in workloads.ADJOINT_PARAMS:
        p = getattr(ch, name)
        hp = h_rel * p
        lp = np.sum((oracle_samples(ch.replace(**{name: p + hp}), steps, every) - target) ** 2)
        lm = np.sum((oracle_samples(ch.replace(**{name: p - hp}), steps, every) - target) ** 2)
        grad.append((lp - lm) / (2 * hp))
    return np.array(grad)


def gpu_gradient(lb, ch, precision, steps, every, seg_len, target, block=1, adjoint_block=None):
    from paper_1504_06123_amd import adjoint
    with lb.Solver([ch], precision=precision) as s:
        if block != 1:
            s.set_block(block)
        if adjoint_block is not None:
            s.set_adjoint_block(adjoint_block)
        u, ckpts = adjoint.forward(s, steps, every, seg_len)
        g = adjoint.backward(s, ckpts, steps, every, seg_len, 2 * (u - target))
    return u, g[0]


def small_channel():
    return workloads.Channel(lx=1, ly=16, tau_lb=1.0, g_inf=2e-3, tau_m=40.0, gamma_c=0.05,
                             n_hist=64, gx=2e-5)


@pytest.mark.parametrize("precision,tol", [("f64", 1e-5), ("f32", 1e-4), ("f32p64", 1e-4)])
def test_adjoint_small_against_oracle_fd(lb, precision, tol):
    ch = small_channel()
    steps, every, seg = 300, 25, 64
    say(f"case adjoint small {precision}")
    target = oracle_samples(ch.replace(g_inf=1.6e-3, tau_m=50.0, gamma_c=0.06, gx=1.7e-5),
                            steps, every)
    fd = oracle_fd(ch, target, steps, every)
    _, g = gpu_gradient(lb, ch, precision, steps, every, seg, target)
    rel = np.abs(g - fd) / np.abs(fd)
    say(f"  fd {fd}\n  adjoint {g}\n  rel {rel}")
    assert np.all(rel < tol), rel


def test_adjoint_f64_tight(lb):
    """With a relative step of 1e-4 the oracle's central differences are
    accurate to ~1e-8 (truncation O(h^2), rounding noise 100x below the 1e-6
    step); the FP64 adjoint must agree to 1e-6 on every parameter."""
    ch = small_channel()
    steps, every, seg = 300, 25, 64
    say("case adjoint small f64, tight")
    target = oracle_samples(ch.replace(g_inf=1.6e-3, tau_m=50.0, gamma_c=0.06, gx=1.7e-5),
                            steps, every)
    fd = oracle_fd(ch, target, steps, every, h_rel=1e-4)
    _, g = gpu_gradient(lb, ch, "f64", steps, every, seg, target)
    rel = np.abs(g - fd) / np.abs(fd)
    say(f"  rel {rel}")
    assert np.all(rel < 1e-6), rel


@pytest.mark.parametrize("adjoint_block", [32, 1])
def test_adjoint_segment_length_and_blocking_invariance(lb, adjoint_block):
    """Both forms of the reverse sweep give the same gradient, bit for bit,
    for any segment length; the forward pass's temporal blocking changes it
    only by rounding."""
    ch = small_channel()
    steps, every = 300, 25
    say(f"case adjoint segment invariance, adjoint block {adjoint_block}")
    target = oracle_samples(ch.replace(gx=1.5e-5), steps, every)
    _, g1 = gpu_gradient(lb, ch, "f64", steps, every, 64, target, adjoint_block=adjoint_block)
    _, g2 = gpu_gradient(lb, ch, "f64", steps, every, 37, target, adjoint_block=adjoint_block)
    assert np.array_equal(g1, g2)
    _, g3 = gpu_gradient(lb, ch, "f64", steps, every, 64, target, block=4)
    assert np.all(np.abs(g3 - g1) <= 1e-10 * np.abs(g1))


def _wide_channel():
    return workloads.Channel(lx=1, ly=200, tau_lb=1.0, g_inf=2e-3, tau_m=40.0, gamma_c=0.05,
                             n_hist=150, gx=2e-7)


@pytest.mark.parametrize("case,precision", [
    ("1x16, window 64", "f64"), ("window 16, shorter than a block", "f64"),
    ("two channels", "f64"), ("1x200, near ages from the ring", "f64"),
    ("windows 16 and 64 in one handle", "f64"), ("1x16, window 64", "f32"),
    ("window 32, the near ages exactly", "f64"), ("window 33, one far age", "f64"),
    ("1x512, the widest blocked channel", "f64"),
])
def test_blocked_sweep_matches_the_per_step_sweep(lb, case, precision):
    """The blocked reverse sweep (the default) against the per-step one: the
    same terms of the history transpose summed in another order, so equal to
    a few FP64 roundings (bound 1e-12 relative per component); and the
    blocked gradient is the same, bit for bit, for every block size and
    segment length, since each entry's window is split at fixed ages."""
    from paper_1504_06123_amd import adjoint
    c0 = small_channel()
    c1 = workloads.Channel(lx=1, ly=23, tau_lb=0.9, g_inf=1e-3, tau_m=25.0, gamma_c=0.08,
                           n_hist=48, gx=1.2e-5)
    chans, seg, seg2 = {
        "1x16, window 64": ([c0], 64, 37),
        "window 16, shorter than a block": ([c0.replace(n_hist=16)], 16, 11),
        "two channels": ([c0, c1], 40, 23),
        "1x200, near ages from the ring": ([_wide_channel()], 64, 37),
        "windows 16 and 64 in one handle": ([c0.replace(n_hist=16), c0], 16, 11),
        "window 32, the near ages exactly": ([c0.replace(n_hist=32)], 32, 19),
        "window 33, one far age": ([c0.replace(n_hist=33)], 33, 20),
        "1x512, the widest blocked channel": (
            [workloads.Channel(lx=1, ly=512, tau_lb=1.0, g_inf=2e-3, tau_m=20.0, gamma_c=0.05,
                               n_hist=40, gx=1e-7)], 40, 23),
    }[case]
    steps, every = 300, 25
    say(f"case blocked vs per-step adjoint sweep, {case}, {precision}")
    target = np.concatenate([oracle_samples(c.replace(gx=0.8 * c.gx), steps, every)
                             for c in chans], axis=1)

    def grad(ablock, seg_len):
        with lb.Solver(chans, precision=precision) as s:
            s.set_adjoint_block(ablock)
            assert s.adjoint_block == ablock
            u, ckpts = adjoint.forward(s, steps, every, seg_len)
            return np.asarray(adjoint.backward(s, ckpts, steps, every, seg_len,
                                               2 * (u - target)))

    per_step = grad(1, seg)
    blocked = grad(32, seg)
    rel = np.abs(blocked - per_step) / np.abs(per_step)
    say(f"  per-step {per_step}\n  blocked  {blocked}\n  rel {rel.max():.2e}")
    assert np.all(rel <= 1e-12), rel
    assert np.array_equal(grad(7, seg), blocked)
    assert np.array_equal(grad(32, seg2), blocked)


def test_blocked_sweep_forms_agree_bit_for_bit(lb):
    """A handle whose channels all have at most 128 nodes runs each block with
    its adjoint state on chip; a wider channel in the handle sends every
    channel through the form that keeps it in device memory.  Same values in
    the same order: the 1 x 16 channel's gradient is the same, bit for bit,
    swept alone and beside a 1 x 200 channel."""
    from paper_1504_06123_amd import adjoint
    c0, wide = small_channel(), _wide_channel()
    steps, every, seg = 300, 25, 64
    say("case blocked sweep, on-chip form vs device-memory form")
    targets = [oracle_samples(c.replace(gx=0.8 * c.gx), steps, every) for c in (c0, wide)]
    with lb.Solver([c0, wide], precision="f64") as s:
        assert s.adjoint_block == 32
        u, ckpts = adjoint.forward(s, steps, every, seg)
        g_mixed = adjoint.backward(s, ckpts, steps, every, seg,
                                   2 * (u - np.concatenate(targets, axis=1)))
    _, g_alone = gpu_gradient(lb, c0, "f64", steps, every, seg, targets[0])
    say(f"  beside 1x200 {g_mixed[0]}\n  alone        {g_alone}")
    assert np.array_equal(g_mixed[0], g_alone)


def test_sweep_form_switched_between_segments(lb):
    """The two forms hand the adjoint state (ring, dbar, fbar, accumulators)
    from one segment to the next in the same layout: a sweep whose segments
    alternate between the blocked and the per-step form gives the per-step
    gradient up to the order of the FP64 history sums (1e-12)."""
    import ctypes
    import torch
    from paper_1504_06123_amd import _lib, adjoint
    ch = small_channel()
    steps, every, seg = 300, 25, 40
    say("case adjoint sweep, form switched between segments")
    target = oracle_samples(ch.replace(gx=1.5e-5), steps, every)
    _, per_step = gpu_gradient(lb, ch, "f64", steps, every, seg, target, adjoint_block=1)
    P = ctypes.POINTER(ctypes.c_double)
    with lb.Solver([ch], precision="f64") as s:
        u, ckpts = adjoint.forward(s, steps, every, seg)
        dL = 2 * (u - target)
        rows = {t: dL[k] for k, t in enumerate(adjoint.sample_steps(steps, every))}
        nbytes = s.lib.lb_adjoint_workspace_bytes(s.h, seg)
        aws = torch.empty(int(nbytes), dtype=torch.uint8, device=s.device)
        _lib.check(s.lib.lb_adjoint_begin(s.h, ctypes.c_void_p(aws.data_ptr()), int(nbytes),
                                          seg), "lb_adjoint_begin")
        for i, (t0, snap) in enumerate(reversed(ckpts)):
            s.set_adjoint_block(32 if i % 2 == 0 else 1)
            n = min(seg, steps - t0)
            g = np.zeros((n, ch.ly))
            for j in range(n):
                if t0 + j in rows:
                    g[j] = rows[t0 + j]
            _lib.check(s.lib.lb_adjoint_segment(s.h, ctypes.c_void_p(snap.data_ptr()),
                                                g.ctypes.data_as(P), n), "lb_adjoint_segment")
        out = np.zeros((1, 4))
        _lib.check(s.lib.lb_adjoint_end(s.h, out.ctypes.data_as(P)), "lb_adjoint_end")
    rel = np.abs(out[0] - per_step) / np.abs(per_step)
    say(f"  alternating {out[0]}\n  per-step    {per_step}\n  rel {rel.max():.2e}")
    assert np.all(rel <= 1e-12), rel


def test_adjoint_block_setting(lb):
    """lb_set_adjoint_block takes 1 .. 32 and refuses the rest; channels
    wider than 512 nodes sweep per step whatever the setting."""
    from paper_1504_06123_amd import _lib
    say("case adjoint block setting")
    with lb.Solver([small_channel()], precision="f64") as s:
        assert s.adjoint_block == 32
        for bad in (0, -1, 33):
            assert s.lib.lb_set_adjoint_block(s.h, bad) == _lib.LB_EINVAL
            assert "adjoint block" in _lib.last_error()
        assert s.adjoint_block == 32
        s.set_adjoint_block(5)
        assert s.adjoint_block == 5
    for ly, form in ((512, 32), (513, 1), (1100, 1)):
        wide = workloads.Channel(lx=1, ly=ly, tau_lb=1.0, g_inf=1e-3, tau_m=10.0, gamma_c=0.1,
                                 n_hist=30, gx=1e-8)
        with lb.Solver([small_channel(), wide], precision="f64") as s:
            s.set_adjoint_block(32)
            assert s.adjoint_block == form, (ly, s.adjoint_block)


def test_adjoint_dot_product_above_1024_nodes(lb):
    """A 1 x 1100 channel (per-step sweep: too wide for the blocked one) in
    the UCM limit, linear in the body force: <J e_gx, w> = <u, w> / g_x."""
    from paper_1504_06123_amd import adjoint
    ch = workloads.Channel(lx=1, ly=1100, tau_lb=1.0, g_inf=1e-3, tau_m=10.0,
                           gamma_c=math.inf, n_hist=30, gx=1e-8)
    steps, every, seg = 120, 10, 30
    say("case adjoint dot product, 1x1100 UCM (per-step sweep)")
    with lb.Solver([ch], precision="f64") as s:
        assert s.adjoint_block == 1
        u, ckpts = adjoint.forward(s, steps, every, seg)
        w = _weights(u.shape, 1507)
        g = adjoint.backward(s, ckpts, steps, every, seg, w)[0]
    jv_w = float(np.sum(u * w) / ch.gx)
    scale = float(np.sum(np.abs(u * w)) / ch.gx)
    say(f"  <J e_gx, w> = {jv_w:.15e}, adjoint {g[3]:.15e}")
    assert abs(g[3] - jv_w) <= 1e-10 * scale


@pytest.mark.parametrize("precision,tol", [("f64", 1e-5), ("f32", 1e-4), ("f32p64", 1e-4)])
def test_adjoint_differentiation_run(lb, precision, tol):
    """1 x 128 channel, window 2048, 4000 steps, samples every 200, checkpoints
    every 256 steps, against the oracle's central differences (golden)."""
    path = os.path.join(GOLDEN, "differentiation.npz")
    if not os.path.exists(path):
        pytest.skip("differentiation.npz not generated")
    gold = np.load(path)
    wl = workloads.differentiation()
    ch = wl.channels[0]
    say(f"case adjoint differentiation run {precision}")
    u, g = gpu_gradient(lb, ch, precision, wl.steps, wl.sample_every, 256, gold["target"],
                        block=1 if precision == "f64" else 8)
    fd = gold["grad_fd"]
    rel = np.abs(g - fd) / np.abs(fd)
    uerr = np.abs(u - gold["u_p0"]).max() / np.abs(gold["u_p0"]).max()
    say(f"  u err {uerr:.2e}\n  fd {fd}\n  adjoint {g}\n  rel {rel}")
    assert np.all(rel < tol), rel
    assert uerr < {"f64": 1e-11, "f32p64": 1e-5, "f32": 1e-5}[precision], uerr


def test_lbfunction_autograd(lb):
    import torch
    from paper_1504_06123_amd import adjoint
    ch = small_channel()
    steps, every, seg = 200, 20, 50
    target = torch.from_numpy(oracle_samples(ch.replace(gx=1.5e-5), steps, every))
    say("case LBFunction")
    with lb.Solver([ch], precision="f64") as s:
        init = s.save_state()
        theta = torch.tensor([[ch.g_inf, ch.tau_m, ch.gamma_c, ch.gx]], dtype=torch.float64,
                             requires_grad=True)
        u = adjoint.LBFunction.apply(theta, s, init, steps, every, seg)
        loss = ((u - target) ** 2).sum()
        loss.backward()
        g_auto = theta.grad.numpy()[0]
    fd = oracle_fd(ch, target.numpy(), steps, every)
    rel = np.abs(g_auto - fd) / np.abs(fd)
    say(f"  rel {rel}")
    assert np.all(rel < 1e-5)


def test_repeated_sweeps_on_one_handle(lb):
    """The reverse sweep of a segment length is captured once and replayed for
    every segment and every later sweep on the handle; a new segment length
    (a new adjoint workspace layout) drops the captured sweeps.  Three
    gradients on one handle, from the same initial state: the first two with
    the same segment length, the third with another, all bitwise equal."""
    import torch
    from paper_1504_06123_amd import adjoint
    ch = small_channel()
    steps, every = 200, 20
    target = torch.from_numpy(oracle_samples(ch.replace(gx=1.5e-5), steps, every))
    say("case adjoint repeated sweeps on one handle")
    grads = []
    with lb.Solver([ch], precision="f64") as s:
        init = s.save_state()
        for seg in (50, 50, 23):
            theta = torch.tensor([[ch.g_inf, ch.tau_m, ch.gamma_c, ch.gx]], dtype=torch.float64,
                                 requires_grad=True)
            u = adjoint.LBFunction.apply(theta, s, init, steps, every, seg)
            ((u - target) ** 2).sum().backward()
            grads.append(theta.grad.numpy()[0].copy())
    say(f"  grads {grads}")
    assert np.array_equal(grads[0], grads[1])
    assert np.array_equal(grads[0], grads[2])


def test_channels_in_one_handle_match_single_channel_sweeps(lb):
    """Channels of one handle are independent: the gradient of a loss summed
    over two channels of different widths and parameters, swept together,
    equals each channel's gradient swept alone, bit for bit (same arithmetic
    in the same order per node, node-ordered reduction per channel)."""
    from paper_1504_06123_amd import adjoint
    c0 = small_channel()
    c1 = workloads.Channel(lx=1, ly=23, tau_lb=0.9, g_inf=1e-3, tau_m=25.0, gamma_c=0.08,
                           n_hist=48, gx=1.2e-5)
    steps, every, seg = 200, 20, 40
    say("case adjoint two channels in one handle")
    targets = [oracle_samples(c.replace(gx=0.8 * c.gx), steps, every) for c in (c0, c1)]
    with lb.Solver([c0, c1], precision="f64") as s:
        u, ckpts = adjoint.forward(s, steps, every, seg)
        g_both = adjoint.backward(s, ckpts, steps, every, seg,
                                  2 * (u - np.concatenate(targets, axis=1)))
    for i, c in enumerate((c0, c1)):
        _, g_one = gpu_gradient(lb, c, "f64", steps, every, seg, targets[i])
        say(f"  ch{i} together {g_both[i]}\n       alone    {g_one}")
        assert np.array_equal(g_both[i], g_one)


def test_long_segments_launch_directly(lb):
    """Segments longer than 1024 steps sweep with direct launches instead of a
    captured graph; the gradient is the same, bit for bit, as with short
    segments (the sweep's arithmetic does not depend on the segment length)."""
    ch = small_channel().replace(n_hist=1200, tau_m=300.0)
    steps, every = 1300, 100
    say("case adjoint segments of 1100 steps (direct) and 100 (graphs)")
    target = oracle_samples(ch.replace(gx=1.5e-5), steps, every)
    _, g_long = gpu_gradient(lb, ch, "f64", steps, every, 1100, target)
    _, g_short = gpu_gradient(lb, ch, "f64", steps, every, 100, target)
    say(f"  long {g_long}\n  short {g_short}")
    assert np.array_equal(g_long, g_short)


# ---------------------------------------------------------------------------
# Dot-product tests <J v, w> = <v, J^T w> in FP64, with J the derivative of
# the sampled velocities with respect to the parameters and J^T w the
# adjoint's gradient of L = <w, u>.  For linear models (Newtonian, and the
# UCM limit gamma_c = inf) the unidirectional channel is linear in the body
# force, u(g_x) = g_x u(1), so J e_gx = u / g_x exactly: the first test
# isolates the transpose of the lattice step (no history), the second adds
# the history transpose in its linear form.  The third takes J v of the
# nonlinear model from the GPU's own FP64 forward by Richardson-extrapolated
# central differences (error O(h^4)).
# ---------------------------------------------------------------------------

def _weights(shape, seed):
    return np.random.default_rng(seed).uniform(-1.0, 1.0, size=shape)


def _gpu_samples(lb, ch, steps, every):
    from paper_1504_06123_amd import adjoint
    with lb.Solver([ch], precision="f64") as s:
        u, _ = adjoint.forward(s, steps, every, steps)
    return u


@pytest.mark.parametrize("name,kw", [
    ("lattice_newtonian", dict(g_inf=0.0)),
    ("history_ucm", dict(gamma_c=math.inf)),
])
def test_adjoint_dot_product_linear(lb, name, kw):
    ch = small_channel().replace(**kw)
    steps, every, seg = 300, 10, 64
    say(f"case adjoint dot product, {name}")
    from paper_1504_06123_amd import adjoint
    with lb.Solver([ch], precision="f64") as s:
        u, ckpts = adjoint.forward(s, steps, every, seg)
        w = _weights(u.shape, 1504)
        g = adjoint.backward(s, ckpts, steps, every, seg, w)[0]
    jv_w = float(np.sum(u * w) / ch.gx)
    scale = float(np.sum(np.abs(u * w)) / ch.gx)
    say(f"  <J e_gx, w> = {jv_w:.15e}, adjoint {g[3]:.15e}, "
        f"diff/scale {abs(g[3] - jv_w) / scale:.2e}")
    assert abs(g[3] - jv_w) <= 1e-10 * scale


def test_adjoint_dot_product_nonlinear(lb):
    ch = small_channel()
    steps, every, seg = 300, 10, 64
    say("case adjoint dot product, nonlinear (nlM)")
    from paper_1504_06123_amd import adjoint
    with lb.Solver([ch], precision="f64") as s:
        u, ckpts = adjoint.forward(s, steps, every, seg)
        w = _weights(u.shape, 1505)
        g = adjoint.backward(s, ckpts, steps, every, seg, w)[0]
    p0 = np.array([getattr(ch, k) for k in workloads.ADJOINT_PARAMS])
    rng = np.random.default_rng(1506)
    for trial in range(3):
        # a direction with a relative component along every parameter
        v = p0 * rng.uniform(-1.0, 1.0, size=4)

        def at(h):
            return _gpu_samples(lb, ch.replace(**dict(zip(workloads.ADJOINT_PARAMS, p0 + h * v))),
                                steps, every)

        def central(h):
            return (at(h) - at(-h)) / (2.0 * h)

        h = 1e-3
        jv = (4.0 * central(h / 2) - central(h)) / 3.0
        lhs = float(np.sum(jv * w))
        rhs = float(np.dot(v, g))
        scale = float(np.sum(np.abs(jv * w)))
        say(f"  trial {trial}: <Jv, w> {lhs:.12e}, <v, J^T w> {rhs:.12e}, "
            f"diff/scale {abs(lhs - rhs) / scale:.2e}")
        assert abs(lhs - rhs) <= 1e-9 * scale
