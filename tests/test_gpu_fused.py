"""Fused in-block steps: when every channel of a handle fits one workgroup,
the steps of a block after its history pass run as one launch (lattice and
in-block history phases per step, workgroup barriers between them).  Same
per-node arithmetic as the separate launches, so results must be identical
bit for bit; the fused runs are also compared with the oracle by the other
GPU tests, whose small blocked handles take this path by default."""
import math

import numpy as np
import pytest

import workloads
from test_gpu_parity import Solver, say  # noqa: F401

pytestmark = pytest.mark.gpu


def _run(Solver, chans, precision, block, mode, steps, graph=0, want=None):
    with Solver(chans, precision=precision) as s:
        s.set_block(block)
        s.set_fused(mode)
        if graph:
            s.set_graph(graph)
        if want is not None:
            assert s.fused == want
        out = []
        done = 0
        for k in (steps // 3, steps // 3 + 5, steps):
            s.step(k - done)
            done = k
            for ci in range(len(chans)):
                out.append(s.fields(ci) + s.stress(ci))
        return out


def _same(a, b):
    for x, y in zip(a, b):
        for p, q in zip(x, y):
            assert np.array_equal(p, q)


@pytest.mark.parametrize("precision", ["f64", "f32p64", "f32"])
@pytest.mark.parametrize("block", [2, 8, 32])
def test_fused_equals_separate_launches_batched(Solver, precision, block):
    """Separate launches, the fused launch, and (LB_F32) its LDS form.  With
    FP64 populations the default (mode 1) runs these channels -- three are
    wider than 512 nodes -- in separate launches; mode 2 forces the
    global-memory fused form."""
    chans = workloads.batched().channels[:12]
    say(f"case fused batched 12 channels {precision} block {block}")
    a = _run(Solver, chans, precision, block, 0, 203, want=0)
    b = _run(Solver, chans, precision, block, 2, 203, want=1)
    c = _run(Solver, chans, precision, block, 1, 203, want=2 if precision == "f32" else 0)
    _same(a, b)
    _same(a, c)


@pytest.mark.parametrize("block", [4, 32])
def test_fused_lds_form_short_windows_and_limits(Solver, block):
    """The LDS form (unidirectional channels) with a window shorter than the
    block, a chunked window and a channel at the 1024-node limit; 2D channels
    of the same sizes take the global-memory fused form (mode 2: by default
    it runs only up to 512 nodes per channel).  Both equal the separate
    launches bit for bit."""
    def uni(ly, n_hist, tau_m):
        return workloads.plain_f64().channels[0].replace(lx=1, ly=ly, n_hist=n_hist,
                                                         tau_m=tau_m, gx=2e-5)

    def twod(lx, ly, n_hist, tau_m):
        return workloads.large_2d(lx=lx, ly=ly, n_hist=n_hist).channels[0].replace(tau_m=tau_m)

    for kind, chans, fused_mode, want in (
            ("unidirectional", [uni(16, 300, 20.0),
                                uni(13, 3, 15.0),       # window shorter than the block
                                uni(1024, 64, 30.0),    # 1024 nodes
                                uni(40, 2000, 100.0)], 1, 2),
            ("2D", [twod(8, 16, 300, 20.0),
                    twod(5, 13, 3, 15.0),
                    twod(32, 32, 64, 30.0),
                    uni(40, 2000, 100.0)], 2, 1)):
        say(f"case fused form, {kind} channels, f32 block {block}")
        runs = []
        for mode in (fused_mode, 0):
            with Solver(chans, precision="f32") as s:
                s.set_tiling(3, 4)     # the long window split into 4 age chunks
                s.set_block(block)
                s.set_fused(mode)
                assert s.fused == (want if mode else 0)
                out = []
                done = 0
                for k in (50, 55, 150):
                    s.step(k - done)
                    done = k
                    for ci in range(len(chans)):
                        out.append(s.fields(ci) + s.stress(ci))
                runs.append(out)
        _same(runs[1], runs[0])


def test_fused_equals_separate_launches_mixed_kinds(Solver):
    """Full tensor, accumulated-strain damping and the paper's coupling on
    small 2D channels, with a unidirectional integral-law channel."""
    base = workloads.large_2d(lx=6, ly=20, n_hist=150).channels[0]
    chans = [base.replace(finger=True, tau_m=20.0),
             base.replace(law="strain_damping", tau_m=25.0),
             base.replace(paper_coupling=True, tau_m=30.0),
             workloads.plain_f64().channels[0].replace(lx=1, ly=40)]
    for precision in ("f32p64", "f32"):
        say(f"case fused mixed kinds {precision} block 8")
        a = _run(Solver, chans, precision, 8, 0, 150, want=0)
        b = _run(Solver, chans, precision, 8, 1, 150, want=1)   # no LDS form here
        _same(a, b)


def test_fused_save_load_mid_span_and_graph(Solver):
    chans = workloads.batched().channels[:6]
    say("case fused save/load mid-span + graph, f32 block 16")
    with Solver(chans, precision="f32") as s:
        s.set_block(16)
        assert s.fused == 2
        s.step(53)                     # 5 steps into a block
        buf = s.save_state()
        s.step(40)
        want = [s.fields(i) + s.stress(i) for i in range(len(chans))]
        s.step(7)
        s.load_state(buf)
        s.step(40)
        got = [s.fields(i) + s.stress(i) for i in range(len(chans))]
    _same(want, got)
    a = _run(Solver, chans, "f32", 16, 1, 256)
    b = _run(Solver, chans, "f32", 16, 1, 256, graph=64)
    _same(a, b)


def test_fused_only_when_every_channel_fits(Solver):
    small = workloads.plain_f64().channels[0].replace(lx=1, ly=64)
    wide = workloads.large_2d(lx=40, ly=30, n_hist=64).channels[0]    # 1200 nodes
    grid = small.replace(hist_blocks=2, hist_block_len=8)
    inst = small.replace(law="instantaneous")
    damped = small.replace(law="strain_damping")
    for chans, prec, want in (([small], "f32", 2), ([small], "f32p64", 1), ([small], "f64", 1),
                              ([small, damped], "f32", 1), ([small, wide], "f32", 0),
                              ([small, grid], "f32", 0), ([small, inst], "f32", 0)):
        with Solver(chans, precision=prec) as s:
            s.set_block(8)
            assert s.fused == want
            s.set_block(1)
            assert s.fused == 0         # no in-block steps to fuse
            s.set_block(8)
            s.set_fused(2)
            assert s.fused == min(want, 1)
            s.set_fused(0)
            assert s.fused == 0
    # FP64 populations above 512 nodes: separate launches by default (the
    # global-memory fused form is slower there), fused on request
    wide_uni = small.replace(ly=600)
    for prec in ("f32p64", "f64"):
        with Solver([small, wide_uni], precision=prec) as s:
            s.set_block(8)
            assert s.fused == 0
            s.set_fused(2)
            assert s.fused == 1
    with Solver([small, wide_uni], precision="f32") as s:
        s.set_block(8)
        assert s.fused == 2


def test_fused_set_params_and_force_mid_block(Solver):
    """A parameter change inside a block restarts the block with a fresh pass
    and a force change cuts a fused span: the LDS form and separate launches
    stay identical across both."""
    chans = workloads.batched().channels[:5]
    say("case fused set_params / set_force mid-block, f32 block 16")
    res = []
    for mode in (0, 1):
        with Solver(chans, precision="f32") as s:
            s.set_block(16)
            s.set_fused(mode)
            s.step(21)                                  # 5 steps into a block
            for ci in range(len(chans)):
                s.lib.lb_set_params(s.h, ci, 3e-3, 80.0, 0.07)
            s.step(11)
            s.set_force(2, 0.0)
            s.step(30)
            res.append([s.fields(ci) + s.stress(ci) for ci in range(len(chans))])
    _same(res[0], res[1])
