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


def _run(Solver, chans, precision, block, fused, steps, graph=0):
    with Solver(chans, precision=precision) as s:
        s.set_block(block)
        s.set_fused(fused)
        if graph:
            s.set_graph(graph)
        assert s.fused == (fused and block > 1)
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
    chans = workloads.batched().channels[:12]
    say(f"case fused batched 12 channels {precision} block {block}")
    a = _run(Solver, chans, precision, block, False, 203)
    b = _run(Solver, chans, precision, block, True, 203)
    _same(a, b)


def test_fused_equals_separate_launches_mixed_kinds(Solver):
    """Full tensor, accumulated-strain damping and the paper's coupling on
    small 2D channels, with a unidirectional integral-law channel."""
    base = workloads.large_2d(lx=6, ly=20, n_hist=150).channels[0]
    chans = [base.replace(finger=True, tau_m=20.0),
             base.replace(law="strain_damping", tau_m=25.0),
             base.replace(paper_coupling=True, tau_m=30.0),
             workloads.plain_f64().channels[0].replace(lx=1, ly=40)]
    say("case fused mixed kinds f32p64 block 8")
    a = _run(Solver, chans, "f32p64", 8, False, 150)
    b = _run(Solver, chans, "f32p64", 8, True, 150)
    _same(a, b)


def test_fused_save_load_mid_span_and_graph(Solver):
    chans = workloads.batched().channels[:6]
    say("case fused save/load mid-span + graph, f32 block 16")
    with Solver(chans, precision="f32") as s:
        s.set_block(16)
        assert s.fused
        s.step(53)                     # 5 steps into a block
        buf = s.save_state()
        s.step(40)
        want = [s.fields(i) + s.stress(i) for i in range(len(chans))]
        s.step(7)
        s.load_state(buf)
        s.step(40)
        got = [s.fields(i) + s.stress(i) for i in range(len(chans))]
    _same(want, got)
    a = _run(Solver, chans, "f32", 16, True, 256)
    b = _run(Solver, chans, "f32", 16, True, 256, graph=64)
    _same(a, b)


def test_fused_only_when_every_channel_fits(Solver):
    small = workloads.plain_f64().channels[0].replace(lx=1, ly=64)
    wide = workloads.large_2d(lx=40, ly=30, n_hist=64).channels[0]    # 1200 nodes
    grid = small.replace(hist_blocks=2, hist_block_len=8)
    inst = small.replace(law="instantaneous")
    for chans, want in (([small], True), ([small, wide], False), ([small, grid], False),
                        ([small, inst], False)):
        with Solver(chans, precision="f32") as s:
            s.set_block(8)
            assert s.fused == want
            s.set_block(1)
            assert not s.fused          # no in-block steps to fuse
            s.set_block(8)
            s.set_fused(False)
            assert not s.fused
