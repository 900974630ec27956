"""GPU parity of the quasi-logarithmic history grid (Sec. III) against the
FP64 oracle's own implementation of the grid, through the C interface.

Same error metric and tolerances as test_gpu_parity: FP64 1e-10, FP32 and
mixed 1e-5 for velocity and 1e-4 for sigma_xy and N1.
"""
import math

import numpy as np
import pytest

import workloads
from test_gpu_parity import (TOL32, TOL64, Solver, compare, nerr, run_gpu,  # noqa: F401
                             run_oracle, say)

pytestmark = pytest.mark.gpu


def _uni(ly, B, C, **kw):
    base = workloads.plain_f64().channels[0]
    return base.replace(lx=1, ly=ly, hist_blocks=B, hist_block_len=C, **kw)


def _twod(lx, ly, B, C, **kw):
    ch = workloads.large_2d(lx=lx, ly=ly, n_hist=2).channels[0]
    return ch.replace(hist_blocks=B, hist_block_len=C, gx=3e-5, **kw)


CASES = {
    # name: (channel, steps, steps_on, sample interval)
    "uni_b3_c8": (_uni(24, 3, 8, tau_m=30.0, gx=4e-5), 400, 250, 50),
    "uni_min_c2_b4": (_uni(9, 4, 2, tau_m=12.0, gx=4e-5), 300, 180, 30),
    "one_block_c7": (_twod(3, 8, 1, 7, tau_m=9.0), 200, 140, 20),
    "2d_b2_odd_c5": (_twod(6, 11, 2, 5, tau_m=20.0), 300, 200, 50),
    "2d_ucm_b3_c6": (_twod(5, 9, 3, 6, tau_m=25.0, gamma_c=math.inf), 300, 300, 50),
    "paper_c128_b4": (_uni(40, 4, 128, tau_m=200.0, gx=2e-5), 2500, 1500, 250),
}


@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("precision", ["f64", "f32p64", "f32"])
def test_grid_matches_oracle(Solver, name, precision):
    ch, steps, on, every = CASES[name]
    say(f"case grid {name} {precision}")
    ref = run_oracle([ch], steps, every, steps_on=on)[0]
    got = run_gpu(Solver, [ch], precision, steps, every, steps_on=on)[0]
    keys = ("ux", "uy", "sxy", "n1") if ch.lx > 1 else ("ux", "sxy", "n1")
    compare(got, ref, TOL64 if precision == "f64" else TOL32, keys=keys,
            label=f"grid {name} {precision}")


def test_grid_and_window_channels_in_one_handle_with_blocking(Solver):
    """A grid channel steps every step while a window channel in the same
    handle takes 8-step history passes; both match their oracles."""
    grid = _uni(20, 3, 8, tau_m=30.0, gx=4e-5)
    win = workloads.large_2d(lx=4, ly=10, n_hist=300).channels[0].replace(tau_m=40.0)
    say("case grid + window, block 8")
    ref = run_oracle([grid, win], 320, 40, steps_on=200)
    got = run_gpu(Solver, [grid, win], "f64", 320, 40, steps_on=200, block=8)
    compare(got[0], ref[0], TOL64, label="grid channel")
    compare(got[1], ref[1], TOL64, keys=("ux", "uy", "sxy", "n1"), label="window channel")


def test_grid_save_load_and_graph_are_bitwise(Solver):
    ch = _twod(6, 10, 3, 6, tau_m=20.0)
    say("case grid save/load + graph")
    with Solver([ch], precision="f32") as s:
        s.step(77)
        buf = s.save_state()
        s.step(61)
        want = s.fields(0), s.stress(0)
        s.step(5)
        s.load_state(buf)
        s.step(61)
        got = s.fields(0), s.stress(0)
    for a, b in zip(want, got):
        for x, y in zip(a, b):
            assert np.array_equal(x, y)
    a = run_gpu(Solver, [ch], "f32", 256, 64)[0]
    b = run_gpu(Solver, [ch], "f32", 256, 64, graph=32)[0]
    for k in a:
        assert np.array_equal(a[k], b[k]), k


def test_grid_full_size_x_invariant_against_column(Solver):
    """The 1024 x 512 channel on the paper's grid (C = 128, B = 6: 8064 steps
    of reach) without perturbation stays x-invariant; every column matches
    the oracle run of one column."""
    ch = workloads.large_2d(perturb=False).channels[0].replace(hist_blocks=6,
                                                                hist_block_len=128)
    col = ch.replace(lx=1)
    steps, every = 300, 100
    say("case grid full size 1024x512 B=6 C=128, 300 steps, f32p64")
    ref = run_oracle([col], steps, every)[0]
    got = run_gpu(Solver, [ch], "f32p64", steps, every)[0]
    for k in ("ux", "sxy", "n1"):
        g = got[k]                                   # [samples][ly][lx]
        spread = float(np.abs(g - g[:, :, :1]).max() / np.abs(g).max())
        assert spread <= 1e-12, (k, spread)
    colgot = {k: got[k][:, :, :1] for k in ("ux", "uy", "sxy", "n1")}
    compare(colgot, ref, TOL32, label="grid full size column")


def test_grid_channels_have_no_adjoint(Solver):
    from paper_1504_06123_amd import _lib
    with Solver([_uni(16, 2, 4)], precision="f64") as s:
        assert s.lib.lb_adjoint_workspace_bytes(s.h, 8) == 0
        assert "grid" in _lib.last_error()


# Temporal blocking on the grid: the entries each grid block holds through a
# block of M = min(steps per pass, 16) steps with the same neighbours go into
# one pass; the others are visited every step.  Needs C >= M + 2 (shorter
# grid blocks fall back to the full walk).
BLOCKED = {
    # name: (channel, steps, steps_on, sample interval, steps per pass)
    "uni_b3_c8_m2": (_uni(24, 3, 8, tau_m=30.0, gx=4e-5), 400, 250, 50, 2),
    "uni_b3_c8_m4": (_uni(24, 3, 8, tau_m=30.0, gx=4e-5), 400, 250, 50, 4),
    "2d_b2_odd_c5_m2": (_twod(6, 11, 2, 5, tau_m=20.0), 300, 200, 50, 2),
    "2d_b3_c10_m8": (_twod(5, 9, 3, 10, tau_m=15.0), 333, 203, 37, 8),
    "2d_ucm_b4_c19_m16": (_twod(4, 9, 4, 19, tau_m=25.0, gamma_c=math.inf), 500, 300, 50, 16),
    "uni_b5_c21_m32": (_uni(16, 5, 21, tau_m=40.0, gx=4e-5), 700, 450, 70, 32),
    "paper_c128_b4_m32": (_uni(40, 4, 128, tau_m=200.0, gx=2e-5), 2500, 1500, 250, 32),
}


@pytest.mark.parametrize("name", list(BLOCKED))
@pytest.mark.parametrize("precision", ["f64", "f32p64", "f32"])
def test_blocked_grid_matches_oracle(Solver, name, precision):
    ch, steps, on, every, block = BLOCKED[name]
    say(f"case blocked grid {name} {precision}")
    ref = run_oracle([ch], steps, every, steps_on=on)[0]
    got = run_gpu(Solver, [ch], precision, steps, every, steps_on=on, block=block)[0]
    keys = ("ux", "uy", "sxy", "n1") if ch.lx > 1 else ("ux", "sxy", "n1")
    compare(got, ref, TOL64 if precision == "f64" else TOL32, keys=keys,
            label=f"blocked grid {name} {precision}")


@pytest.mark.parametrize("block", [2, 8, 16, 32])
def test_blocked_grid_equals_unblocked_in_fp64(Solver, block):
    """Blocking re-associates the same sums: in FP64 the blocked and the
    unblocked grid agree to rounding (the only other difference is the FP64
    rounding of the averaged shear rate of a combination inside a block)."""
    ch = _twod(5, 12, 3, 34, tau_m=30.0)
    say(f"case blocked grid vs unblocked, block {block}")
    a = run_gpu(Solver, [ch], "f64", 410, 41, steps_on=260)[0]
    b = run_gpu(Solver, [ch], "f64", 410, 41, steps_on=260, block=block)[0]
    for k in ("ux", "uy", "sxy", "n1"):
        assert nerr(b[k], a[k]) <= 1e-12, (k, nerr(b[k], a[k]))


def test_blocked_grid_save_load_mid_block_and_graph_are_bitwise(Solver):
    ch = _twod(6, 10, 3, 12, tau_m=20.0)
    say("case blocked grid save/load mid-block + graph")
    with Solver([ch], precision="f32") as s:
        s.set_block(8)
        s.step(77)           # 5 steps into a block
        buf = s.save_state()
        s.step(61)
        want = s.fields(0), s.stress(0)
        s.step(5)
        s.load_state(buf)
        s.step(61)
        got = s.fields(0), s.stress(0)
    for a, b in zip(want, got):
        for x, y in zip(a, b):
            assert np.array_equal(x, y)
    a = run_gpu(Solver, [ch], "f32", 256, 64, block=8)[0]
    b = run_gpu(Solver, [ch], "f32", 256, 64, block=8, graph=32)[0]
    for k in a:
        assert np.array_equal(a[k], b[k]), k


def test_set_params_mid_block_starts_a_new_block(Solver):
    """A parameter change inside a block must not reuse block sums formed
    with the old decay rates: blocked runs (grid and window channel in one
    handle) agree with unblocked ones in FP64 across the change."""
    grid = _twod(4, 9, 3, 20, tau_m=25.0)
    win = workloads.large_2d(lx=4, ly=9, n_hist=200).channels[0].replace(tau_m=30.0)
    say("case set_params mid-block, block 16")
    res = []
    for block in (1, 16):
        with Solver([grid, win], precision="f64") as s:
            s.set_block(block)
            s.step(29)       # 13 steps into the second block
            for ci in range(2):
                s.lib.lb_set_params(s.h, ci, 2e-3, 12.0, 0.05)
            s.step(40)
            res.append([s.stress(ci) + s.fields(ci) for ci in range(2)])
    for ci in range(2):
        for x, y in zip(res[0][ci], res[1][ci]):
            assert nerr(y, x) <= 1e-12, (ci, nerr(y, x))


def test_blocked_grid_full_size_bench_launch(Solver):
    """The 1024 x 512 channel on the grid (C = 128, B = 6) in the launch the
    benchmark times (32 steps per pass, persistent, 64-step graphs): stays
    x-invariant without perturbation and every column matches the oracle."""
    ch = workloads.large_2d(perturb=False).channels[0].replace(hist_blocks=6,
                                                                hist_block_len=128)
    col = ch.replace(lx=1)
    steps, every = 320, 64
    say("case blocked grid full size 1024x512 B=6 C=128, 320 steps, f32p64, block 32")
    ref = run_oracle([col], steps, every)[0]
    got = run_gpu(Solver, [ch], "f32p64", steps, every, block=32, persistent=True,
                  graph=64)[0]
    for k in ("ux", "sxy", "n1"):
        g = got[k]
        spread = float(np.abs(g - g[:, :, :1]).max() / np.abs(g).max())
        assert spread <= 1e-12, (k, spread)
    colgot = {k: got[k][:, :, :1] for k in ("ux", "uy", "sxy", "n1")}
    compare(colgot, ref, TOL32, label="blocked grid full size column")
