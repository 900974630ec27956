"""GPU parity of the full-tensor Finger path (Eq. gitt with -d_t'B =
E kappa E^T + transpose, Eq. eeval) against the FP64 oracle's own
implementation, through the C interface.

Same error metric and tolerances as test_gpu_parity.
"""
import numpy as np
import pytest

import workloads
from test_gpu_parity import (TOL32, TOL64, Solver, compare, nerr, run_gpu,  # noqa: F401
                             run_oracle, say)

pytestmark = pytest.mark.gpu

KEYS = ("ux", "uy", "sxy", "n1")


def _twod(lx, ly, n_hist, **kw):
    ch = workloads.large_2d(lx=lx, ly=ly, n_hist=n_hist).channels[0]
    # a perturbation a hundred times the recipe's: velocity gradients of all
    # four kinds matter over the run
    return ch.replace(u0=ch.u0 * 100.0, finger=True, gx=2e-5, **kw)


@pytest.mark.parametrize("precision", ["f64", "f32p64", "f32"])
def test_finger_2d_matches_oracle(Solver, precision):
    ch = _twod(6, 11, 120, tau_m=30.0)
    say(f"case finger 2d 6x11 {precision}")
    ref = run_oracle([ch], 400, 50, steps_on=250)[0]
    got = run_gpu(Solver, [ch], precision, 400, 50, steps_on=250)[0]
    assert np.abs(ref["n1"]).max() > 0
    compare(got, ref, TOL64 if precision == "f64" else TOL32, keys=KEYS,
            label=f"finger 2d {precision}")


def test_finger_chunked_and_blocked_f64(Solver):
    """Window split into age ranges (FP64 congruence combine) and temporal
    blocking (deformation since the pass as a common factor): rounding-order
    changes only."""
    ch = _twod(5, 9, 420, tau_m=40.0)
    say("case finger chunked + blocked f64")
    ref = run_oracle([ch], 360, 40)[0]
    base = run_gpu(Solver, [ch], "f64", 360, 40)[0]
    compare(base, ref, TOL64, keys=KEYS, label="finger base")
    for chunks in (1, 3):
        for M in (2, 4, 8, 16):
            got = run_gpu(Solver, [ch], "f64", 360, 40, chunks=[chunks], block=M)[0]
            compare(got, ref, TOL64, keys=KEYS, label=f"finger chunks={chunks} M={M}")
            for k in ("ux", "sxy", "n1"):
                assert nerr(got[k], base[k]) < 1e-12, (chunks, M, k)


def test_finger_short_windows_blocked(Solver):
    for H in (2, 5, 9):
        ch = _twod(3, 8, H, tau_m=4.0)
        say(f"case finger window {H}")
        ref = run_oracle([ch], 200, 25)[0]
        for M in (1, 4, 16):
            got = run_gpu(Solver, [ch], "f64", 200, 25, block=M)[0]
            compare(got, ref, TOL64, keys=KEYS, label=f"finger H={H} M={M}")


def test_finger_f32_blocked_2d(Solver):
    ch = _twod(24, 16, 512, tau_m=100.0)
    say("case finger f32 24x16 window 512")
    ref = run_oracle([ch], 600, 100)[0]
    for prec in ("f32p64", "f32"):
        for M in (1, 16):
            got = run_gpu(Solver, [ch], prec, 600, 100, block=M)[0]
            compare(got, ref, TOL32, keys=KEYS, label=f"finger 24x16 {prec} M={M}")


def test_finger_unidirectional_equals_reduced_oracle(Solver):
    """For unidirectional flow the full tensor reduces exactly to the simple
    shear path: the GPU full-tensor run matches the reduced oracle."""
    base = workloads.plain_f64().channels[0].replace(lx=1, ly=20, n_hist=200, tau_m=40.0,
                                                     gx=4e-5)
    say("case finger unidirectional vs reduced oracle")
    ref = run_oracle([base], 300, 50, steps_on=200)[0]
    got = run_gpu(Solver, [base.replace(finger=True)], "f64", 300, 50, steps_on=200,
                  block=8)[0]
    compare(got, ref, TOL64, keys=("ux", "sxy", "n1"), label="finger uni")


def test_finger_persistent_graph_save_load_bitwise(Solver):
    ch = _twod(8, 12, 200, tau_m=40.0)
    say("case finger persistent / graph / save-load")
    a = run_gpu(Solver, [ch], "f32", 256, 64, block=8)[0]
    b = run_gpu(Solver, [ch], "f32", 256, 64, block=8, persistent=True)[0]
    c = run_gpu(Solver, [ch], "f32", 256, 64, block=8, graph=32)[0]
    for k in a:
        assert np.array_equal(a[k], b[k]), ("persistent", k)
        assert np.array_equal(a[k], c[k]), ("graph", k)
    with Solver([ch], precision="f32") as s:
        s.set_block(8)
        s.step(150)
        buf = s.save_state()
        s.step(77)
        want = s.fields(0), s.stress(0)
        s.step(3)
        s.load_state(buf)
        s.step(77)
        got = s.fields(0), s.stress(0)
    for x, y in zip(want, got):
        for u, v in zip(x, y):
            assert np.array_equal(u, v)


def test_finger_limits(Solver):
    from paper_1504_06123_amd import _lib
    ch = _twod(4, 8, 64)
    with Solver([ch], precision="f64") as s:
        with pytest.raises(_lib.LBError):
            s.set_block(32)
        s.set_block(16)
        assert s.lib.lb_adjoint_workspace_bytes(s.h, 8) == 0
        assert "Finger" in _lib.last_error()


def test_finger_full_size_x_invariant_against_column(Solver):
    """The unperturbed 1024 x 512 channel with the full tensor, 5000 steps in
    16-step passes: x-invariant flow, every column equals the stored FP64
    oracle column of the reduced path (the full tensor reduces to it)."""
    import os
    from test_gpu_long_runs import GOLDEN, tolerance  # noqa: F401
    path = os.path.join(GOLDEN, "large_2d_column.npz")
    if not os.path.exists(path):
        pytest.skip("large_2d_column.npz not generated")
    gold = np.load(path)
    ch = workloads.large_2d(perturb=False).channels[0].replace(finger=True)
    steps, every = int(gold["steps"]), int(gold["sample_every"])
    say(f"case finger full size 1024x512, {steps} steps, f32p64")
    got = run_gpu(Solver, [ch], "f32p64", steps, every, block=16, persistent=True)[0]
    for k in ("ux", "sxy", "n1"):
        g = got[k]
        spread = float(np.abs(g - g[:, :, :1]).max() / np.abs(g).max())
        assert spread <= 1e-12, (k, spread)
        ref = gold[f"c0_{k}"].reshape(g[:, :, :1].shape)
        err = nerr(g[:, :, :1], ref)
        say(f"  finger full size {k}: {err:.2e}")
        assert err <= (1e-5 if k == "ux" else 1e-4), (k, err)
