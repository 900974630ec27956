"""GPU parity of the alternative constitutive laws against the FP64 oracle:
the accumulated-strain damping variant of Sec. II (blocked passes with the
common per-step factor) and the instantaneous law of Eq. inlM.

Same error metric and tolerances as test_gpu_parity.
"""
import numpy as np
import pytest

import workloads
from test_gpu_parity import (TOL32, TOL64, Solver, compare, nerr, run_gpu,  # noqa: F401
                             run_oracle, say)

pytestmark = pytest.mark.gpu


def _twod(lx, ly, n_hist, **kw):
    ch = workloads.large_2d(lx=lx, ly=ly, n_hist=n_hist).channels[0]
    return ch.replace(u0=ch.u0 * 30.0, gx=2e-5, **kw)


@pytest.mark.parametrize("precision", ["f64", "f32p64", "f32"])
@pytest.mark.parametrize("block", [1, 8, 32])
def test_strain_damping_matches_oracle(Solver, precision, block):
    ch = _twod(6, 11, 200, tau_m=40.0, gamma_c=0.02, law="strain_damping")
    say(f"case strain damping 6x11 {precision} block {block}")
    ref = run_oracle([ch], 400, 50, steps_on=250)[0]
    got = run_gpu(Solver, [ch], precision, 400, 50, steps_on=250, block=block)[0]
    compare(got, ref, TOL64 if precision == "f64" else TOL32, keys=("ux", "uy", "sxy", "n1"),
            label=f"strain damping {precision} M={block}")


def test_strain_damping_short_windows_and_ucm(Solver):
    for H, gc in ((2, 0.05), (7, 0.05), (40, float("inf"))):
        ch = workloads.plain_f64().channels[0].replace(lx=1, ly=10, n_hist=H, tau_m=6.0,
                                                       gamma_c=gc, gx=4e-5,
                                                       law="strain_damping")
        say(f"case strain damping window {H} gamma_c {gc}")
        ref = run_oracle([ch], 250, 25)[0]
        for M in (1, 4, 32):
            got = run_gpu(Solver, [ch], "f64", 250, 25, block=M)[0]
            compare(got, ref, TOL64, label=f"strain damping H={H} M={M}")


@pytest.mark.parametrize("precision", ["f64", "f32p64", "f32"])
def test_instantaneous_law_matches_oracle(Solver, precision):
    ch = _twod(6, 11, 2, tau_m=20.0, law="instantaneous")
    say(f"case instantaneous 6x11 {precision}")
    ref = run_oracle([ch], 400, 50, steps_on=250)[0]
    got = run_gpu(Solver, [ch], precision, 400, 50, steps_on=250, block=8)[0]
    compare(got, ref, TOL64 if precision == "f64" else TOL32, keys=("ux", "uy", "sxy", "n1"),
            label=f"instantaneous {precision}")


def test_laws_mixed_in_one_handle(Solver):
    """Three channels with three laws advance together, blocked by 8."""
    chans = [workloads.plain_f64().channels[0].replace(lx=1, ly=12, n_hist=150, tau_m=20.0,
                                                       gx=4e-5, law=law)
             for law in ("nlm", "strain_damping", "instantaneous")]
    say("case three laws in one handle")
    ref = run_oracle(chans, 300, 50)
    got = run_gpu(Solver, chans, "f64", 300, 50, block=8)
    for c, (g, r) in enumerate(zip(got, ref)):
        compare(g, r, TOL64, label=f"law channel {c}")
