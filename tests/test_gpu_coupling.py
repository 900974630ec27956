"""GPU parity of the paper's own stress coupling (Eq. bodyforce with the
density rate d_t delta rho, Eq. hydrofields) against the FP64 oracle.

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
    return ch.replace(u0=ch.u0 * 50.0, paper_coupling=True, gx=2e-5, **kw)


@pytest.mark.parametrize("precision", ["f64", "f32p64", "f32"])
def test_paper_coupling_2d_matches_oracle(Solver, precision):
    ch = _twod(6, 11, 150, tau_m=30.0)
    say(f"case paper coupling 2d {precision}")
    ref = run_oracle([ch], 400, 50, steps_on=250)[0]
    got = run_gpu(Solver, [ch], precision, 400, 50, steps_on=250)[0]
    keys = ("ux", "uy", "rho", "sxy", "n1")
    tol = TOL64 if precision == "f64" else dict(TOL32, rho=1e-5)
    if precision != "f64":
        got = dict(got, rho=got["rho"] - 1.0)
        ref = dict(ref, rho=ref["rho"] - 1.0)
    compare(got, ref, tol, keys=keys, label=f"paper coupling {precision}")


@pytest.mark.parametrize("block", [1, 8, 32])
def test_paper_coupling_unidirectional_blocked(Solver, block):
    ch = workloads.plain_f64().channels[0].replace(lx=1, ly=24, n_hist=300, tau_m=40.0,
                                                   gx=4e-5, paper_coupling=True)
    say(f"case paper coupling 1x24 block {block}")
    ref = run_oracle([ch], 500, 50, steps_on=300)[0]
    got = run_gpu(Solver, [ch], "f64", 500, 50, steps_on=300, block=block)[0]
    compare(got, ref, TOL64, keys=("ux", "sxy", "n1"), label=f"paper coupling uni M={block}")


def test_paper_coupling_with_full_tensor(Solver):
    ch = _twod(5, 9, 120, tau_m=25.0, finger=True)
    say("case paper coupling + full tensor")
    ref = run_oracle([ch], 300, 50)[0]
    got = run_gpu(Solver, [ch], "f64", 300, 50, block=8)[0]
    compare(got, ref, TOL64, keys=("ux", "uy", "sxy", "n1"), label="paper coupling finger")


def test_paper_coupling_save_load_bitwise(Solver):
    """The lagged trace is part of the state: a resumed run is identical."""
    ch = _twod(8, 12, 100, tau_m=30.0)
    with Solver([ch], precision="f32") as s:
        s.set_block(4)
        s.step(101)
        buf = s.save_state()
        s.step(40)
        want = s.fields(0), s.stress(0)
        s.step(7)
        s.load_state(buf)
        s.step(40)
        got = s.fields(0), s.stress(0)
    for x, y in zip(want, got):
        for u, v in zip(x, y):
            assert np.array_equal(u, v)
