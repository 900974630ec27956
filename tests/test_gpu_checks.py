"""Failure detection at readouts on the GPU, forced from the host: a channel
driven by a finite but enormous body force overflows (u^2 in the equilibrium
becomes infinite, then NaN; no kernel indexes by value, so every kernel
still runs normally) and its readouts return LB_ENONFINITE; a channel
accelerated past |u| = 0.1 raises the Mach guard as a warning."""
import os
import warnings

import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu


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


@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_diverging_run_returns_enonfinite(lb, precision):
    from paper_1504_06123_amd import _lib
    ch = workloads.plain_f64().channels[0].replace(lx=2, ly=8, n_hist=16, gx=1e200)
    say(f"case diverging run, {precision}")
    with lb.Solver([ch], precision=precision) as s:
        s.step(5)
        with pytest.raises(_lib.LBError) as e:
            s.stress(0)
        assert e.value.status == _lib.LB_ENONFINITE
        with warnings.catch_warnings():
            warnings.simplefilter("ignore")
            with pytest.raises(_lib.LBError) as e:
                s.fields(0)
        assert e.value.status == _lib.LB_ENONFINITE
        # the handle stays usable; with the check off the values come back
        s.set_checks(finite=False, mach=False)
        sxy, _ = s.stress(0)
        assert not np.isfinite(sxy).all()
        s.step(1)


def test_mach_guard_warns(lb):
    from paper_1504_06123_amd import MachWarning
    ch = workloads.plain_f64().channels[0].replace(lx=1, ly=8, n_hist=16, gx=4e-3, g_inf=0.0)
    say("case Mach guard")
    with lb.Solver([ch], precision="f64") as s:
        s.step(10)                       # |u| about 0.04
        with warnings.catch_warnings():
            warnings.simplefilter("error")
            _, ux, _ = s.fields(0)
        assert np.abs(ux).max() < 0.1
        s.step(190)                      # |u| near its steady 0.19
        with pytest.warns(MachWarning):
            _, ux, _ = s.fields(0)
        assert np.abs(ux).max() > 0.1 and np.isfinite(ux).all()
        s.set_checks(mach=False)
        with warnings.catch_warnings():
            warnings.simplefilter("error")
            s.fields(0)
