"""lb_adjoint_begin_noalloc: the adjoint sweep in the library's own static
device array instead of a caller-allocated workspace.  Through the C
interface, two sweeps in a row -- the second on a smaller channel, window
and segment, so it runs over what the first left in the array -- each give
the gradient of the caller-workspace sweep on the same run, bit for bit (the
same kernels and arithmetic; only the workspace address differs); both also
meet the FP64 finite-difference bar of the oracle.  A workspace larger than
the array is refused with LB_ENOMEM before any device work."""
import os

import numpy as np
import pytest

import oracle
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


def _samples(ch, steps, every):
    wl = workloads.Workload("a", [ch], "f64", steps_on=steps, sample_every=every)
    return oracle.run_workload(wl)[0]["ux"][:, :, 0]


def _gradient(lb, ch, steps, every, seg, target, library_workspace):
    from paper_1504_06123_amd import adjoint
    with lb.Solver([ch], precision="f64") as s:
        u, ckpts = adjoint.forward(s, steps, every, seg)
        return adjoint.backward(s, ckpts, steps, every, seg, 2 * (u - target),
                                library_workspace=library_workspace)[0]


def test_noalloc_sweep_equals_caller_workspace_sweep(lb):
    big = workloads.Channel(lx=1, ly=48, tau_lb=1.0, g_inf=2e-3, tau_m=40.0, gamma_c=0.05,
                            n_hist=160, gx=2e-5)
    small = workloads.Channel(lx=1, ly=12, tau_lb=0.9, g_inf=1e-3, tau_m=25.0, gamma_c=0.08,
                              n_hist=40, gx=1.2e-5)
    for name, ch, steps, every, seg in (("first, 1x48 window 160", big, 320, 20, 64),
                                        ("second, smaller: 1x12 window 40", small, 120, 10, 24)):
        say(f"case no-alloc adjoint sweep, {name}")
        target = _samples(ch.replace(gx=0.8 * ch.gx), steps, every)
        g_lib = _gradient(lb, ch, steps, every, seg, target, True)
        g_ref = _gradient(lb, ch, steps, every, seg, target, False)
        say(f"  library array {g_lib}\n  caller workspace {g_ref}")
        assert np.array_equal(g_lib, g_ref)


def test_noalloc_sweep_refuses_more_than_the_array(lb):
    from paper_1504_06123_amd import _lib
    ch = workloads.Channel(lx=1, ly=1024, tau_lb=1.0, g_inf=1e-3, tau_m=400.0, gamma_c=0.1,
                           n_hist=4096, gx=1e-6)
    say("case no-alloc adjoint sweep, workspace above 64 MiB")
    with lb.Solver([ch], precision="f64") as s:
        need = s.lib.lb_adjoint_workspace_bytes(s.h, 1024)
        assert need > 64 << 20
        assert s.lib.lb_adjoint_begin_noalloc(s.h, 1024) == _lib.LB_ENOMEM
        assert "exceeds" in _lib.last_error()
