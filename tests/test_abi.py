"""C interface checks that need no GPU: the library loads, exports every
function include/lbmax.h declares, and host-side validation rejects bad
descriptions before any device work."""
import ctypes
import math
import os
import re

import numpy as np
import pytest

import workloads

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "lbmax.h")


@pytest.fixture(scope="module")
def lib():
    from paper_1504_06123_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        from paper_1504_06123_amd import build
        build.build()
    return _lib.load()


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(lb_[a-z_]+)\s*\(", text)))


def test_header_declares_the_interface():
    names = _declared()
    for must in ("lb_init", "lb_step", "lb_stress", "lb_grad", "lb_fields",
                 "lb_set_force", "lb_save_state", "lb_load_state", "lb_destroy",
                 "lb_workspace_bytes", "lb_last_error"):
        assert must in names


def test_library_exports_every_declared_symbol(lib):
    from paper_1504_06123_amd import _lib
    for name in _declared():
        assert hasattr(lib, name), name
        assert name in _lib.SIGNATURES, f"binding lacks {name}"


def _desc(**kw):
    from paper_1504_06123_amd import make_descs
    ch = workloads.plain_f64().channels[0].replace(**kw)
    arr, keep = make_descs([ch])
    return arr, keep


def test_workspace_bytes_valid_and_scaling(lib):
    arr, _ = _desc()
    b64 = lib.lb_workspace_bytes(arr, 1, 0)
    b32 = lib.lb_workspace_bytes(arr, 1, 1)
    assert b64 > 0 and b32 > 0 and b64 > b32
    # the ring dominates: doubling the window adds about a ring's worth
    arr2, _ = _desc(n_hist=2000)
    assert lib.lb_workspace_bytes(arr2, 1, 0) - b64 >= 1000 * 64 * 8


def test_workspace_bytes_large_2d_fits(lib):
    from paper_1504_06123_amd import make_descs
    wl = workloads.large_2d(perturb=False)
    arr, _ = make_descs(wl.channels)
    nb = lib.lb_workspace_bytes(arr, 1, 1)
    # two FP32 rings (s, r) of 4096 x 524288 plus small planes, chunk
    # partials and block sums
    ring = 2 * 4096 * 524288 * 4
    assert ring <= nb < ring * 1.06


@pytest.mark.parametrize("field,value,msg", [
    ("ly", 2, "ly"), ("lx", 0, "lx"), ("n_hist", 1, "n_hist"),
    ("tau_lb", 0.5, "tau_lb"), ("tau_lb", math.nan, "tau_lb"),
    ("g_inf", -1e-3, "g_inf"), ("tau_m", 0.0, "tau_m"), ("tau_m", math.inf, "tau_m"),
    ("gamma_c", 0.0, "gamma_c"), ("gamma_c", math.nan, "gamma_c"),
    ("gx", math.inf, "force"),
])
def test_invalid_descriptions_rejected(lib, field, value, msg):
    arr, _ = _desc(**{field: value})
    assert lib.lb_workspace_bytes(arr, 1, 1) == 0
    assert msg in lib.lb_last_error().decode()
    h = ctypes.c_void_p()
    # validation happens before any device call: a bogus pointer is never used
    st = lib.lb_init(arr, 1, 1, ctypes.c_void_p(256), 1 << 40, None, ctypes.byref(h))
    assert st == -1 and not h.value


def test_gamma_c_infinite_is_the_linear_limit(lib):
    arr, _ = _desc(gamma_c=math.inf)
    assert lib.lb_workspace_bytes(arr, 1, 1) > 0


def test_non_finite_u0_rejected(lib):
    from paper_1504_06123_amd import make_descs
    ch = workloads.plain_f64().channels[0]
    u0 = np.zeros((2, ch.ly, ch.lx))
    u0[1, 3, 2] = math.nan
    arr, keep = make_descs([ch.replace(u0=u0)])
    assert lib.lb_workspace_bytes(arr, 1, 1) == 0
    assert "u0" in lib.lb_last_error().decode()


def test_init_argument_errors(lib):
    arr, _ = _desc()
    need = lib.lb_workspace_bytes(arr, 1, 1)
    h = ctypes.c_void_p()
    assert lib.lb_init(arr, 1, 1, None, need, None, ctypes.byref(h)) == -1
    assert lib.lb_init(arr, 1, 1, ctypes.c_void_p(0x1000 + 8), need, None, ctypes.byref(h)) == -2
    assert "aligned" in lib.lb_last_error().decode()
    assert lib.lb_init(arr, 1, 1, ctypes.c_void_p(0x1000), need - 256, None, ctypes.byref(h)) == -2
    assert "too small" in lib.lb_last_error().decode()
    assert lib.lb_init(arr, 0, 1, ctypes.c_void_p(0x1000), need, None, ctypes.byref(h)) == -1
    assert lib.lb_init(arr, 1, 7, ctypes.c_void_p(0x1000), need, None, ctypes.byref(h)) == -1
    assert lib.lb_init(arr, 1, 1, ctypes.c_void_p(0x1000), need, None, None) == -1


def test_null_handle_calls(lib):
    assert lib.lb_step(None, 1) == -1
    assert lib.lb_set_force(None, 0, 0.0, 0.0) == -1
    assert lib.lb_stress(None, 0, None, None) == -1
    assert lib.lb_fields(None, 0, None, None, None) == -1
    assert lib.lb_save_state(None, None) == -1
    assert lib.lb_destroy(None) == -1
    assert lib.lb_time(None) == -1
    assert lib.lb_state_bytes(None) == 0
    assert lib.lb_max_chunks(None, 0) == 0


def test_state_layout_sections_are_aligned():
    from paper_1504_06123_amd import state_layout
    wl = workloads.batched()
    secs, total = state_layout(wl.channels[:5], "f32")
    for sec in secs:
        assert "ring_r" not in sec  # unidirectional channels keep s only
        for off, rows, n in sec.values():
            assert off % 256 == 0
    secs, _ = state_layout(workloads.plain_f64().channels, "f64")
    assert "ring_r" in secs[0]
    assert total % 256 == 0
