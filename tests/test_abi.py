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
    ("lx", (1 << 22) + 1, "too many nodes"),
])
def test_invalid_descriptions_rejected(lib, field, value, msg):
    arr, _ = _desc(**{field: value})
    assert lib.lb_workspace_bytes(arr, 1, 1) == 0
    assert msg in lib.lb_last_error().decode()
    h = ctypes.c_void_p()
    # validation happens before any device call: a bogus pointer is never used
    st = lib.lb_init(arr, 1, 1, ctypes.c_void_p(256), 1 << 40, None, ctypes.byref(h))
    assert st == -1 and not h.value


def test_fp32_window_limited_to_exact_ages(lib):
    """FP32 histories take entry ages as FP32 numbers, exact below 2^24: a
    longer window is rejected for them and accepted in FP64."""
    arr, _ = _desc(n_hist=(1 << 24) + 1)
    for prec in (1, 2):
        assert lib.lb_workspace_bytes(arr, 1, prec) == 0
        assert "2^24" in lib.lb_last_error().decode()
    assert lib.lb_workspace_bytes(arr, 1, 0) > 0
    arr, _ = _desc(n_hist=1 << 24)
    assert lib.lb_workspace_bytes(arr, 1, 1) > 0


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
    assert lib.lb_set_fused(None, 1) == -1
    assert lib.lb_set_fused(None, 3) == -1
    assert lib.lb_get_fused(None) == 0
    assert lib.lb_set_adjoint_block(None, 32) == -1
    assert lib.lb_get_adjoint_block(None) == 0
    assert lib.lb_adjoint_workspace_bytes(None, 64) == 0


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


def test_descriptor_layout_matches_the_header(tmp_path):
    """The ctypes record has the layout a C compiler gives lb_channel_desc."""
    import subprocess
    from paper_1504_06123_amd import _lib
    src = tmp_path / "layout.c"
    fields = [f for f, _ in _lib.ChannelDesc._fields_]
    src.write_text('#include <stddef.h>\n#include <stdio.h>\n#include "lbmax.h"\n'
                   "int main(void) {\n"
                   '  printf("%zu\\n", sizeof(lb_channel_desc));\n' +
                   "".join(f'  printf("%zu\\n", offsetof(lb_channel_desc, {f}));\n'
                           for f in fields) + "  return 0;\n}\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"), str(src), "-o",
                    str(exe)], check=True)
    vals = [int(v) for v in subprocess.run([str(exe)], check=True, capture_output=True,
                                           text=True).stdout.split()]
    assert vals[0] == ctypes.sizeof(_lib.ChannelDesc)
    for f, off in zip(fields, vals[1:]):
        assert getattr(_lib.ChannelDesc, f).offset == off, f


@pytest.mark.parametrize("kw,msg", [
    (dict(hist_blocks=-1), "hist_blocks"), (dict(hist_blocks=21), "hist_blocks"),
    (dict(hist_blocks=3, hist_block_len=1), "hist_block_len"),
    (dict(hist_blocks=20, hist_block_len=4096), "2^hist_blocks"),
])
def test_invalid_history_grids_rejected(lib, kw, msg):
    arr, _ = _desc(**kw)
    assert lib.lb_workspace_bytes(arr, 1, 1) == 0
    assert msg in lib.lb_last_error().decode()


def test_grid_channel_workspace_replaces_the_window(lib):
    """A grid channel holds B*C entries per node (s, |gamma_dot| and three
    gradient components in 2D) and no uniform window: n_hist is ignored."""
    from paper_1504_06123_amd import make_descs
    ch = workloads.large_2d(lx=64, ly=32, n_hist=4096).channels[0]
    a_win, _ = make_descs([ch])
    a_grid, _ = make_descs([ch.replace(hist_blocks=6, hist_block_len=128)])
    a_grid2, _ = make_descs([ch.replace(hist_blocks=6, hist_block_len=128, n_hist=1)])
    w, g = lib.lb_workspace_bytes(a_win, 1, 1), lib.lb_workspace_bytes(a_grid, 1, 1)
    assert g == lib.lb_workspace_bytes(a_grid2, 1, 1) > 0
    N = 64 * 32
    # the grid also keeps one FP64 strain plane per grid block for blocking
    assert w - g >= 2 * 4096 * N * 4 - 5 * 6 * 128 * N * 4 - 6 * N * 8 - 4096


def test_state_layout_of_grid_channels():
    from paper_1504_06123_amd import state_layout
    uni = workloads.plain_f64().channels[0].replace(lx=1, hist_blocks=3, hist_block_len=8)
    twod = workloads.plain_f64().channels[0].replace(hist_blocks=2, hist_block_len=5)
    secs, _ = state_layout([uni, twod], "f32p64")
    assert secs[0]["grid_s"][1] == 24 and "grid_r" not in secs[0] and "ring_s" not in secs[0]
    assert secs[1]["grid_s"][1] == 10 and secs[1]["grid_d"][1] == 30
