"""Python handle over liblbmax: torch owns the device memory and the stream.

Every step of the computation runs in the library's HIP kernels; this class
only allocates the workspace, forwards calls and converts outputs to numpy.
"""
from __future__ import annotations

import ctypes
import math
import warnings
from typing import Optional, Sequence

import numpy as np

from . import _lib


class MachWarning(UserWarning):
    """A velocity readout found |u| above the lattice Mach guard (0.1)."""


def _precision_code(precision: str) -> int:
    p = precision.lower()
    if p in ("f64", "fp64", "float64", "double"):
        return _lib.LB_F64
    if p in ("f32", "fp32", "float32", "float"):
        return _lib.LB_F32
    if p in ("f32p64", "f32_p64", "mixed"):
        return _lib.LB_F32_P64
    raise ValueError(f"unknown precision {precision!r}")


def make_descs(channels: Sequence) -> tuple:
    """Fill lb_channel_desc records from objects with the channel attributes
    (lx, ly, tau_lb, g_inf, tau_m, gamma_c, n_hist, gx, gy, u0, and optionally
    hist_blocks, hist_block_len for the quasi-logarithmic grid and finger for
    the full Finger tensor).  Returns the
    ctypes array and the list of u0 buffers it points into (keep alive)."""
    n = len(channels)
    arr = (_lib.ChannelDesc * n)()
    keep = []
    for i, ch in enumerate(channels):
        d = arr[i]
        d.lx, d.ly = int(ch.lx), int(ch.ly)
        d.tau_lb = float(ch.tau_lb)
        d.g_inf, d.tau_m, d.gamma_c = float(ch.g_inf), float(ch.tau_m), float(ch.gamma_c)
        d.n_hist = int(ch.n_hist)
        d.gx, d.gy = float(ch.gx), float(getattr(ch, "gy", 0.0))
        d.hist_blocks = int(getattr(ch, "hist_blocks", 0))
        d.hist_block_len = int(getattr(ch, "hist_block_len", 0)) if d.hist_blocks else 0
        d.finger = 1 if getattr(ch, "finger", False) else 0
        d.paper_coupling = 1 if getattr(ch, "paper_coupling", False) else 0
        d.law = _lib.LAWS[getattr(ch, "law", "nlm")]
        u0 = getattr(ch, "u0", None)
        if u0 is not None:
            buf = np.ascontiguousarray(np.asarray(u0, dtype=np.float64).reshape(2, ch.ly, ch.lx))
            keep.append(buf)
            d.u0 = buf.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        else:
            d.u0 = None
    return arr, keep


def workspace_bytes(channels: Sequence, precision: str = "f32") -> int:
    lib = _lib.load()
    arr, _keep = make_descs(channels)
    nbytes = lib.lb_workspace_bytes(arr, len(channels), _precision_code(precision))
    if nbytes == 0:
        raise _lib.LBError(_lib.LB_EINVAL, "lb_workspace_bytes", _lib.last_error())
    return int(nbytes)


class Solver:
    """A set of channels advanced together on one GPU.

    channels: sequence of channel descriptions (see make_descs).
    precision: "f32" (FP32 populations stored as remainders against the
    equilibrium of FP64 moments; FP32 history whose window sums are FP32
    partial sums added into Kahan-compensated FP32 totals; FP64 strain),
    "f32p64" (FP64 populations, the same FP32 history) or "f64".
    """

    def __init__(self, channels: Sequence, precision: str = "f32",
                 device: str = "cuda:0", stream=None):
        import torch

        self.lib = _lib.load()
        self.channels = list(channels)
        self.precision = precision
        self.prec_code = _precision_code(precision)
        self.device = torch.device(device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        arr, keep = make_descs(self.channels)
        nbytes = self.lib.lb_workspace_bytes(arr, len(self.channels), self.prec_code)
        if nbytes == 0:
            raise _lib.LBError(_lib.LB_EINVAL, "lb_workspace_bytes", _lib.last_error())
        self.ws = torch.empty(int(nbytes), dtype=torch.uint8, device=self.device)
        h = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            st = self.lib.lb_init(arr, len(self.channels), self.prec_code,
                                  ctypes.c_void_p(self.ws.data_ptr()), int(nbytes),
                                  ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(h))
        del keep
        _lib.check(st, "lb_init")
        self.h = h

    # -- lifetime -----------------------------------------------------------
    def close(self):
        if getattr(self, "h", None):
            self.lib.lb_destroy(self.h)
            self.h = None
        self._adjoint_ws = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    # -- stepping ----------------------------------------------------------
    @property
    def t(self) -> int:
        return int(self.lib.lb_time(self.h))

    def step(self, n: int = 1):
        _lib.check(self.lib.lb_step(self.h, int(n)), "lb_step")

    def set_force(self, ch: int, gx: float, gy: float = 0.0):
        _lib.check(self.lib.lb_set_force(self.h, int(ch), float(gx), float(gy)), "lb_set_force")

    def set_graph(self, steps_per_graph: int):
        _lib.check(self.lib.lb_set_graph(self.h, int(steps_per_graph)), "lb_set_graph")

    def set_block(self, steps_per_pass: int):
        """Steps served by one history pass (temporal blocking: 1, 2, 4, 8, 16, 32)."""
        _lib.check(self.lib.lb_set_block(self.h, int(steps_per_pass)), "lb_set_block")

    def set_fused(self, mode=1):
        """Fused in-block steps for handles whose channels all fit one
        workgroup: 0 (or False) separate launches, 1 (or True, the default)
        fused with the LDS-resident form where it applies, else in the
        global-memory form up to 512 nodes per channel, 2 fused in the
        global-memory form; see lb_set_fused."""
        _lib.check(self.lib.lb_set_fused(self.h, int(mode)), "lb_set_fused")

    def set_adjoint_block(self, steps: int):
        """Reverse steps per blocked launch pair of the adjoint sweep (1: the
        per-step kernels); see lb_set_adjoint_block."""
        _lib.check(self.lib.lb_set_adjoint_block(self.h, int(steps)), "lb_set_adjoint_block")

    @property
    def adjoint_block(self) -> int:
        return int(self.lib.lb_get_adjoint_block(self.h))

    @property
    def fused(self) -> int:
        """0 not fused, 1 fused launch, 2 its LDS-resident form."""
        return int(self.lib.lb_get_fused(self.h))

    def set_persistent(self, enable: bool = True):
        """Persistent history pass: resident workgroups claim tiles from a counter."""
        _lib.check(self.lib.lb_set_persistent(self.h, 1 if enable else 0), "lb_set_persistent")

    @property
    def block(self) -> int:
        return int(self.lib.lb_get_block(self.h))

    def max_chunks(self, ch: int) -> int:
        return int(self.lib.lb_max_chunks(self.h, int(ch)))

    def set_tiling(self, ch: int, n_chunks: int, nodes_per_lane: int = None):
        """History-kernel launch shape of channel ch (age chunks, nodes per lane)."""
        if nodes_per_lane is None:
            nodes_per_lane = self.tiling(ch)[1]
        _lib.check(self.lib.lb_set_tiling(self.h, int(ch), int(n_chunks), int(nodes_per_lane)),
                   "lb_set_tiling")

    def tiling(self, ch: int):
        a, b = ctypes.c_int32(), ctypes.c_int32()
        _lib.check(self.lib.lb_get_tiling(self.h, int(ch), ctypes.byref(a), ctypes.byref(b)),
                   "lb_get_tiling")
        return a.value, b.value

    # -- readouts (FP64 numpy, [ly][lx]) -------------------------------------
    def _shape(self, ch):
        c = self.channels[ch]
        return (int(c.ly), int(c.lx))

    def fields(self, ch: int = 0):
        sh = self._shape(ch)
        rho, ux, uy = (np.empty(sh) for _ in range(3))
        P = ctypes.POINTER(ctypes.c_double)
        _lib.check(self.lib.lb_fields(self.h, int(ch), rho.ctypes.data_as(P),
                                      ux.ctypes.data_as(P), uy.ctypes.data_as(P)), "lb_fields")
        if self.lib.lb_warnings(self.h) & _lib.LB_WARN_MACH:
            warnings.warn(MachWarning(
                f"channel {ch}: |u| exceeds 0.1 (lattice Mach number above 0.17); the "
                "lattice-Boltzmann step is accurate only at small Mach number"), stacklevel=2)
        return rho, ux, uy

    def set_checks(self, finite: bool = True, mach: bool = True) -> None:
        """Readout checks (lb_set_checks): non-finite values raise LBError
        with status LB_ENONFINITE; speeds above 0.1 warn (MachWarning)."""
        flags = (_lib.LB_CHECK_FINITE if finite else 0) | (_lib.LB_CHECK_MACH if mach else 0)
        _lib.check(self.lib.lb_set_checks(self.h, flags), "lb_set_checks")

    def stress(self, ch: int = 0):
        sh = self._shape(ch)
        sxy, n1 = np.empty(sh), np.empty(sh)
        P = ctypes.POINTER(ctypes.c_double)
        _lib.check(self.lib.lb_stress(self.h, int(ch), sxy.ctypes.data_as(P),
                                      n1.ctypes.data_as(P)), "lb_stress")
        return sxy, n1

    def grad(self, ch: int = 0):
        k = np.empty((4,) + self._shape(ch))
        P = ctypes.POINTER(ctypes.c_double)
        _lib.check(self.lib.lb_grad(self.h, int(ch), k.ctypes.data_as(P)), "lb_grad")
        return k

    # -- state ---------------------------------------------------------------
    def state_bytes(self) -> int:
        return int(self.lib.lb_state_bytes(self.h))

    def save_state(self, buf=None):
        import torch
        if buf is None:
            buf = torch.empty(self.state_bytes(), dtype=torch.uint8, device=self.device)
        _lib.check(self.lib.lb_save_state(self.h, ctypes.c_void_p(buf.data_ptr())), "lb_save_state")
        return buf

    def load_state(self, buf):
        _lib.check(self.lib.lb_load_state(self.h, ctypes.c_void_p(buf.data_ptr())), "lb_load_state")

    # -- timing ---------------------------------------------------------------
    def profile(self, enable: bool = True):
        _lib.check(self.lib.lb_profile(self.h, 1 if enable else 0), "lb_profile")

    def kernel_time(self, which: int = 0):
        ms = ctypes.c_double()
        cnt = ctypes.c_int64()
        _lib.check(self.lib.lb_kernel_time(self.h, int(which), ctypes.byref(ms),
                                           ctypes.byref(cnt)), "lb_kernel_time")
        return ms.value, cnt.value


STATE_MAGIC = 0x4C424D4158535431
STATE_VERSION = 6


def pack_state_header(t: int, n_ch: int, precision: str, total_bytes: int,
                      block_len: int = 1, block_pos: int = 0) -> bytes:
    """The 256-byte state header (include/lbmax.h)."""
    import struct
    hdr = struct.pack("<QIIqiiQii", STATE_MAGIC, STATE_VERSION, _precision_code(precision),
                      int(t), int(n_ch), 0, int(total_bytes), int(block_len), int(block_pos))
    return hdr + bytes(256 - len(hdr))


def state_layout(channels: Sequence, precision: str = "f32"):
    """Byte offsets of the sections of a state buffer (include/lbmax.h)."""
    code = _precision_code(precision)
    R = 8                                        # stress, velocity, density planes
    RP = 4 if code == _lib.LB_F32 else 8         # stored populations
    RH = 8 if code == _lib.LB_F64 else 4         # history ring

    def up(x):
        return (x + 255) // 256 * 256

    off = 256
    out = []
    for ch in channels:
        N = int(ch.lx) * int(ch.ly)
        uni = (int(ch.lx) == 1 and float(getattr(ch, "gy", 0.0)) == 0.0 and
               (getattr(ch, "u0", None) is None or
                not np.any(np.asarray(ch.u0, dtype=np.float64).reshape(2, -1)[1])))
        sec = {}
        finger = bool(getattr(ch, "finger", False))
        for name, rows in (("pop", 9), ("sig", 3), ("vel", 2), ("drho", 1), ("trp", 1)):
            sec[name] = (off, rows, N)
            off = up(off + rows * N * (RP if name == "pop" else R))
        B = int(getattr(ch, "hist_blocks", 0))
        if B:
            rows = B * int(ch.hist_block_len)
            for name, k in (("grid_s", 1),) + (() if uni else (("grid_r", 1), ("grid_d", 3))):
                sec[name] = (off, k * rows, N)
                off = up(off + k * rows * N * RH)
        elif getattr(ch, "law", "nlm") == "instantaneous":
            pass
        elif finger:
            sec["ring"] = (off, 8 * int(ch.n_hist), N)
            off = up(off + 8 * int(ch.n_hist) * N * RH)
        else:
            for name in ("ring_s",) + (() if uni else ("ring_r",)):
                sec[name] = (off, int(ch.n_hist), N)
                off = up(off + int(ch.n_hist) * N * RH)
        nblk = 96 if finger else 64 + B
        sec["blk"] = (off, nblk, N)   # doubles
        off = up(off + nblk * N * 8)
        sec["force"] = (off, 1, 2)
        off = up(off + 16)
        out.append(sec)
    return out, off
