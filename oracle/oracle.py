"""ctypes binding of the FP64 C oracle (oracle/lb_oracle.c).

TEST INFRASTRUCTURE ONLY.  Every function forwards to the C code, which
follows the paper step by step; this file adds argument marshalling and a
driver that runs a seeded workload with its force schedule and sampling.
"""
from __future__ import annotations

import ctypes
import os
from typing import Dict, List, Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liblboracle.so")
_lib = None

# constitutive laws (Channel.law): the integral nlM model, its accumulated-
# strain damping variant, the instantaneous law
LAWS = {"nlm": 0, "strain_damping": 1, "instantaneous": 2}

_D = ctypes.POINTER(ctypes.c_double)
_I = ctypes.POINTER(ctypes.c_int)


def load():
    """Load (building first if absent) the oracle shared library."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        from . import build as _b
        _b.build()
    lib = ctypes.CDLL(_LIB_PATH)
    sig = {
        "orc_lattice": (None, [_I, _I, _D, _I]),
        "orc_equilibrium": (None, [ctypes.c_double] * 3 + [_D]),
        "orc_force_term": (None, [ctypes.c_double] * 5 + [_D]),
        "orc_collide": (None, [ctypes.c_double, _D] + [ctypes.c_double] * 5 + [_D]),
        "orc_density_momentum": (None, [_D, _D, _D, _D]),
        "orc_velocity_gradient": (None, [ctypes.c_int, ctypes.c_int, _D, _D, _D, _D, _D, _D]),
        "orc_shear_rate": (ctypes.c_double, [ctypes.c_double] * 4),
        "orc_stress_divergence": (None, [ctypes.c_int, ctypes.c_int, _D, _D, _D, _D, _D]),
        "orc_stream": (None, [ctypes.c_int, ctypes.c_int, _D, _D]),
        "orc_history_sum": (None, [ctypes.c_int, ctypes.c_int, _D, _D, _D,
                                   ctypes.c_double, ctypes.c_double, ctypes.c_double, _D, _D]),
        "orc_history_sum_ages": (None, [ctypes.c_int, _D, _D, ctypes.c_double,
                                        ctypes.c_double, ctypes.c_double, _D, _D]),
        "orc_create": (ctypes.c_void_p, [ctypes.c_int, ctypes.c_int] + [ctypes.c_double] * 4
                       + [ctypes.c_int, ctypes.c_double, ctypes.c_double, _D]),
        "orc_destroy": (None, [ctypes.c_void_p]),
        "orc_set_force": (None, [ctypes.c_void_p, ctypes.c_double, ctypes.c_double]),
        "orc_step": (None, [ctypes.c_void_p, ctypes.c_long]),
        "orc_time": (ctypes.c_long, [ctypes.c_void_p]),
        "orc_fields": (ctypes.c_int, [ctypes.c_void_p, _D, _D, _D]),
        "orc_stress": (ctypes.c_int, [ctypes.c_void_p, _D, _D]),
        "orc_grad": (ctypes.c_int, [ctypes.c_void_p, _D]),
        "orc_mass": (ctypes.c_double, [ctypes.c_void_p]),
        "orc_get_state": (None, [ctypes.c_void_p, _D, _D, _D, _D, _D, _D, _D,
                                 ctypes.POINTER(ctypes.c_long)]),
        "orc_set_state": (None, [ctypes.c_void_p, _D, _D, _D, _D, _D, _D, _D, ctypes.c_long]),
        "orc_set_history_grid": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.c_int]),
        "orc_set_finger": (ctypes.c_int, [ctypes.c_void_p]),
        "orc_set_paper_coupling": (ctypes.c_int, [ctypes.c_void_p]),
        "orc_set_law": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int]),
        "orc_history_sum_wm": (None, [ctypes.c_int, ctypes.c_int, _D, _D, _D,
                                      ctypes.c_double, ctypes.c_double, ctypes.c_double, _D,
                                      _D]),
        "orc_instantaneous": (None, [ctypes.c_double] * 5 + [_D, _D]),
        "orc_trace_prev": (ctypes.c_int, [ctypes.c_void_p, _D]),
        "orc_force_term_paper": (None, [ctypes.c_double] * 5 + [_D, ctypes.c_double, _D]),
        "orc_expm2": (None, [_D, _D]),
        "orc_finger_sum": (None, [ctypes.c_int, ctypes.c_int, _D, _D, ctypes.c_double,
                                  ctypes.c_double, ctypes.c_double, _D]),
        "orc_qgrid_create": (ctypes.c_void_p, [ctypes.c_int, ctypes.c_int]),
        "orc_qgrid_destroy": (None, [ctypes.c_void_p]),
        "orc_qgrid_push": (None, [ctypes.c_void_p, ctypes.c_long] + [ctypes.c_double] * 4),
        "orc_qgrid_capacity": (ctypes.c_int, [ctypes.c_void_p]),
        "orc_qgrid_entries": (ctypes.c_int, [ctypes.c_void_p, _D, _D, _D, _D]),
        "orc_qgrid_sum": (None, [ctypes.c_void_p, ctypes.c_long] + [ctypes.c_double] * 3
                          + [_D, _D]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def _p(a: Optional[np.ndarray]):
    if a is None:
        return None
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(_D)


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


# --------------------------------------------------------------------------
# Unit entry points (one step of the scheme each)
# --------------------------------------------------------------------------

def lattice():
    lib = load()
    cx = (ctypes.c_int * 9)()
    cy = (ctypes.c_int * 9)()
    w = (ctypes.c_double * 9)()
    opp = (ctypes.c_int * 9)()
    lib.orc_lattice(cx, cy, w, opp)
    return np.array(cx[:]), np.array(cy[:]), np.array(w[:]), np.array(opp[:])


def equilibrium(rho: float, ux: float, uy: float) -> np.ndarray:
    out = np.zeros(9)
    load().orc_equilibrium(rho, ux, uy, _p(out))
    return out


def force_term(tau_lb: float, ux: float, uy: float, fx: float, fy: float) -> np.ndarray:
    out = np.zeros(9)
    load().orc_force_term(tau_lb, ux, uy, fx, fy, _p(out))
    return out


def collide(tau_lb, n, rho, ux, uy, fx, fy) -> np.ndarray:
    n = _f64(n)
    out = np.zeros(9)
    load().orc_collide(tau_lb, _p(n), rho, ux, uy, fx, fy, _p(out))
    return out


def density_momentum(n):
    n = _f64(n)
    r, a, b = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
    load().orc_density_momentum(_p(n), ctypes.byref(r), ctypes.byref(a), ctypes.byref(b))
    return r.value, a.value, b.value


def velocity_gradient(ux: np.ndarray, uy: np.ndarray):
    """ux, uy: [ly][lx] -> (kxx, kxy, kyx, kyy), each [ly][lx]."""
    ux, uy = _f64(ux), _f64(uy)
    ly, lx = ux.shape
    outs = [np.zeros((ly, lx)) for _ in range(4)]
    load().orc_velocity_gradient(lx, ly, _p(ux), _p(uy), *[_p(o) for o in outs])
    return tuple(outs)


def shear_rate(kxx, kxy, kyx, kyy) -> float:
    return load().orc_shear_rate(kxx, kxy, kyx, kyy)


def stress_divergence(sxx: np.ndarray, sxy: np.ndarray, syy: Optional[np.ndarray] = None):
    sxx, sxy = _f64(sxx), _f64(sxy)
    syy = None if syy is None else _f64(syy)
    ly, lx = sxx.shape
    fx, fy = np.zeros((ly, lx)), np.zeros((ly, lx))
    load().orc_stress_divergence(lx, ly, _p(sxx), _p(sxy), _p(syy), _p(fx), _p(fy))
    return fx, fy


def stream(nstar: np.ndarray) -> np.ndarray:
    """nstar: [9][ly][lx] post-collision populations -> streamed populations."""
    nstar = _f64(nstar)
    _, ly, lx = nstar.shape
    out = np.zeros_like(nstar)
    load().orc_stream(lx, ly, _p(nstar), _p(out))
    return out


def history_sum(n_hist, s_age, r_age, dgam_age, g_inf, tau_m, gamma_c, n_live=None):
    s_age, r_age, dgam_age = _f64(s_age), _f64(r_age), _f64(dgam_age)
    if n_live is None:
        n_live = len(s_age)
    a, b = ctypes.c_double(), ctypes.c_double()
    load().orc_history_sum(int(n_hist), int(n_live), _p(s_age), _p(r_age), _p(dgam_age),
                           g_inf, tau_m, gamma_c, ctypes.byref(a), ctypes.byref(b))
    return a.value, b.value


def history_sum_wm(n_hist, s_age, r_age, dgam_age, g_inf, tau_m, gamma_c, n_live=None):
    """History sum with the accumulated-strain damping (Sec. II variant)."""
    s_age, r_age, dgam_age = _f64(s_age), _f64(r_age), _f64(dgam_age)
    if n_live is None:
        n_live = len(s_age)
    a, b = ctypes.c_double(), ctypes.c_double()
    load().orc_history_sum_wm(int(n_hist), int(n_live), _p(s_age), _p(r_age), _p(dgam_age),
                              g_inf, tau_m, gamma_c, ctypes.byref(a), ctypes.byref(b))
    return a.value, b.value


def instantaneous(s, r, g_inf, tau_m, gamma_c):
    a, b = ctypes.c_double(), ctypes.c_double()
    load().orc_instantaneous(s, r, g_inf, tau_m, gamma_c, ctypes.byref(a), ctypes.byref(b))
    return a.value, b.value


def history_sum_ages(s_age, r_age, g_inf, tau_m, gamma_c):
    """History integral from a full window of shear history given by age."""
    s_age, r_age = _f64(s_age), _f64(r_age)
    a, b = ctypes.c_double(), ctypes.c_double()
    load().orc_history_sum_ages(len(s_age), _p(s_age), _p(r_age), g_inf, tau_m, gamma_c,
                                ctypes.byref(a), ctypes.byref(b))
    return a.value, b.value


def force_term_paper(tau_lb, ux, uy, fx, fy, sbar, dr) -> np.ndarray:
    """Eq. bodyforce in full: sbar = traceless stress (xx, xy, yy), dr the
    density rate d_t delta rho."""
    sbar = _f64(sbar).reshape(3)
    out = np.zeros(9)
    load().orc_force_term_paper(tau_lb, ux, uy, fx, fy, _p(sbar), dr, _p(out))
    return out


def expm2(a) -> np.ndarray:
    """exp of a 2x2 matrix (row-major [2][2])."""
    a = _f64(a).reshape(4)
    out = np.zeros(4)
    load().orc_expm2(_p(a), _p(out))
    return out.reshape(2, 2)


def finger_sum(n_hist, k_age, g_inf, tau_m, gamma_c, f_age=None):
    """Full-tensor history integral over a window given by age: k_age
    [n_live][2][2] velocity gradients (kappa_ab = d_b u_a); f_age the factors
    exp(kappa dt) (computed with expm2 when None).  Returns (sxx, sxy, syy)."""
    k_age = _f64(k_age).reshape(-1, 4)
    if f_age is None:
        f_age = np.array([expm2(k.reshape(2, 2)).reshape(4) for k in k_age])
    f_age = _f64(f_age).reshape(-1, 4)
    out = np.zeros(3)
    load().orc_finger_sum(int(n_hist), len(k_age), _p(np.ascontiguousarray(k_age)),
                          _p(np.ascontiguousarray(f_age)), g_inf, tau_m, gamma_c, _p(out))
    return tuple(out)


class QGrid:
    """The quasi-logarithmic history grid of one node (B blocks of C entries),
    driven directly: push velocity gradients step by step, read the entries
    newest first, evaluate the history integral."""

    def __init__(self, B: int, C: int):
        self.lib = load()
        self.B, self.C = B, C
        self.h = self.lib.orc_qgrid_create(B, C)
        if not self.h:
            raise ValueError("oracle rejected the grid")
        self.t = 0

    def close(self):
        if self.h:
            self.lib.orc_qgrid_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def push(self, kxx=0.0, kxy=0.0, kyx=0.0, kyy=0.0):
        """The entry of step self.t; then the step counter advances."""
        self.lib.orc_qgrid_push(self.h, self.t, kxx, kxy, kyx, kyy)
        self.t += 1

    def entries(self):
        """Live entries newest first: start time, duration, kappa [n][4] and
        the strain gamma(t, t0) for the last pushed step t."""
        cap = self.lib.orc_qgrid_capacity(self.h)
        t0, dt, st = np.zeros(cap), np.zeros(cap), np.zeros(cap)
        k4 = np.zeros((cap, 4))
        n = self.lib.orc_qgrid_entries(self.h, _p(t0), _p(dt), _p(k4), _p(st))
        return t0[:n], dt[:n], k4[:n], st[:n]

    def sum(self, g_inf, tau_m, gamma_c):
        """(sigma_xy, sigma_xx) at the last pushed step."""
        a, b = ctypes.c_double(), ctypes.c_double()
        self.lib.orc_qgrid_sum(self.h, self.t - 1, g_inf, tau_m, gamma_c, ctypes.byref(a),
                               ctypes.byref(b))
        return a.value, b.value


# --------------------------------------------------------------------------
# Channel object
# --------------------------------------------------------------------------

class OracleChannel:
    """One channel of the FP64 oracle.  Arrays are [ly][lx] (x fastest)."""

    def __init__(self, ch):
        self.lib = load()
        self.lx, self.ly, self.n_hist = ch.lx, ch.ly, ch.n_hist
        u0 = None if ch.u0 is None else _f64(ch.u0).reshape(2, ch.ly, ch.lx)
        self._u0 = u0
        self.h = self.lib.orc_create(ch.lx, ch.ly, ch.tau_lb, ch.g_inf, ch.tau_m,
                                     ch.gamma_c, ch.n_hist, ch.gx, ch.gy, _p(u0))
        if not self.h:
            raise ValueError("oracle rejected the channel description")
        law = LAWS[getattr(ch, "law", "nlm")]
        if law and self.lib.orc_set_law(self.h, law) != 0:
            raise ValueError("oracle rejected the constitutive law")
        if getattr(ch, "paper_coupling", False):
            if self.lib.orc_set_paper_coupling(self.h) != 0:
                raise ValueError("oracle rejected the paper coupling")
        if getattr(ch, "finger", False):
            if self.lib.orc_set_finger(self.h) != 0:
                raise ValueError("oracle rejected the full-tensor path")
        if getattr(ch, "hist_blocks", 0):
            if self.lib.orc_set_history_grid(self.h, ch.hist_blocks, ch.hist_block_len) != 0:
                raise ValueError("oracle rejected the history grid")

    def close(self):
        if self.h:
            self.lib.orc_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def t(self) -> int:
        return self.lib.orc_time(self.h)

    def set_force(self, gx: float, gy: float = 0.0):
        self.lib.orc_set_force(self.h, gx, gy)

    def step(self, n: int = 1):
        self.lib.orc_step(self.h, int(n))

    def _shape(self):
        return (self.ly, self.lx)

    def fields(self):
        rho, ux, uy = (np.zeros(self._shape()) for _ in range(3))
        if self.lib.orc_fields(self.h, _p(rho), _p(ux), _p(uy)) != 0:
            raise RuntimeError("no completed step")
        return rho, ux, uy

    def stress(self):
        sxy, n1 = np.zeros(self._shape()), np.zeros(self._shape())
        if self.lib.orc_stress(self.h, _p(sxy), _p(n1)) != 0:
            raise RuntimeError("no completed step")
        return sxy, n1

    def grad(self):
        k = np.zeros((4,) + self._shape())
        if self.lib.orc_grad(self.h, _p(k)) != 0:
            raise RuntimeError("no completed step")
        return k

    def mass(self) -> float:
        return self.lib.orc_mass(self.h)

    def trace_prev(self) -> np.ndarray:
        """tr sigma two steps back (paper coupling only), [ly][lx]."""
        out = np.zeros(self._shape())
        if self.lib.orc_trace_prev(self.h, _p(out)) != 0:
            raise RuntimeError("not a paper-coupling channel")
        return out

    def get_state(self) -> Dict[str, np.ndarray]:
        N, H = self.lx * self.ly, self.n_hist
        st = dict(n=np.zeros((9, N)), sig_xy=np.zeros(N), sig_xx=np.zeros(N),
                  ring_s=np.zeros((H, N)), ring_r=np.zeros((H, N)),
                  ring_g=np.zeros((H, N)), gam=np.zeros(N))
        t = ctypes.c_long()
        self.lib.orc_get_state(self.h, *[_p(st[k]) for k in
                                         ("n", "sig_xy", "sig_xx", "ring_s", "ring_r",
                                          "ring_g", "gam")], ctypes.byref(t))
        st["t"] = t.value
        return st

    def set_state(self, t: int, n=None, sig_xy=None, sig_xx=None, ring_s=None,
                  ring_r=None, ring_g=None, gam=None):
        arrs = [None if a is None else _f64(a) for a in
                (n, sig_xy, sig_xx, ring_s, ring_r, ring_g, gam)]
        N, H = self.lx * self.ly, self.n_hist
        sizes = (9 * N, N, N, H * N, H * N, H * N, N)
        for a, sz in zip(arrs, sizes):
            assert a is None or a.size == sz
        self.lib.orc_set_state(self.h, *[_p(a) for a in arrs], int(t))


def run_workload(wl, steps: Optional[int] = None, sample_every: Optional[int] = None,
                 channels: Optional[List[int]] = None):
    """Run a seeded workload in the oracle, one channel after another.

    Returns, per channel, a dict of sampled outputs: 't' (completed-step
    index of each sample, i.e. the step the outputs belong to), 'ux', 'uy',
    'rho', 'sxy', 'n1' with shape [samples][ly][lx].  The force schedule is
    the workload's: on for steps_on steps, then zero.
    """
    steps = wl.steps if steps is None else steps
    every = wl.sample_every if sample_every is None else sample_every
    idxs = range(len(wl.channels)) if channels is None else channels
    out = []
    for ci in idxs:
        ch = wl.channels[ci]
        oc = OracleChannel(ch)
        rec = {k: [] for k in ("t", "ux", "uy", "rho", "sxy", "n1")}
        marks = sorted({m for m in list(range(every, steps + 1, every)) + [wl.steps_on, steps]
                        if 0 < m <= steps})
        done = 0
        for m in marks:
            if done >= wl.steps_on:
                oc.set_force(0.0, 0.0)
            oc.step(m - done)
            done = m
            if done % every == 0:
                rho, ux, uy = oc.fields()
                sxy, n1 = oc.stress()
                rec["t"].append(done - 1)
                for k, v in (("ux", ux), ("uy", uy), ("rho", rho), ("sxy", sxy), ("n1", n1)):
                    rec[k].append(v)
        oc.close()
        out.append({k: np.array(v) for k, v in rec.items()})
    return out
