"""Gradients of sampled-velocity losses through the solver.

The forward run saves a state snapshot at the start of every segment of
`seg_len` steps (checkpointing keeps memory at one snapshot per segment plus
one segment of recorded step inputs inside the library) and samples u_x every
`sample_every` steps.  The backward sweep replays each segment from its
snapshot, last to first, and applies the library's hand-written discrete
adjoint (lb_adjoint_*), which returns dL/d(G_inf, tau, gamma_c, g_x) per
channel.

LBFunction wraps this as a torch.autograd.Function of the parameter tensor
theta [n_ch, 4] (float64, CPU): the output is the sampled u_x, shape
[n_samples, sum of lx*ly], and backward() runs the adjoint.
"""
from __future__ import annotations

import ctypes
from typing import List

import numpy as np

from . import _lib

PARAMS = ("g_inf", "tau_m", "gamma_c", "gx")


def set_theta(solver, theta) -> None:
    """Apply theta [n_ch, 4] = (G_inf, tau, gamma_c, g_x) to every channel."""
    theta = np.asarray(theta, dtype=np.float64).reshape(len(solver.channels), 4)
    for ch, (g, tau, gc, gx) in enumerate(theta):
        _lib.check(solver.lib.lb_set_params(solver.h, ch, float(g), float(tau), float(gc)),
                   "lb_set_params")
        solver.set_force(ch, float(gx), 0.0)


def sample_steps(steps: int, sample_every: int) -> List[int]:
    """Indices of the steps whose u_x is sampled (0-based step index)."""
    return [t - 1 for t in range(sample_every, steps + 1, sample_every)]


def forward(solver, steps: int, sample_every: int, seg_len: int):
    """Run `steps` steps from the solver's current state; return the sampled
    u_x [n_samples, sum N] and the list of (t0, snapshot) per segment."""
    ckpts = []
    samples = []
    t_start = solver.t
    marks = set(t + 1 for t in sample_steps(steps, sample_every))
    done = 0
    while done < steps:
        n = min(seg_len, steps - done)
        ckpts.append((solver.t, solver.save_state()))
        end = done + n
        while done < end:
            nxt = min([m for m in marks if m > done] + [end])
            solver.step(nxt - done)
            done = nxt
            if done in marks:
                samples.append(np.concatenate([solver.fields(ch)[1].ravel()
                                               for ch in range(len(solver.channels))]))
    assert solver.t == t_start + steps
    return np.array(samples), ckpts


def backward(solver, ckpts, steps: int, sample_every: int, seg_len: int, dL_dsamples,
             t_start: int = 0, library_workspace: bool = False):
    """dL/dtheta [n_ch, 4] for the run of forward(); dL_dsamples has the shape
    of its samples.  The solver's forward state is overwritten.  With
    library_workspace the sweep runs in the library's own device array
    (lb_adjoint_begin_noalloc) instead of a workspace allocated here."""
    import torch
    dL_dsamples = np.asarray(dL_dsamples, dtype=np.float64)
    total = dL_dsamples.shape[1]
    per_step = {t: dL_dsamples[k] for k, t in enumerate(sample_steps(steps, sample_every))}
    if library_workspace:
        _lib.check(solver.lib.lb_adjoint_begin_noalloc(solver.h, seg_len),
                   "lb_adjoint_begin_noalloc")
    else:
        nbytes = solver.lib.lb_adjoint_workspace_bytes(solver.h, seg_len)
        if nbytes == 0:
            raise _lib.LBError(_lib.LB_EINVAL, "lb_adjoint_workspace_bytes", _lib.last_error())
        # One adjoint workspace per solver and segment length, kept between
        # sweeps: the library keeps its captured reverse-sweep graphs only
        # while the workspace address and segment length stay the same.
        cached = getattr(solver, "_adjoint_ws", None)
        if cached is not None and cached[0] == seg_len and cached[1].numel() == int(nbytes):
            aws = cached[1]
        else:
            aws = torch.empty(int(nbytes), dtype=torch.uint8, device=solver.device)
            solver._adjoint_ws = (seg_len, aws)
        _lib.check(solver.lib.lb_adjoint_begin(solver.h, ctypes.c_void_p(aws.data_ptr()),
                                               int(nbytes), seg_len), "lb_adjoint_begin")
    P = ctypes.POINTER(ctypes.c_double)
    for t0, snap in reversed(ckpts):
        rel0 = t0 - t_start
        n = min(seg_len, steps - rel0)
        g = np.zeros((n, total))
        for i in range(n):
            if rel0 + i in per_step:
                g[i] = per_step[rel0 + i]
        _lib.check(solver.lib.lb_adjoint_segment(solver.h, ctypes.c_void_p(snap.data_ptr()),
                                                 g.ctypes.data_as(P), n),
                   "lb_adjoint_segment")
    out = np.zeros((len(solver.channels), 4))
    _lib.check(solver.lib.lb_adjoint_end(solver.h, out.ctypes.data_as(P)), "lb_adjoint_end")
    return out


def _autograd_function():
    import torch

    class LBFunction(torch.autograd.Function):
        """samples = LBFunction.apply(theta, solver, init_state, steps, sample_every, seg_len)

        theta: float64 CPU tensor [n_ch, 4] (G_inf, tau, gamma_c, g_x); the
        solver restarts from init_state (a lb_save_state buffer) each call."""

        @staticmethod
        def forward(ctx, theta, solver, init_state, steps, sample_every, seg_len):
            solver.load_state(init_state)
            set_theta(solver, theta.detach().cpu().numpy())
            t_start = solver.t
            samples, ckpts = forward(solver, steps, sample_every, seg_len)
            ctx.solver, ctx.ckpts = solver, ckpts
            ctx.args = (steps, sample_every, seg_len, t_start)
            return torch.from_numpy(samples)

        @staticmethod
        def backward(ctx, grad):
            steps, every, seg_len, t_start = ctx.args
            g = backward(ctx.solver, ctx.ckpts, steps, every, seg_len,
                         grad.detach().cpu().numpy(), t_start)
            return torch.from_numpy(g), None, None, None, None, None

    return LBFunction


_cache = {}


def __getattr__(name):
    if name == "LBFunction":
        if name not in _cache:
            _cache[name] = _autograd_function()
        return _cache[name]
    raise AttributeError(name)
