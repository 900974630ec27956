"""Seeded synthetic workloads for the hybrid lattice-Boltzmann channel runs.

This module holds input recipes only: channel geometry, material and
lattice parameters, seeded random draws and run schedules.  It contains none
of the method's arithmetic, so that the FP64 oracle (``oracle/``) and the
GPU path (``paper_1504_06123_amd``) can both consume identical inputs without
sharing any code that computes the method.

The shapes follow the startup / cessation channel studies of the paper
(Sec. IV: planar pressure-driven channel, walls at both sides, flow along x,
times measured against the Maxwell time tau and the background time tau_0).
Every drawn number is produced here from a fixed seed and is available as a
plain float or numpy array; nothing downstream draws random numbers of its
own for these runs.

Parameter defaults not fixed per workload: BGK relaxation tau_LB = 1,
rho = 1, gamma_c = 0.1 (the paper's strain scale, Sec. II).
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional

import numpy as np

BASE_SEED = 1504


@dataclasses.dataclass
class Channel:
    """One planar channel: x periodic (lx nodes), y between two walls (ly nodes).

    u0, when given, is the initial velocity field with shape [2][ly][lx]
    (component, y, x); None means the fluid starts at rest.
    """

    lx: int
    ly: int
    tau_lb: float = 1.0
    g_inf: float = 1e-3
    tau_m: float = 100.0
    gamma_c: float = 0.1
    n_hist: int = 1000
    gx: float = 1e-6
    gy: float = 0.0
    u0: Optional[np.ndarray] = None
    # History grid: hist_blocks = 0 keeps the uniform window of n_hist steps;
    # hist_blocks = B >= 1 uses the quasi-logarithmic grid of B blocks of
    # hist_block_len entries whose step doubles from block to block.
    hist_blocks: int = 0
    hist_block_len: int = 128
    # Stress from the full Finger tensor (Eq. gitt with -d_t'B = E k E^T +
    # (E k E^T)^T, E the ordered product of exp(kappa dt)) instead of the
    # simple-shear reduction; sigma_yy then enters the force.
    finger: bool = False
    # Stress coupling: False enters div sigma as a body force (default);
    # True uses the paper's forcing term (Eq. bodyforce: traceless stress in
    # the second moment, trace through a density rate).
    paper_coupling: bool = False
    # Constitutive law: "nlm" the integral nonlinear Maxwell model (Eqs.
    # gitt, nlmax); "strain_damping" its variant with the accumulated strain
    # in the damping (Sec. II); "instantaneous" the instantaneous law (Eq. inlM).
    law: str = "nlm"

    @property
    def nodes(self) -> int:
        return self.lx * self.ly

    def replace(self, **kw) -> "Channel":
        return dataclasses.replace(self, **kw)


@dataclasses.dataclass
class Workload:
    """A run: channels advanced together, the force schedule, and sampling.

    The force of every channel is on for ``steps_on`` steps and then set to
    zero for ``steps_off`` steps (cessation).  ``sample_every`` is the output
    interval in steps.  ``precision`` is "f64" or "f32".
    """

    name: str
    channels: List[Channel]
    precision: str
    steps_on: int
    steps_off: int = 0
    sample_every: int = 1
    seed: int = BASE_SEED
    note: str = ""

    @property
    def steps(self) -> int:
        return self.steps_on + self.steps_off

    @property
    def nodes(self) -> int:
        return sum(c.nodes for c in self.channels)

    @property
    def entries_per_step(self) -> int:
        """History entries visited per step (nodes x window length)."""
        return sum(c.nodes * c.n_hist for c in self.channels)


def _log_uniform(rng: np.random.Generator, lo: float, hi: float, size=None):
    return np.exp(rng.uniform(math.log(lo), math.log(hi), size))


def _pow2_ceil(x: float) -> int:
    return 1 << int(math.ceil(math.log2(x)))


# --------------------------------------------------------------------------
# The five run shapes
# --------------------------------------------------------------------------

def plain_f64() -> Workload:
    """Small FP64 channel: 4 x 16 nodes, tau = 100 steps, window 1000, startup."""
    ch = Channel(lx=4, ly=16, tau_lb=1.0, g_inf=1e-3, tau_m=100.0,
                 gamma_c=0.1, n_hist=1000, gx=1e-6)
    return Workload("plain_f64_4x16", [ch], "f64", steps_on=2000,
                    sample_every=1, seed=BASE_SEED)


def startup_cessation(seed: int = BASE_SEED + 1, grid=None) -> Workload:
    """Quasi-1D channel 1 x 256, tau = 2000, window 8192, on 20000 then off 20000.

    The body force is drawn log-uniform in [1e-7, 1e-5] from the seed.
    ``grid=(B, C)`` replaces the window by the quasi-logarithmic grid of B
    blocks of C entries.
    """
    rng = np.random.default_rng(seed)
    gx = float(_log_uniform(rng, 1e-7, 1e-5))
    ch = Channel(lx=1, ly=256, tau_lb=1.0, g_inf=1e-3, tau_m=2000.0,
                 gamma_c=0.1, n_hist=8192, gx=gx)
    if grid is not None:
        ch = ch.replace(hist_blocks=int(grid[0]), hist_block_len=int(grid[1]))
    return Workload("startup_cessation_1x256", [ch], "f32", steps_on=20000,
                    steps_off=20000, sample_every=1000, seed=seed)


# Amplitude of the seeded initial-velocity perturbation of the large 2D run:
# 1 % of the Poiseuille centreline scale g*Ly^2 / (8*(nu + G*tau)) of that
# channel (g = 5e-6, Ly = 512, nu = 1/6, G*tau = 1), i.e. 0.01 * 0.14043.
LARGE_2D_PERTURBATION = 1.4043e-3


def large_2d(seed: int = BASE_SEED + 2, lx: int = 1024, ly: int = 512,
             n_hist: int = 4096, perturb: bool = True) -> Workload:
    """2D channel 1024 x 512, tau = 1000, window 4096, g = 5e-6, 5000 steps.

    The initial velocity (both components) is LARGE_2D_PERTURBATION times
    seeded uniform noise in [-1, 1] at every node; ``perturb=False`` gives the
    x-invariant start from rest.  ``lx``/``ly``/``n_hist`` allow reduced grids
    of the same recipe.
    """
    u0 = None
    if perturb:
        rng = np.random.default_rng(seed)
        u0 = LARGE_2D_PERTURBATION * rng.uniform(-1.0, 1.0, size=(2, ly, lx))
    ch = Channel(lx=lx, ly=ly, tau_lb=1.0, g_inf=1e-3, tau_m=1000.0,
                 gamma_c=0.1, n_hist=n_hist, gx=5e-6, u0=u0)
    return Workload(f"large_2d_{lx}x{ly}", [ch], "f32", steps_on=5000,
                    sample_every=500, seed=seed)


def batched(seed: int = BASE_SEED + 3, n_channels: int = 64) -> Workload:
    """64 independent quasi-1D channels of uneven width, one launch per phase.

    Ly log-uniform in [16, 1024] (rounded), tau uniform in [50, 2000] steps,
    G_inf log-uniform in [1e-4, 1e-2], g_x log-uniform in [1e-7, 1e-5];
    window length 10*tau rounded up to a power of two.  10000 steps, startup.
    """
    rng = np.random.default_rng(seed)
    ly = np.rint(_log_uniform(rng, 16, 1024, n_channels)).astype(int)
    tau = rng.uniform(50.0, 2000.0, n_channels)
    g_inf = _log_uniform(rng, 1e-4, 1e-2, n_channels)
    gx = _log_uniform(rng, 1e-7, 1e-5, n_channels)
    chans = [Channel(lx=1, ly=int(ly[i]), tau_lb=1.0, g_inf=float(g_inf[i]),
                     tau_m=float(tau[i]), gamma_c=0.1,
                     n_hist=_pow2_ceil(10.0 * tau[i]), gx=float(gx[i]))
             for i in range(n_channels)]
    return Workload(f"batched_{n_channels}ch", chans, "f32", steps_on=10000,
                    sample_every=1000, seed=seed)


# Base ("true") parameters of the differentiation run and the seeded
# evaluation point: p0 = p_true * (1 + 0.2 * sign_i), signs drawn from the seed.
ADJOINT_TRUE = dict(g_inf=1e-3, tau_m=200.0, gamma_c=0.1, gx=1e-6)
ADJOINT_PARAMS = ("g_inf", "tau_m", "gamma_c", "gx")


def adjoint_point(seed: int = BASE_SEED + 4) -> dict:
    rng = np.random.default_rng(seed)
    signs = rng.choice([-1.0, 1.0], size=len(ADJOINT_PARAMS))
    return {k: ADJOINT_TRUE[k] * (1.0 + 0.2 * s)
            for k, s in zip(ADJOINT_PARAMS, signs)}


def differentiation(seed: int = BASE_SEED + 4, ly: int = 128,
                    n_hist: int = 2048, steps: int = 4000,
                    sample_every: int = 200) -> Workload:
    """1 x 128 channel, window 2048, startup for 4000 steps in FP32.

    The channel carries the evaluation point p0; the target profile is made by
    the same solver at ADJOINT_TRUE.  Samples of u_x(y) every 200 steps.
    """
    p = adjoint_point(seed)
    ch = Channel(lx=1, ly=ly, tau_lb=1.0, g_inf=p["g_inf"], tau_m=p["tau_m"],
                 gamma_c=p["gamma_c"], n_hist=n_hist, gx=p["gx"])
    return Workload(f"differentiation_1x{ly}", [ch], "f32", steps_on=steps,
                    sample_every=sample_every, seed=seed)


def true_channel(ch: Channel) -> Channel:
    """The differentiation channel at the true parameters."""
    return ch.replace(**ADJOINT_TRUE)


# --------------------------------------------------------------------------
# Channels of the transient studies of Sec. IV (startup and cessation of
# pressure-driven channel flow: Figs. Qall, QT, us, figtau, compModels,
# uoffcut, ncut, noffcut)
# --------------------------------------------------------------------------

# The paper's BGK relaxation (Sec. III) and a channel of 2H = 32 nodes.
SEC4_TAU_LB = 0.9
SEC4_HALF_WIDTH = 16
SEC4_MODELS = ("nlm", "ucm", "instantaneous", "newtonian")


def sec4_wall_time(half_width: int = SEC4_HALF_WIDTH, tau_lb: float = SEC4_TAU_LB) -> float:
    """Transverse momentum-diffusion time t_wall = 4 H^2 rho / (pi^2 eta_inf)
    of Sec. IV in steps, with rho = 1 and eta_inf = (tau_LB - 1/2) / 3."""
    eta = (tau_lb - 0.5) / 3.0
    return 4.0 * half_width ** 2 / (math.pi ** 2 * eta)


def sec4_channel(twall_over_tau0: float, theta: float = 10.0, model: str = "nlm",
                 half_width: int = SEC4_HALF_WIDTH) -> Channel:
    """One channel of the Sec. IV transient studies: 1 x 2H nodes, at rest.

    The paper varies the channel width to set t_wall / tau_0; here H is fixed
    and the ratio sets the background time tau_0 = t_wall / ratio instead
    (G_inf = eta_inf / tau_0), which gives the same dimensionless problem.
    The Maxwell time is tau = theta tau_0, gamma_c = 0.1, and the driving
    force density g = G_inf / (2H) (the pressure drop over one channel width
    equals G_inf, Fig. steadystate; the yield stress G_inf gamma_c then leaves
    a plug |y| / H < 2 gamma_c).  The window holds 6 tau steps: history
    older than that weighs at most e^-6 even where the fluid is unsheared;
    10 tau for the UCM, whose memory decays with tau alone everywhere (and
    which the tests hold to a closed form).
    Models: "nlm" the integral nonlinear Maxwell model (Eqs. gitt, nlmax);
    "ucm" its linear limit gamma_c = inf; "instantaneous" Eq. inlM; and
    "newtonian" G_inf = 0.  The last three keep the nlm channel's force.
    """
    if model not in SEC4_MODELS:
        raise ValueError(f"unknown model {model!r}")
    eta = (SEC4_TAU_LB - 0.5) / 3.0
    tau0 = sec4_wall_time(half_width) / twall_over_tau0
    g_inf = eta / tau0
    tau = theta * tau0
    ch = Channel(lx=1, ly=2 * half_width, tau_lb=SEC4_TAU_LB, g_inf=g_inf, tau_m=tau,
                 gamma_c=0.1, n_hist=int(math.ceil(6.0 * tau)), gx=g_inf / (2 * half_width))
    if model == "ucm":
        ch = ch.replace(gamma_c=math.inf, n_hist=int(math.ceil(10.0 * tau)))
    elif model == "instantaneous":
        ch = ch.replace(law="instantaneous", n_hist=2)
    elif model == "newtonian":
        ch = ch.replace(g_inf=0.0, n_hist=2)
    return ch


def appendix_ucm_channel(width: int, theta: float, s2: float, u_steady: float = 1e-5) -> Channel:
    """A wide UCM channel of the appendix (Figs. fMvelstr, funnyMaxwell):
    1 x width nodes, theta = tau / tau_0, and the dimensionless retardation
    time S2 = eta_max tau_0 / (rho L^2) with L = width and eta_max =
    G_inf (tau + tau_0) = eta_inf (theta + 1); the relaxation time is then
    S1 = S2 tau / tau_0.  tau_LB = 0.9, rho = 1.  The model is linear, so the
    force only scales the flow: g gives the steady centreline speed
    u_steady = g H^2 / (2 eta_max), small enough to keep the elastic
    overshoots (about 15 to 20 times that) at small Mach number.  The window
    holds 10 tau."""
    eta = (SEC4_TAU_LB - 0.5) / 3.0
    tau0 = s2 * width * width / (eta * (theta + 1.0))
    g_inf = eta / tau0
    tau = theta * tau0
    half = width / 2.0
    eta_max = eta * (theta + 1.0)
    return Channel(lx=1, ly=width, tau_lb=SEC4_TAU_LB, g_inf=g_inf, tau_m=tau,
                   gamma_c=math.inf, n_hist=int(math.ceil(10.0 * tau)),
                   gx=2.0 * u_steady * eta_max / (half * half))


ALL = {
    "plain_f64": plain_f64,
    "startup_cessation": startup_cessation,
    "large_2d": large_2d,
    "batched": batched,
    "differentiation": differentiation,
}


# --------------------------------------------------------------------------
# Synthetic history windows (inputs for kernel-level parity at full size)
# --------------------------------------------------------------------------

def random_history(rng: np.random.Generator, n_hist: int, nodes: int,
                   s_scale: float = 1e-3, r_scale: float = 2e-3,
                   dtype=np.float32):
    """Seeded random ring contents: s in [-s_scale, s_scale], r in [0, r_scale].

    Returned as slot-major arrays [n_hist][nodes] in ``dtype``.
    """
    s = rng.uniform(-s_scale, s_scale, size=(n_hist, nodes)).astype(dtype)
    r = rng.uniform(0.0, r_scale, size=(n_hist, nodes)).astype(dtype)
    return s, r
