"""The transient studies of Sec. IV, re-run on the GPU path: qualitative checks.

The paper shows these studies only as figures whose data it does not print,
so nothing here is a parity check against values (parity unpinned); the same
solver is held to the oracle by the other GPU tests.  Each test below states
a behaviour that the paper's text describes for a figure and checks that the
runs show it, with margins taken from the runs.

One handle carries every channel (1 x 32 nodes each, FP64, 32 steps per
pass): startup from rest for T_ON steps, then cessation (force off) for
T_OFF steps, sampled every EVERY steps.  Channels are set by t_wall / tau_0,
the ratio of the transverse momentum-diffusion time to the background time
(``workloads.sec4_channel``).  "Twin" channels keep the force on through the
cessation phase, for the superposition identity of linear models.  The
velocity, shear stress and N1 at the position y/H = 0.51 of the figures are
interpolated linearly between the two nearest nodes.
"""
import math

import numpy as np
import pytest

import workloads
from closed_forms import channel_node_positions, maxwell_channel_startup
from test_gpu_parity import Solver, say  # noqa: F401

pytestmark = pytest.mark.gpu

T_ON = 60000
T_OFF = 60000
EVERY = 50
FINE_SPAN, FINE_EVERY = 2000, 5  # velocity profiles right after cessation
WIDE = (1.0, 2.0, 4.0, 8.0)  # t_wall / tau_0 >= 1
ALL_NLM = (0.1, 0.5) + WIDE

CASES = ([("nlm", r, 10.0) for r in ALL_NLM]
         + [("nlm", r, 100.0) for r in (1.0, 4.0)]
         + [(m, r, 10.0) for m in ("ucm", "instantaneous", "newtonian") for r in (0.1, 1.0)])
TWINS = [("newtonian", 1.0, 10.0), ("ucm", 1.0, 10.0), ("nlm", 1.0, 10.0)]


class Run:
    """Time series of one channel: startup samples [0, n_on), cessation
    samples [n_on, n_on + n_off); full profiles alongside, and velocity
    profiles every FINE_EVERY steps over the first FINE_SPAN of cessation."""

    def __init__(self, prof_u, prof_s, prof_n, fine_u, n_on):
        self.pu, self.ps, self.pn, self.fine_u = prof_u, prof_s, prof_n, fine_u
        ly = prof_u.shape[1]
        h = ly / 2.0
        yp = (ly - 1) / 2.0 + 0.51 * h
        y0 = int(math.floor(yp))
        w = yp - y0
        at = lambda p: (1.0 - w) * p[:, y0] + w * p[:, y0 + 1]  # noqa: E731
        self.u, self.sxy, self.n1 = at(prof_u), at(prof_s), at(prof_n)
        self.n_on = n_on
        # |y| / H of the upper half's nodes, centre outwards
        self.upper = np.arange(ly // 2, ly)
        self.yh = (self.upper - (ly - 1) / 2.0) / h

    @property
    def u_on(self):
        return self.u[:self.n_on]

    @property
    def u_off(self):
        return self.u[self.n_on:]

    @property
    def u_end(self):
        """Velocity when the force is switched off (the startup's end)."""
        return self.u[self.n_on - 1]


@pytest.fixture(scope="module")
def runs(Solver):
    chans = [workloads.sec4_channel(r, th, m) for m, r, th in CASES + TWINS]
    n_on, n_off = T_ON // EVERY, T_OFF // EVERY
    say(f"case Sec. IV transients: {len(chans)} channels 1 x 32, {T_ON} steps on, "
        f"{T_OFF} off, f64")
    store = [([], [], [], []) for _ in chans]
    with Solver(chans, precision="f64") as s:
        s.set_block(32)
        s.set_graph(64)
        for phase, n in (("on", n_on), ("off", n_off)):
            if phase == "off":
                for i in range(len(CASES)):
                    s.set_force(i, 0.0, 0.0)
            for j in range(n):
                if phase == "off" and j * EVERY < FINE_SPAN:
                    for _ in range(EVERY // FINE_EVERY):
                        s.step(FINE_EVERY)
                        for i, st in enumerate(store):
                            st[3].append(s.fields(i)[1][:, 0])
                else:
                    s.step(EVERY)
                for i, st in enumerate(store):
                    _, ux, _ = s.fields(i)
                    sxy, n1 = s.stress(i)
                    st[0].append(ux[:, 0])
                    st[1].append(sxy[:, 0])
                    st[2].append(n1[:, 0])
            say(f"  {phase} phase done")
    out = [Run(np.array(a), np.array(b), np.array(c), np.array(f), n_on) for a, b, c, f in store]
    return {k: r for k, r in zip([(m, r, th) for m, r, th in CASES]
                                 + [("twin",) + t for t in TWINS], out)}


def crossings(x, level):
    s = np.sign(np.asarray(x) - level)
    s = s[s != 0]
    return int(np.sum(s[1:] != s[:-1]))


def test_startup_velocity_overshoots_only_in_narrow_channels(runs):
    """Fig. Qall (Sec. IV, transient dynamics): the startup velocity rises
    monotonically in wide channels and overshoots its steady value before
    settling in narrow ones (t_wall << tau_0: the Newtonian profile forms
    before the structural stress)."""
    narrow = runs[("nlm", 0.1, 10.0)]
    peak = narrow.u_on.max() / narrow.u_end
    drift = abs(narrow.u_on[-1] - narrow.u_on[-100]) / narrow.u_end
    say(f"  narrow: peak / steady {peak:.4f}, drift over the last 5000 steps {drift:.1e}")
    assert peak >= 1.10 and drift <= 1e-4
    for r in (0.5,) + WIDE:
        run = runs[("nlm", r, 10.0)]
        peak = run.u_on.max() / run.u_end
        say(f"  t_wall/tau_0 = {r}: peak / steady {peak:.6f}")
        assert peak <= 1.0 + 1e-4


def test_integral_and_instantaneous_models_reach_the_same_steady_flow(runs):
    """Fig. steadystate: the integral model and the instantaneous model
    (Eq. inlM) reach the same steady channel flow."""
    for r in (0.1, 1.0):
        a, b = runs[("nlm", r, 10.0)].u_end, runs[("instantaneous", r, 10.0)].u_end
        say(f"  t_wall/tau_0 = {r}: integral {a:.6e}, instantaneous {b:.6e}")
        assert abs(a - b) <= 1e-3 * abs(b)


def test_normal_stress_difference_positive_with_startup_overshoot_in_wide_channels(runs):
    """Sec. IV: sigma_xx - sigma_yy > 0 at all times in laminar channel
    flow (theta = 10, the figures' case); after startup N1 overshoots for
    t_wall >~ tau_0 and rises monotonically in the narrowest channel
    (Fig. Qall, bottom left).  The discrete history sum (trapezoid weights,
    strain from the exclusive prefix) may dip below zero by a few 1e-6 of
    the channel's N1 scale where N1 itself is near zero.  With theta = 100
    positivity is reported, not asserted: N1 is the integral of
    (d G / d t') gamma^2, positive only while G grows with t', and the
    damping by the rate at the past time t' lets a rate that grows with t'
    break that."""
    for key, run in runs.items():
        if key[0] in ("nlm", "ucm"):
            low = run.pn.min() / np.abs(run.pn).max()
            k, y = np.unravel_index(np.argmin(run.pn), run.pn.shape)
            phase = "startup" if k < run.n_on else "cessation"
            t = (k + 1 - (0 if k < run.n_on else run.n_on)) * EVERY
            say(f"  {key}: min N1 / max N1 {low:+.1e} ({phase}, step {t}, "
                f"y/H {abs(y - (run.pn.shape[1] - 1) / 2) / (run.pn.shape[1] / 2):.2f})")
            if key[2] == 10.0:
                assert low >= -1e-5, key
    narrow = runs[("nlm", 0.1, 10.0)].n1[:T_ON // EVERY]
    assert narrow.max() <= narrow[-1] * (1.0 + 1e-3)
    assert np.diff(narrow).min() >= -1e-9 * narrow.max()
    for r in WIDE:
        n1 = runs[("nlm", r, 10.0)].n1[:T_ON // EVERY]
        say(f"  t_wall/tau_0 = {r}: N1 peak / steady {n1.max() / n1[-1]:.3f}")
        assert n1.max() >= 1.05 * n1[-1]


def test_cessation_oscillates_for_the_integral_model_only(runs):
    """Figs. QT and us: after cessation the integral model's velocity swings
    below zero (the stored stresses drive a counter-flow); the instantaneous
    model decays without oscillation."""
    for r in ALL_NLM:
        run = runs[("nlm", r, 10.0)]
        low = run.u_off.min() / run.u_end
        say(f"  integral t_wall/tau_0 = {r}: min u / u_steady after cessation {low:+.4f}")
        assert low <= -0.01
    for r in (0.1, 1.0):
        run = runs[("instantaneous", r, 10.0)]
        low = run.u_off.min() / run.u_end
        say(f"  instantaneous t_wall/tau_0 = {r}: {low:+.2e}")
        assert low >= -1e-5


def test_cessation_velocity_leads_the_shear_stress(runs):
    """Figs. QT (right) and us: after cessation the velocity and the shear
    stress decay with a phase shift, the velocity first: it reaches zero
    while the stress, still dominated by past contributions, is positive;
    that stress then drives the counter-flow and itself turns negative.  In
    the instantaneous model the stress follows the velocity gradients and
    does not oscillate (it dips by a few 1e-5 of its steady value as the
    profile's shape relaxes; values at y/H = 0.51, each divided by its steady value:
    the shear stress there is negative, the velocity falling towards the
    wall)."""
    n_on = T_ON // EVERY
    for r in ALL_NLM:
        run = runs[("nlm", r, 10.0)]
        u, sxy = run.u[n_on:] / run.u_end, run.sxy[n_on:] / run.sxy[n_on - 1]
        t_u = int(np.argmax(u <= 0))
        t_s = int(np.argmax(sxy <= 0))
        say(f"  integral t_wall/tau_0 = {r}: zero at step {(t_u + 1) * EVERY} (u), "
            f"{(t_s + 1) * EVERY} (sigma_xy); min sigma_xy / steady {sxy.min():+.3f}")
        assert (u <= 0).any() and (sxy <= 0).any()
        assert t_u < t_s and sxy[t_u] > 0
        assert sxy.min() <= -0.03
    for r in (0.1, 1.0):
        run = runs[("instantaneous", r, 10.0)]
        s_low = (run.sxy[n_on:] / run.sxy[n_on - 1]).min()
        say(f"  instantaneous t_wall/tau_0 = {r}: min sigma_xy / steady {s_low:+.1e}")
        assert s_low >= -1e-3


def test_cessation_normal_stress_decays_monotonically(runs):
    """Fig. Qall (bottom right), Fig. noffcut: after cessation N1 decays
    monotonically.  Checked at y/H = 0.51 until N1 has fallen to 1e-4 of its
    value at cessation (later, the counter-flow's small new strain shows)."""
    for r in ALL_NLM:
        n1 = runs[("nlm", r, 10.0)].n1[T_ON // EVERY - 1:]
        live = n1 >= 1e-4 * n1[0]
        stop = int(np.argmin(live)) if not live.all() else len(n1)
        rise = np.diff(n1[:stop]).max() / n1[0] if stop > 1 else 0.0
        say(f"  t_wall/tau_0 = {r}: largest rise before N1 < 1e-4 N1(0): {rise:.1e}")
        assert rise <= 1e-12


def test_startup_cessation_symmetry_holds_only_for_linear_models(runs):
    """Sec. IV: for Newtonian and linear viscoelastic (UCM) fluids the flow
    after cessation mirrors the startup, u_off(t) = u_on(T + t) - u_on(t)
    (superposition; u_on continued by the twin channel); nonlinear models
    break it."""
    n_on = T_ON // EVERY
    for model in ("newtonian", "ucm", "nlm"):
        run, twin = runs[(model, 1.0, 10.0)], runs[("twin", model, 1.0, 10.0)]
        cont = twin.u[n_on:]          # startup continued past T_ON
        lhs = run.u_off
        rhs = cont - run.u_on[:len(cont)]
        err = np.abs(lhs - rhs).max() / np.abs(run.u_on).max()
        say(f"  {model}: |u_off - (u_on(T + t) - u_on(t))| / max u_on = {err:.2e}")
        if model == "nlm":
            assert err >= 0.01
        else:
            assert err <= 1e-9


def test_normalised_transients_collapse_only_without_a_relaxation_time(runs):
    """Fig. QT: as functions of t / t_wall, the Newtonian and instantaneous
    transients of different widths collapse; the integral model's do not,
    since structural relaxation brings a time scale of its own."""
    for model, bound in (("newtonian", 1e-9), ("instantaneous", 1e-5)):
        a, b = runs[(model, 0.1, 10.0)], runs[(model, 1.0, 10.0)]
        d = np.abs(a.u / a.u_end - b.u / b.u_end).max()
        say(f"  {model}: largest difference of u / u_steady {d:.1e}")
        assert d <= bound
    a, b = runs[("nlm", 0.1, 10.0)], runs[("nlm", 1.0, 10.0)]
    d = np.abs(a.u / a.u_end - b.u / b.u_end).max()
    say(f"  integral: {d:.3f}")
    assert d >= 0.05


def test_ucm_oscillates_and_shear_thinning_removes_it(runs):
    """Fig. compModels: the UCM (no shear thinning) flows far slower, with
    the viscosity eta_inf (1 + theta) of its structural relaxation, and its
    startup overshoots and oscillates at every width; with shear thinning the
    oscillation is gone."""
    for r in (0.1, 1.0):
        ucm, nlm, newt = (runs[(m, r, 10.0)] for m in ("ucm", "nlm", "newtonian"))
        ratio = ucm.u_end / newt.u_end
        peak = ucm.u_on.max() / ucm.u_end
        say(f"  t_wall/tau_0 = {r}: UCM / Newtonian {ratio:.4f}, UCM peak {peak:.2f}, "
            f"UCM / integral {ucm.u_end / nlm.u_end:.3f}")
        assert abs(ratio - 1.0 / 11.0) <= 0.01 / 11.0
        assert peak >= 2.0
        assert ucm.u_end <= 0.2 * nlm.u_end
    ucm, nlm = runs[("ucm", 1.0, 10.0)], runs[("nlm", 1.0, 10.0)]
    assert crossings(ucm.u_on, ucm.u_end) >= 3
    assert crossings(nlm.u_on[int(np.argmax(nlm.u_on)):], nlm.u_end * (1 - 1e-6)) == 0


def test_longer_relaxation_time_lowers_the_velocity(runs):
    """Fig. figtau: with theta = 100 instead of 10 the startup velocity
    tends to a lower value (the plug is more viscous), and in channels with
    t_wall >= tau_0 it still rises without overshoot."""
    for r in (1.0, 4.0):
        slow, fast = runs[("nlm", r, 100.0)], runs[("nlm", r, 10.0)]
        say(f"  t_wall/tau_0 = {r}: u(theta 100) / u(theta 10) at the switch "
            f"{slow.u_end / fast.u_end:.4f}")
        assert slow.u_end < fast.u_end
        assert slow.u_on.max() <= slow.u_end * (1.0 + 1e-4)


def test_startup_normal_stress_profiles(runs):
    """Fig. ncut: N1 tends to a profile that grows from the centre towards
    the walls; in wider channels (t_wall >= tau_0) the transient profiles
    peak inside the channel, between y/H = 0.5 and 1, above the wall value,
    which the narrow channel does not show."""
    n_on = T_ON // EVERY
    for r in ALL_NLM:
        run = runs[("nlm", r, 10.0)]
        prof = run.pn[:n_on, run.upper]
        steady = prof[-1]
        assert np.diff(steady).min() >= -1e-12 * steady.max(), r
        interior = [p for p in prof if p.argmax() < len(p) - 1 and p.max() > p[-1] * (1 + 1e-3)]
        where = run.yh[interior[0].argmax()] if interior else None
        say(f"  t_wall/tau_0 = {r}: {len(interior)} transient profiles peak inside"
            + (f" (first at y/H = {where:.2f})" if interior else ""))
        if r >= 1.0:
            assert interior and 0.5 <= where < 1.0
        if r == 0.1:
            assert not interior


def test_cessation_centre_velocity_against_its_surroundings(runs):
    """Fig. uoffcut: after cessation the velocity reaches zero at different
    times across the channel; in the integral model the plug does not stop
    as a plug, its centre comes to rest before positions nearer the plug's
    edge, while in the UCM the centre is the last to come to rest.  First
    times at which u <= 0 over |y|/H <= 0.5, from profiles every
    FINE_EVERY steps."""
    for model in ("nlm", "ucm"):
        for r in (0.1, 1.0):
            run = runs[(model, r, 10.0)]
            prof = run.fine_u[:, run.upper]  # centre outwards
            inner = run.yh <= 0.5
            stopped = prof[:, inner] <= 0
            assert stopped.any(axis=0).all(), (model, r)
            first = (np.argmax(stopped, axis=0) + 1) * FINE_EVERY
            say(f"  {model} t_wall/tau_0 = {r}: steps to rest at y/H = "
                + ", ".join(f"{y:.2f}: {f}" for y, f in zip(run.yh[inner], first)))
            if model == "nlm":
                assert first[0] < first.max()
            else:
                assert first[0] == first.max()


def test_ucm_matches_the_analytic_startup_and_stopping_flow(runs):
    """Appendix, Fig. UCM: the UCM channel flow (with the background
    viscosity) after applying and after removing the force, at the figure's
    two widths, against its closed form (tests/closed_forms.py; stopping as
    u_on(T + t) - u_on(t) by linearity), every node over the whole run; the
    paper notes the same precision for stopping as for startup.  The bound
    is the lattice's second-order error at 2H = 32 (the oracle shows it
    shrinking fourfold per doubling of H)."""
    n_on = T_ON // EVERY
    for r in (0.1, 1.0):
        run = runs[("ucm", r, 10.0)]
        ch = workloads.sec4_channel(r, 10.0, "ucm")
        eta = (ch.tau_lb - 0.5) / 3.0
        t_on = EVERY * np.arange(1, n_on + 1)
        ys = channel_node_positions(ch.ly)
        ref_on = maxwell_channel_startup(ys, t_on, ch.ly / 2, 1.0, eta, ch.g_inf, ch.tau_m, ch.gx)
        ref_cont = maxwell_channel_startup(ys, T_ON + t_on, ch.ly / 2, 1.0, eta, ch.g_inf,
                                           ch.tau_m, ch.gx)
        scale = np.abs(ref_on).max()
        e_on = np.abs(run.pu[:n_on] - ref_on).max() / scale
        e_off = np.abs(run.pu[n_on:] - (ref_cont - ref_on)).max() / scale
        say(f"  t_wall/tau_0 = {r}: startup error {e_on:.2e}, stopping error {e_off:.2e}")
        assert e_on <= 2.5e-3 and e_off <= 2.5e-3


def test_wide_ucm_channels_track_the_closed_form(Solver):
    """Appendix, Figs. fMvelstr and funnyMaxwell: very viscous UCM fluids in
    wide channels (S2 = 0.05 and 0.01 << 1, S1 = 20 >> 1) respond almost
    elastically (shear waves from the walls, overshoots of about 15 times
    the steady speed) and reach their steady flow only on the scale of tau.
    The run tracks the closed form over 40000 steps (about 6 tau at
    theta = 400 and 2 tau at theta = 2000, in lattice units), and the error
    shrinks fourfold when the channel doubles: second order in 1/H even in
    this wave-dominated regime."""
    cases = [(64, 400.0, 0.05), (128, 400.0, 0.05), (256, 2000.0, 0.01), (512, 2000.0, 0.01)]
    chans = [workloads.appendix_ucm_channel(w, th, s2) for w, th, s2 in cases]
    steps, every = 40000, 100
    say(f"case appendix UCM: widths {[c.ly for c in chans]}, {steps} steps, f64")
    us = [[] for _ in chans]
    with Solver(chans, precision="f64") as s:
        s.set_block(32)
        s.set_graph(64)
        for _ in range(steps // every):
            s.step(every)
            for i in range(len(chans)):
                us[i].append(s.fields(i)[1][:, 0])
    ts = every * np.arange(1, steps // every + 1)
    errs = []
    for (w, th, s2), ch, u in zip(cases, chans, us):
        eta = (ch.tau_lb - 0.5) / 3.0
        ref = maxwell_channel_startup(channel_node_positions(w), ts, w / 2, 1.0, eta, ch.g_inf,
                                      ch.tau_m, ch.gx, n_modes=4000)
        errs.append(float(np.abs(np.array(u) - ref).max() / np.abs(ref).max()))
        say(f"  width {w}, theta {th:.0f}: peak / steady {np.abs(ref).max() / 1e-5:.0f}, "
            f"error {errs[-1]:.2e}")
    assert errs[1] <= 1.2e-2 and errs[3] <= 1e-2
    assert errs[0] / errs[1] >= 3.5 and errs[2] / errs[3] >= 3.5
