"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Each test checks one step of the oracle against something other than the
oracle itself: constants the paper prints, defining moment identities,
polynomial exactness of the stencils, closed forms of the history integral,
an independent recursion, conservation laws, symmetries, and the Newtonian
channel solution.  A plausible mistake in any step (dropped term, wrong sign
or index, transposed operand) fails at least one of them.
"""
import json
import math
import os

import numpy as np
import pytest

import oracle
import workloads

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _paper():
    with open(os.path.join(GOLDEN, "paper_constants.json")) as f:
        return json.load(f)


# --------------------------------------------------------------------------
# Lattice constants (Sec. III)
# --------------------------------------------------------------------------

def test_lattice_matches_printed_d2q9():
    p = _paper()
    cx, cy, w, opp = oracle.lattice()
    vel = p["d2q9_velocities"]["value"]
    wts = p["d2q9_weights"]["value"]
    got = {(int(a), int(b)): float(c) for a, b, c in zip(cx, cy, w)}
    for cls in ("rest", "axis", "diagonal"):
        for v in vel[cls]:
            assert got[tuple(v)] == pytest.approx(wts[cls], abs=1e-16)
    assert len(got) == 9
    for i in range(9):
        assert cx[opp[i]] == -cx[i] and cy[opp[i]] == -cy[i]
    # second moment of the weights fixes c_s^2 (isotropy of D2Q9)
    cs2 = p["sound_speed_squared"]["value"]
    assert np.sum(w * cx * cx) == pytest.approx(cs2, abs=1e-16)
    assert np.sum(w * cx * cy) == pytest.approx(0.0, abs=1e-16)
    assert np.sum(w) == pytest.approx(1.0, abs=1e-15)


# --------------------------------------------------------------------------
# Equilibrium and forcing (Sec. III): defining moments
# --------------------------------------------------------------------------

@pytest.mark.parametrize("seed", range(5))
def test_equilibrium_moments(seed):
    rng = np.random.default_rng(seed)
    rho = 1.0 + 0.1 * rng.standard_normal()
    u = 0.05 * rng.standard_normal(2)
    cx, cy, _, _ = oracle.lattice()
    neq = oracle.equilibrium(rho, u[0], u[1])
    cs2 = 1.0 / 3.0
    assert neq.sum() == pytest.approx(rho, rel=1e-14)
    assert (cx * neq).sum() == pytest.approx(rho * u[0], abs=1e-15)
    assert (cy * neq).sum() == pytest.approx(rho * u[1], abs=1e-15)
    c = np.stack([cx, cy])
    for a in range(2):
        for b in range(2):
            pi = (c[a] * c[b] * neq).sum()
            want = rho * cs2 * (a == b) + rho * u[a] * u[b]
            assert pi == pytest.approx(want, abs=1e-15)


@pytest.mark.parametrize("tau", [0.6, 0.9, 1.0, 1.7])
def test_force_term_moments(tau):
    rng = np.random.default_rng(7)
    u = 0.05 * rng.standard_normal(2)
    f = 1e-4 * rng.standard_normal(2)
    cx, cy, _, _ = oracle.lattice()
    F = oracle.force_term(tau, u[0], u[1], f[0], f[1])
    pre = 1.0 - 1.0 / (2.0 * tau)
    c = np.stack([cx, cy])
    assert abs(F.sum()) < 1e-19
    for a in range(2):
        assert (c[a] * F).sum() == pytest.approx(pre * f[a], rel=1e-13)
        for b in range(2):
            want = pre * (u[a] * f[b] + u[b] * f[a])
            assert (c[a] * c[b] * F).sum() == pytest.approx(want, abs=1e-20)


def test_collision_conserves_mass_and_adds_force_momentum():
    """With u = (j + f/2)/rho (Eq. hydrofields) one collision changes the
    momentum by exactly f and leaves the mass unchanged."""
    rng = np.random.default_rng(3)
    cx, cy, w, _ = oracle.lattice()
    for tau in (0.7, 1.0, 1.4):
        n = w * (1.0 + 0.05 * rng.standard_normal(9))
        f = 1e-3 * rng.standard_normal(2)
        rho, jx, jy = oracle.density_momentum(n)
        ux, uy = (jx + f[0] / 2) / rho, (jy + f[1] / 2) / rho
        ns = oracle.collide(tau, n, rho, ux, uy, f[0], f[1])
        assert ns.sum() == pytest.approx(rho, rel=1e-15)
        assert (cx * ns).sum() == pytest.approx(jx + f[0], abs=1e-16)
        assert (cy * ns).sum() == pytest.approx(jy + f[1], abs=1e-16)


# --------------------------------------------------------------------------
# Streaming with bounce-back walls
# --------------------------------------------------------------------------

def test_stream_moves_and_reflects():
    lx, ly = 5, 4
    cx, cy, _, opp = oracle.lattice()
    for i in range(9):
        for (x, y) in [(0, 0), (2, 1), (4, 3), (3, 2)]:
            ns = np.zeros((9, ly, lx))
            ns[i, y, x] = 1.0
            out = oracle.stream(ns)
            yy = y + cy[i]
            if 0 <= yy < ly:
                assert out[i, yy, (x + cx[i]) % lx] == 1.0
            else:
                assert out[opp[i], y, x] == 1.0
            assert out.sum() == 1.0


def test_stream_is_a_permutation():
    rng = np.random.default_rng(0)
    ns = rng.permutation(9 * 3 * 7).astype(float).reshape(9, 3, 7)
    out = oracle.stream(ns)
    assert np.array_equal(np.sort(out.ravel()), np.sort(ns.ravel()))


# --------------------------------------------------------------------------
# Finite-difference stencils: exact on quadratics
# --------------------------------------------------------------------------

def test_velocity_gradient_exact_on_wall_quadratics():
    """A quadratic vanishing at both halfway walls y = -1/2, ly - 1/2 is
    differentiated exactly at every row, including the wall rows."""
    lx, ly = 6, 9
    y = np.arange(ly)[:, None] * np.ones((1, lx))
    a, b = 1.7e-3, -0.6e-3
    ux = a * (y + 0.5) * (ly - 0.5 - y)
    uy = b * (y + 0.5) * (ly - 0.5 - y)
    kxx, kxy, kyx, kyy = oracle.velocity_gradient(ux, uy)
    d = (ly - 1 - 2 * y)
    np.testing.assert_allclose(kxy, a * d, rtol=0, atol=1e-17)
    np.testing.assert_allclose(kyy, b * d, rtol=0, atol=1e-17)
    assert np.abs(kxx).max() == 0 and np.abs(kyx).max() == 0


def test_velocity_gradient_x_is_periodic_central():
    lx, ly = 8, 5
    x = np.arange(lx)[None, :] * np.ones((ly, 1))
    k = 2 * math.pi / lx
    ux = np.sin(k * x)
    uy = 0.3 * np.cos(k * x)
    kxx, kxy, kyx, kyy = oracle.velocity_gradient(ux, uy)
    np.testing.assert_allclose(kxx, math.sin(k) * np.cos(k * x), atol=1e-15)
    np.testing.assert_allclose(kyx, -0.3 * math.sin(k) * np.sin(k * x), atol=1e-15)
    # y-constant field: zero interior y-derivative; at the wall rows the
    # quadratic through the wall value 0 gives +-4/3 of the field value
    assert np.abs(kxy[1:-1]).max() == 0 and np.abs(kyy[1:-1]).max() == 0
    np.testing.assert_allclose(kxy[0], 4.0 / 3.0 * ux[0], atol=1e-15)
    np.testing.assert_allclose(kxy[-1], -4.0 / 3.0 * ux[-1], atol=1e-15)


def test_stress_divergence_exact_on_quadratics():
    lx, ly = 4, 7
    y = np.arange(ly)[:, None] * np.ones((1, lx))
    sxy = 2e-4 + 3e-5 * y - 7e-6 * y * y
    sxx = np.zeros((ly, lx))
    fx, fy = oracle.stress_divergence(sxx, sxy)
    np.testing.assert_allclose(fx, 3e-5 - 14e-6 * y, rtol=0, atol=1e-18)
    assert np.abs(fy).max() == 0.0
    # x-dependence enters f_x through sigma_xx and f_y through sigma_xy
    x = np.arange(lx)[None, :] * np.ones((ly, 1))
    k = 2 * math.pi / lx
    fx, fy = oracle.stress_divergence(np.cos(k * x), np.sin(k * x))
    np.testing.assert_allclose(fx, -math.sin(k) * np.sin(k * x), atol=1e-15)
    np.testing.assert_allclose(fy, math.sin(k) * np.cos(k * x), atol=1e-15)


def test_shear_rate_invariants():
    """II_D = (1/2) tr D^2 with D = kappa + kappa^T (Sec. II)."""
    assert oracle.shear_rate(0, 3e-3, 0, 0) == pytest.approx(3e-3, rel=1e-15)
    assert oracle.shear_rate(0, -3e-3, 0, 0) == pytest.approx(3e-3, rel=1e-15)
    # planar extension diag(e, -e): II_D = 4 e^2
    assert oracle.shear_rate(2e-3, 0, 0, -2e-3) == pytest.approx(4e-3, rel=1e-15)
    # rigid rotation carries no shear rate (frame indifference)
    assert oracle.shear_rate(0, 5e-3, -5e-3, 0) == 0.0


# --------------------------------------------------------------------------
# History integral: closed forms, limits, recursion
# --------------------------------------------------------------------------

G, TAU, GC = 1e-3, 100.0, 0.1


def _const_history(n_hist, t, s):
    """Age arrays for constant shear s switched on at t' = 0."""
    live = min(t + 1, n_hist)
    s_age = np.zeros(n_hist)
    s_age[:live] = s
    r_age = np.abs(s_age)
    return s_age, r_age


@pytest.mark.parametrize("s", [1e-4, -2e-3, 5e-2])
@pytest.mark.parametrize("t", [0, 1, 7, 300])
def test_history_constant_shear_untruncated(s, t):
    """t < N_h - 1: sigma_xy = G s [(1 - q^{t+1})/(1 - q) - 1/2],
    N1 = 2 G s^2 q (1 - (t+1) q^t + t q^{t+1}) / (1 - q)^2."""
    n_hist = 1000
    s_age, r_age = _const_history(n_hist, t, s)
    sxy, n1 = oracle.history_sum_ages(s_age, r_age, G, TAU, GC)
    lam = 1.0 / TAU + abs(s) / GC
    q = math.exp(-lam)
    want_xy = G * s * ((1 - q ** (t + 1)) / (1 - q) - 0.5)
    want_n1 = 2 * G * s * s * q * (1 - (t + 1) * q ** t + t * q ** (t + 1)) / (1 - q) ** 2
    assert sxy == pytest.approx(want_xy, rel=1e-12)
    assert n1 == pytest.approx(want_n1, rel=1e-10, abs=1e-30)


@pytest.mark.parametrize("n_hist", [2, 3, 50, 1000])
def test_history_constant_shear_truncated(n_hist):
    """t >= N_h - 1, n = N_h - 1: sigma_xy = G s (1+q)(1-q^n) / (2(1-q)),
    N1 = 2 G s^2 [sum_{k<=n} k q^k - n q^n / 2]."""
    s = 3e-3
    s_age = np.full(n_hist, s)
    sxy, n1 = oracle.history_sum_ages(s_age, np.abs(s_age), G, TAU, GC)
    lam = 1.0 / TAU + s / GC
    q = math.exp(-lam)
    n = n_hist - 1
    want_xy = G * s * (1 + q) * (1 - q ** n) / (2 * (1 - q))
    # sum_{k=1}^{n} k q^k in closed form
    skq = q * (1 - (n + 1) * q ** n + n * q ** (n + 1)) / (1 - q) ** 2
    want_n1 = 2 * G * s * s * (skq - 0.5 * n * q ** n)
    assert sxy == pytest.approx(want_xy, rel=1e-12)
    assert n1 == pytest.approx(want_n1, rel=1e-11)


def test_history_steady_state_matches_instantaneous_nlm():
    """Long-time constant shear reproduces the steady nlM of Eq. (inlM):
    sigma_xy = G tau_M s and N1 = 2 G tau_M^2 s^2 with
    tau_M = 1/(1/tau + |s|/gamma_c), up to the trapezoid factors
    (lam/2)coth(lam/2) and (lam/2)^2/sinh^2(lam/2) (both 1 + O(lam^2))."""
    n_hist = 20000
    for s in (1e-5, 1e-4, 1e-3):
        s_age = np.full(n_hist, s)
        sxy, n1 = oracle.history_sum_ages(s_age, np.abs(s_age), G, TAU, GC)
        lam = 1.0 / TAU + s / GC
        tau_m = 1.0 / lam
        fac_xy = (lam / 2) / math.tanh(lam / 2)
        fac_n1 = (lam / 2) ** 2 / math.sinh(lam / 2) ** 2
        assert sxy == pytest.approx(G * tau_m * s * fac_xy, rel=1e-12)
        assert n1 == pytest.approx(2 * G * tau_m ** 2 * s * s * fac_n1, rel=1e-9)
        assert abs(fac_xy - 1) < lam ** 2 / 11 and abs(fac_n1 - 1) < lam ** 2 / 11


def test_history_maxwell_relation_and_yield_stress():
    """Small shear: sigma/s -> eta = G tau (Maxwell relation, Sec. I).
    Glassy limit tau -> infinity, s >> gamma_c/tau: sigma_xy -> G gamma_c
    (yield stress of the model, Sec. IV.A)."""
    p = _paper()
    n_hist = 30000
    s = 1e-7
    s_age = np.full(n_hist, s)
    sxy, _ = oracle.history_sum_ages(s_age, np.abs(s_age), G, TAU, GC)
    assert sxy / s == pytest.approx(G * TAU, rel=1e-4)
    gc = p["gamma_c"]["value"]
    s = 1e-3   # lam = s/gamma_c = 0.01, trapezoid factor 1 + lam^2/12
    s_age = np.full(n_hist, s)
    sxy, _ = oracle.history_sum_ages(s_age, np.abs(s_age), G, 1e9, gc)
    assert sxy == pytest.approx(G * gc, rel=2e-5)


def test_history_linear_maxwell_startup():
    """Linear Maxwell model, Eq. (maxwell), at constant shear from t = 0:
    sigma(t) = G tau s (1 - exp(-t/tau)).  The discrete sum differs by the
    endpoint weight at t' = 0 (at most G s/2 exp(-t/tau)) and by the
    trapezoid factor (1/2tau) coth(1/2tau) = 1 + O(1/tau^2)."""
    n_hist = 5000
    s = 1e-3
    tau = 100.0
    for t in (10, 100, 400, 2000):
        s_age, _ = _const_history(n_hist, t, s)
        sxy, _ = oracle.history_sum_ages(s_age, np.zeros(n_hist), G, tau, math.inf)
        cont = G * tau * s * (1 - math.exp(-t / tau))
        bound = 0.5 * G * s * math.exp(-t / tau) + 0.5 * G * s + G * tau * s / (12 * tau ** 2)
        assert abs(sxy - cont) <= bound
    # t -> infinity: sigma = G s (1/2) coth(1/(2 tau)); relative to G tau s
    s_age = np.full(n_hist, s)
    sxy, _ = oracle.history_sum_ages(s_age, np.zeros(n_hist), G, tau, math.inf)
    want = G * tau * s * (0.5 / tau) / math.tanh(0.5 / tau) * (1 - math.exp(-(n_hist - 1) / tau))
    assert sxy == pytest.approx(want, rel=1e-6)
    assert sxy / (G * tau * s) - 1 == pytest.approx(1.0 / (12 * tau ** 2), rel=1e-2)


def _recursive_ucm(s_seq, q, n_hist):
    """Independent O(1)-per-step recursions for the linear (UCM) case:
    R_t = sum_{k<N} q^k s_{t-k} = q R_{t-1} + s_t - q^N s_{t-N},
    P_t = sum_{k<N} q^k s_{t-k} gamma_{t,t-k}
        = q (P_{t-1} + s_{t-1} R_{t-1}) - q^N s_{t-N} gamma_{t,t-N}.
    The half weights at k = 0 and k = N - 1 are applied afterwards."""
    T = len(s_seq)
    R = P = 0.0
    Gam = np.concatenate([[0.0], np.cumsum(s_seq)])  # Gamma_t = sum_{j<t} s_j
    out = []
    qN = q ** n_hist
    for t in range(T):
        s_prev = s_seq[t - 1] if t >= 1 else 0.0
        old = s_seq[t - n_hist] if t - n_hist >= 0 else 0.0
        g_old = Gam[t] - Gam[t - n_hist] if t - n_hist >= 0 else 0.0
        P = q * (P + s_prev * R) - qN * old * g_old
        R = q * R + s_seq[t] - qN * old
        k_last = n_hist - 1
        s_last = s_seq[t - k_last] if t - k_last >= 0 else 0.0
        g_last = Gam[t] - Gam[t - k_last] if t - k_last >= 0 else 0.0
        sxy = R - 0.5 * s_seq[t] - 0.5 * q ** k_last * s_last
        sxx = 2 * (P - 0.5 * q ** k_last * s_last * g_last)
        out.append((sxy, sxx))
    return np.array(out)


@pytest.mark.parametrize("n_hist", [2, 5, 64])
def test_history_brute_force_equals_recursion(n_hist):
    """Linear case (gamma_c = inf): the brute-force window sum with the
    accumulated strain from the Gamma prefix equals the recursions."""
    rng = np.random.default_rng(11)
    T = 3 * n_hist + 17
    s_seq = 1e-3 * rng.standard_normal(T)
    tau = 7.0
    q = math.exp(-1.0 / tau)
    rec = _recursive_ucm(s_seq, q, n_hist)
    for t in range(T):
        s_age = np.zeros(n_hist)
        for k in range(n_hist):
            if t - k >= 0:
                s_age[k] = s_seq[t - k]
        sxy, sxx = oracle.history_sum_ages(s_age, np.abs(s_age), 1.0, tau, math.inf)
        assert sxy == pytest.approx(rec[t, 0], rel=1e-12, abs=1e-18)
        assert sxx == pytest.approx(rec[t, 1], rel=1e-9, abs=1e-18)


def test_history_damping_uses_past_shear_rate():
    """Eq. (nlmax): the damping exp(-(t-t')|gamma_dot(t')|/gamma_c) takes the
    shear rate at the past time t', not the current one."""
    n_hist = 40
    s_age = np.zeros(n_hist)
    r_age = np.zeros(n_hist)
    s_age[10] = 1e-3
    r_age[10] = 0.0        # the past entry was unsheared
    r_age[0] = 1e3         # a huge current shear rate must not damp it
    sxy, _ = oracle.history_sum_ages(s_age, r_age, 1.0, 50.0, 0.1)
    assert sxy == pytest.approx(1e-3 * math.exp(-10 / 50.0), rel=1e-15)


# --------------------------------------------------------------------------
# Whole channel: conservation, Newtonian solution, symmetries, LTI identity
# --------------------------------------------------------------------------

def test_mass_conserved_2d_nlm():
    ch = workloads.large_2d(lx=8, ly=12, n_hist=64).channels[0]
    ch = ch.replace(tau_m=30.0)
    oc = oracle.OracleChannel(ch)
    m0 = oc.mass()
    oc.step(300)
    assert abs(oc.mass() - m0) / m0 < 1e-13


def test_newtonian_poiseuille_exact():
    """G_inf = 0: the steady BGK channel flow with the half-force velocity and
    halfway bounce-back is the parabola (viscosity (tau_LB - 1/2)/3, Sec. III)
    plus the uniform slip g (16 tau^2 - 16 tau + 1) / (24 nu)."""
    p = _paper()
    assert "tau_LB - 1/2" in p["newtonian_viscosity"]["value"]
    for tau in (0.8, 1.0):
        ly, g = 12, 1e-6
        ch = workloads.Channel(lx=1, ly=ly, tau_lb=tau, g_inf=0.0, n_hist=2, gx=g)
        oc = oracle.OracleChannel(ch)
        oc.step(20000)
        _, ux, uy = oc.fields()
        nu = (tau - 0.5) / 3.0
        y = np.arange(ly)
        want = g / (2 * nu) * (y + 0.5) * (ly - 0.5 - y) + g * (16 * tau ** 2 - 16 * tau + 1) / (24 * nu)
        np.testing.assert_allclose(ux[:, 0], want, rtol=1e-9)
        assert np.abs(uy).max() < 1e-9 * np.abs(ux).max()  # rounding level


def test_newtonian_momentum_diffusion_time():
    """Cessation of Newtonian channel flow decays with the slowest diffusive
    mode, rate 1/t_wall = pi^2 nu / (2H)^2 (Sec. IV.B, with eta_inf the BGK
    viscosity and 2H = ly); the lattice value converges at O(ly^-2)."""
    errs = []
    for ly in (16, 32):
        ch = workloads.Channel(lx=1, ly=ly, tau_lb=1.0, g_inf=0.0, n_hist=2, gx=1e-6)
        oc = oracle.OracleChannel(ch)
        nu = 0.5 / 3.0
        t_wall = ly * ly / (math.pi ** 2 * nu)
        oc.step(int(2 * t_wall))
        oc.set_force(0.0)
        oc.step(int(1.5 * t_wall))
        u1 = oc.fields()[1][ly // 2, 0]
        dt = int(0.5 * t_wall)
        oc.step(dt)
        u2 = oc.fields()[1][ly // 2, 0]
        rate = -math.log(u2 / u1) / dt
        errs.append(abs(rate * t_wall - 1))
    assert errs[0] < 0.05 and errs[1] < errs[0] / 3


@pytest.mark.parametrize("model", ["newtonian", "ucm"])
def test_startup_cessation_symmetry_linear_models(model):
    """Linear models (Newtonian, UCM) obey u_off(T0 + t) = u_on(T0 + t) - u_on(t)
    (Sec. IV.B, startup/cessation symmetry)."""
    g_inf = 0.0 if model == "newtonian" else 1e-3
    ch = workloads.Channel(lx=1, ly=16, tau_lb=1.0, g_inf=g_inf, tau_m=50.0,
                           gamma_c=math.inf, n_hist=300, gx=1e-6)
    T0, T1 = 400, 300
    on = oracle.OracleChannel(ch)
    u_on = []
    for _ in range(T0 + T1):
        on.step(1)
        u_on.append(on.fields()[1][:, 0].copy())
    off = oracle.OracleChannel(ch)
    off.step(T0)
    off.set_force(0.0)
    scale = np.abs(u_on).max()
    for t in range(T1):
        off.step(1)
        u_off = off.fields()[1][:, 0]
        want = u_on[T0 + t] - u_on[t]
        assert np.abs(u_off - want).max() / scale < 1e-11


def test_channel_symmetries():
    """Mirror symmetry about the channel centre, odd symmetry under g -> -g,
    and exact x-invariance for an x-invariant start."""
    base = workloads.Channel(lx=4, ly=10, tau_lb=1.0, g_inf=1e-3, tau_m=40.0,
                             gamma_c=0.1, n_hist=120, gx=2e-5)
    a = oracle.OracleChannel(base)
    b = oracle.OracleChannel(base.replace(gx=-2e-5))
    a.step(250)
    b.step(250)
    _, ua, va = a.fields()
    sa, na = a.stress()
    _, ub, _ = b.fields()
    sb, nb = b.stress()
    # x-invariance: all columns identical
    for arr in (ua, sa, na):
        assert np.array_equal(arr, arr[:, :1] * np.ones((1, 4)))
    # mirror: u even, sigma_xy odd, N1 even about the centre line
    sc = np.abs(ua).max()
    assert np.abs(ua - ua[::-1]).max() / sc < 1e-12
    assert np.abs(sa + sa[::-1]).max() / np.abs(sa).max() < 1e-10
    assert np.abs(na - na[::-1]).max() / np.abs(na).max() < 1e-10
    # sign: u and sigma_xy flip, N1 unchanged
    np.testing.assert_allclose(ub, -ua, rtol=1e-13, atol=1e-22)
    np.testing.assert_allclose(sb, -sa, rtol=1e-12, atol=1e-24)
    np.testing.assert_allclose(nb, na, rtol=1e-12, atol=1e-28)
    # the paper's claim N1 = sigma_xx - sigma_yy >= 0 in channel flow (Sec. IV.B)
    assert na.min() >= 0.0


def test_ucm_steady_centreline_maxwell_relation():
    """UCM steady channel flow has the effective viscosity nu + eta_s with the
    discrete Maxwell viscosity eta_s = G (1/2) coth(1/(2 tau)) (Sec. I relation
    eta = G tau up to O(tau^-2)); the centreline velocity approaches
    g ly^2 / (8 nu_eff) at second order in 1/ly."""
    errs = []
    for ly in (12, 24):
        g, tau, Gm = 1e-6, 15.0, 5e-3
        ch = workloads.Channel(lx=1, ly=ly, tau_lb=1.0, g_inf=Gm, tau_m=tau,
                               gamma_c=math.inf, n_hist=600, gx=g)
        oc = oracle.OracleChannel(ch)
        nu = 0.5 / 3
        eta_s = Gm * 0.5 / math.tanh(0.5 / tau) * (1 - math.exp(-599 / tau))
        nu_eff = nu + eta_s
        t_wall = ly * ly / (math.pi ** 2 * nu_eff)
        oc.step(int(25 * t_wall) + 1000)
        _, ux, _ = oc.fields()
        uc = 0.5 * (ux[ly // 2, 0] + ux[ly // 2 - 1, 0])
        y = ly / 2 - 0.5
        want = g / (2 * nu_eff) * (y + 0.5) * (ly - 0.5 - y)
        errs.append(abs(uc / want - 1))
    assert errs[0] < 0.05
    assert errs[1] < errs[0] / 3


@pytest.mark.parametrize("twall_over_tau0", [0.1, 1.0])
def test_ucm_startup_matches_the_modal_solution_at_second_order(twall_over_tau0):
    """Appendix, Fig. UCM: startup channel flow of the UCM with the background
    viscosity (theta = 10, the figure's two widths) against its closed form
    (the modal solution of tests/closed_forms.py, the problem Waters and King
    solved), every node over six t_wall.  The oracle's error shrinks about
    fourfold when the channel doubles: second order in 1/H."""
    from closed_forms import channel_node_positions, maxwell_channel_startup
    errs = []
    for half in (4, 8):
        ch = workloads.sec4_channel(twall_over_tau0, 10.0, "ucm", half_width=half)
        eta = (ch.tau_lb - 0.5) / 3.0
        steps = int(round(6 * workloads.sec4_wall_time(half)))
        every = max(1, steps // 60)
        oc = oracle.OracleChannel(ch)
        ts, us, done = [], [], 0
        while done < steps:
            oc.step(every)
            done += every
            ts.append(done)
            us.append(oc.fields()[1][:, 0].copy())
        ref = maxwell_channel_startup(channel_node_positions(ch.ly), ts, half, 1.0, eta,
                                      ch.g_inf, ch.tau_m, ch.gx)
        errs.append(float(np.abs(np.array(us) - ref).max() / np.abs(ref).max()))
    assert errs[0] < 2e-2 and errs[1] < 5e-3, errs
    assert errs[0] / errs[1] > 3.5, errs


@pytest.mark.parametrize("twall_over_tau0", [0.1, 1.0])
def test_nonlinear_startup_departs_from_ucm_at_first_order_in_the_driving(twall_over_tau0):
    """Eq. nlmax with gamma_c large against the shear the driving produces:
    the damping adds |s'|/gamma_c to each entry's decay rate, a correction of
    first order in the shear rate, so the startup flow departs from the UCM
    flow (gamma_c = inf, linear in the force) by a relative amount
    proportional to the driving -- halving the force halves it -- and, since
    damping only removes stress, the nonlinear flow is nowhere slower.  A
    dropped damping term gives no departure; a wrong sign, a slower flow; a
    damping of the wrong order in s, another ratio."""
    base = workloads.sec4_channel(twall_over_tau0, 10.0, "ucm", half_width=4)
    eta = (base.tau_lb - 0.5) / 3.0
    steps = int(round(6 * workloads.sec4_wall_time(4)))
    every = max(1, steps // 60)
    # the steady wall shear rate of the linear flow sets gamma_c: a departure
    # of about 1e-3 to 1e-2, far above rounding and with second-order terms
    # near 1e-5
    s_wall = base.gx * 4 / (eta + base.g_inf * base.tau_m)
    gamma_c = 100.0 * s_wall * base.tau_m

    def run(ch):
        oc = oracle.OracleChannel(ch)
        us = []
        for _ in range(steps // every):
            oc.step(every)
            us.append(oc.fields()[1][:, 0].copy())
        oc.close()
        return np.array(us)

    ucm = run(base)
    dev = []
    for amp in (1.0, 0.5):
        nlm = run(base.replace(gx=amp * base.gx, gamma_c=gamma_c))
        lin = amp * ucm
        scale = np.abs(lin).max()
        dev.append(np.abs(nlm - lin).max() / scale)
        assert (nlm - lin).min() >= -1e-12 * scale
    assert dev[0] > 1e-4, dev
    assert 1.95 < dev[0] / dev[1] < 2.05, dev


@pytest.mark.parametrize("kw", [{}, {"finger": True}, {"law": "strain_damping"},
                                {"paper_coupling": True}])
def test_short_window_equals_long_window_before_it_fills(kw):
    """The ring starts zero-filled (rest before t = 0), so before step
    n_hist - 1 the entries past the pushed ones are exact zeros (zero shear
    rate and gradient: no stress term, an identity deformation factor, no
    accumulated strain) and the end weight falls on a zero: a 128-entry
    window gives the same numbers as the 4096-entry one up to step 126, bit
    for bit, for every law and tensor form (the identity the stored
    full-size 96-step runs rely on)."""
    base = workloads.large_2d(lx=12, ly=10, n_hist=4096).channels[0].replace(**kw)
    outs = []
    for h in (4096, 128):
        oc = oracle.OracleChannel(base.replace(n_hist=h))
        oc.step(126)
        outs.append(oc.fields() + oc.stress() + (oc.grad(),))
        oc.close()
    for a, b in zip(*outs):
        assert np.array_equal(a, b)


def test_nlm_steady_channel_solves_the_pointwise_momentum_balance():
    """Steady shear-thinning channel flow (Sec. IV, steady state): integrating
    the momentum balance from the centre line gives, at each height,
    nu s + sigma_ss(s) = -g (y - y_c), where sigma_ss(s) is the history sum of
    Eq. (gitt) with the modulus of Eq. (nlmax) for a shear rate held at s over
    the whole window (fixed trapezoid weights, n_hist entries).  Solved
    pointwise with a root finder, independently of the coupled lattice /
    history iteration; the oracle's steady shear rate must approach it at
    second order in 1/ly (g scaled with 1/ly keeps the shear-rate profile,
    here thinned to about half the Maxwell stress at the walls)."""
    from scipy.optimize import brentq

    errs = []
    for ly, steps in ((16, 6000), (32, 20000)):
        g, tau, Gm, gc, H = 1e-4 * 16 / ly, 12.0, 4e-3, 0.05, 400
        ch = workloads.Channel(lx=1, ly=ly, tau_lb=1.0, g_inf=Gm, tau_m=tau, gamma_c=gc,
                               n_hist=H, gx=g)
        oc = oracle.OracleChannel(ch)
        oc.step(steps)
        s = oc.grad()[1][:, 0]
        oc.close()
        nu = 0.5 / 3
        w = np.ones(H)
        w[0] = w[-1] = 0.5
        k = np.arange(H)

        def sig(sv):
            return Gm * sv * np.sum(w * np.exp(-k * (1.0 / tau + abs(sv) / gc)))

        yc = (ly - 1) / 2
        want = np.array([brentq(lambda sv: nu * sv + sig(sv) + g * (y - yc), -1.0, 1.0)
                         for y in range(ly)])
        # thinning is strong: sigma_ss / (G tau s) at the largest rate
        smax = np.abs(want).max()
        assert sig(smax) / (Gm * tau * smax) < 0.6
        inner = slice(2, ly - 2)
        errs.append(np.abs(s[inner] - want[inner]).max() / smax)
    assert errs[0] < 3e-3, errs
    assert errs[1] < errs[0] / 3, errs


# --------------------------------------------------------------------------
# Quasi-logarithmic history grid (Sec. III)
# --------------------------------------------------------------------------

def _drive(grid, kappa_hist):
    for k in kappa_hist:
        grid.push(*k)


def _seeded_kappa(n, seed, scale=1e-3):
    rng = np.random.default_rng(workloads.BASE_SEED + seed)
    return rng.uniform(-scale, scale, size=(n, 4))


@pytest.mark.parametrize("B,C,t", [(1, 5, 17), (3, 4, 19), (3, 4, 64), (4, 6, 101),
                                   (5, 128, 1000)])
def test_qgrid_structure(B, C, t):
    """Block steps double going back, entries tile time without gaps, the
    newest is the current step, and every block holds C or C - 1 entries."""
    g = oracle.QGrid(B, C)
    _drive(g, np.zeros((t + 1, 4)))
    t0, dt, _, _ = g.entries()
    assert t0[0] == t and dt[0] == 1
    assert np.all(t0[:-1] == t0[1:] + dt[1:])          # contiguous, newest first
    assert set(np.unique(dt)) == {2.0 ** k for k in range(B)}
    assert np.all(np.diff(dt) >= 0)                      # steps only grow with age
    for k in range(B):
        assert np.sum(dt == 2.0 ** k) in (C - 1, C)
    # the grid reaches back about C (2^B - 1) steps
    span = t0[0] + dt[0] - t0[-1]
    assert C * (2 ** B - 1) - 2 ** B <= span <= C * (2 ** B - 1) + 1


@pytest.mark.parametrize("B,C", [(3, 4), (4, 8), (6, 16)])
def test_qgrid_entries_hold_interval_means_and_exact_strain(B, C):
    """Each entry's kappa is the mean of the step kappas over its interval
    (zero before t = 0), and its strain is the exact sum of the step shear
    rates from its start to t - 1: combining two entries averages kappa and
    multiplies the deformation factors."""
    T = C * 2 ** B + 37
    kap = _seeded_kappa(T, 40 + B)
    g = oracle.QGrid(B, C)
    _drive(g, kap)
    t = T - 1
    t0, dt, k4, strain = g.entries()

    def raw(a, b):  # rows for steps a .. b-1, zeros before 0
        out = np.zeros((b - a, 4))
        for i, tt in enumerate(range(a, b)):
            if tt >= 0:
                out[i] = kap[tt]
        return out

    for e in range(len(t0)):
        a, b = int(t0[e]), int(t0[e] + dt[e])
        np.testing.assert_allclose(k4[e], raw(a, b).mean(axis=0), rtol=0, atol=1e-18)
        want = raw(a, t)[:, 1].sum() if e > 0 else 0.0
        assert abs(strain[e] - want) <= 1e-15, (e, strain[e], want)


@pytest.mark.parametrize("C,t", [(8, 30), (9, 31), (64, 500)])
def test_qgrid_single_block_is_the_uniform_window(C, t):
    """With one block the grid is a uniform window of the last C (or C - 1)
    steps, and its integral equals the uniform-window history sum of that
    length."""
    kap = _seeded_kappa(t + 1, 50 + C, scale=2e-2)
    g = oracle.QGrid(1, C)
    _drive(g, kap)
    t0, dt, _, _ = g.entries()
    n = len(t0)
    assert n in (C, C - 1) and np.all(dt == 1) and t0[-1] == t - n + 1
    s_age = kap[::-1][:n, 1]
    r_age = np.array([oracle.shear_rate(*kap[t - a]) for a in range(n)])
    for G, tau, gc in ((1e-3, 7.0, 0.1), (2e-3, 40.0, math.inf)):
        want = oracle.history_sum_ages(s_age, r_age, G, tau, gc)
        got = g.sum(G, tau, gc)
        np.testing.assert_allclose(got, want, rtol=1e-13, atol=0)


@pytest.mark.parametrize("B,C,tau", [(4, 128, 200.0), (6, 128, 1000.0), (3, 64, 50.0)])
def test_qgrid_constant_shear_continuum_limit(B, C, tau):
    """Constant shear rate s for longer than the grid reaches back (UCM, no
    damping): the non-uniform trapezoid rule gives the continuum integrals
    sigma_xy = G s tau (1 - e^{-A/tau}) and N1 = 2 G s^2 tau^2 (1 - e^{-A/tau}
    (1 + A/tau)) over the grid's reach A, within the trapezoid error bound
    h^2 / (12 tau^2) of the widest step h."""
    s, G = 3e-4, 1e-3
    T = C * 2 ** (B + 1)
    g = oracle.QGrid(B, C)
    _drive(g, np.tile([0.0, s, 0.0, 0.0], (T, 1)))
    t0, dt, _, _ = g.entries()
    assert t0[-1] >= 0                    # only sheared entries left
    A = (T - 1) - t0[-1]
    sxy, sxx = g.sum(G, tau, math.inf)
    want_xy = G * s * tau * (1 - math.exp(-A / tau))
    want_n1 = 2 * G * s * s * tau * tau * (1 - math.exp(-A / tau) * (1 + A / tau))
    bound = dt.max() ** 2 / (12 * tau ** 2)
    assert abs(sxy / want_xy - 1) <= 1.5 * bound, (sxy, want_xy, bound)
    assert abs(sxx / want_n1 - 1) <= 3.0 * bound, (sxx, want_n1, bound)


def test_qgrid_damping_uses_the_averaged_gradient():
    """The damping of a combined entry is sqrt(II_D) of its averaged kappa.
    Grid X sees kappa_xx = +b, -b, +b, ... and grid Y kappa_xx = +b always,
    both with kappa_xy = a: every single step has the same shear rate and the
    same |gamma_dot| in both, so they differ only where entries were combined
    -- X's averaged kappa_xx is 0 there (damping |a|), Y's is b.  Averaging
    the rates instead would make the two sums equal."""
    B, C, T = 3, 8, 200
    a, b = 2e-3, 4e-2
    gx, gy = oracle.QGrid(B, C), oracle.QGrid(B, C)
    for t in range(T):
        gx.push(b * (-1) ** t, a, 0.0, 0.0)
        gy.push(b, a, 0.0, 0.0)
    tx, dx, kx, _ = gx.entries()
    ty, dy, ky, _ = gy.entries()
    assert np.array_equal(tx, ty) and np.array_equal(dx, dy)
    merged = dx > 1
    assert np.allclose(kx[merged, 0], 0.0, atol=1e-18) and np.allclose(ky[merged, 0], b)
    G, tau, gc = 1e-3, 60.0, 5e-3
    sx, _ = gx.sum(G, tau, gc)
    sy, _ = gy.sum(G, tau, gc)
    # X's combined entries are damped by |a| instead of sqrt(2 b^2 + a^2)
    assert sx > sy * (1 + 1e-3), (sx, sy)
    # without damping the two grids carry the same shear history
    assert abs(gx.sum(G, tau, math.inf)[0] - gy.sum(G, tau, math.inf)[0]) <= 1e-18


# --------------------------------------------------------------------------
# Full-tensor Finger path (Eq. gitt, -d_t'B = E kappa E^T + transpose,
# Eq. eeval)
# --------------------------------------------------------------------------

def test_expm2_matches_scipy():
    import scipy.linalg as sla
    rng = np.random.default_rng(workloads.BASE_SEED + 60)
    for scale in (1e-6, 1e-3, 0.1, 1.0, 7.0):
        for _ in range(20):
            a = rng.normal(size=(2, 2)) * scale
            want = sla.expm(a)
            got = oracle.expm2(a)
            # forward error of scaling and squaring: rounding relative to
            # e^{|A|}, doubled by each squaring
            nrm = np.abs(a).sum()
            sq = max(0, math.ceil(math.log2(max(nrm / 0.25, 1.0))))
            assert np.abs(got - want).max() <= 4e-15 * 2 ** sq * math.exp(nrm)


def _shear_history(n, seed, scale=2e-3):
    rng = np.random.default_rng(workloads.BASE_SEED + seed)
    return rng.uniform(-scale, scale, size=n)


@pytest.mark.parametrize("n_hist,live", [(50, 50), (64, 20)])
def test_finger_reduces_to_simple_shear(n_hist, live):
    """For unidirectional flow (kappa = [[0, s], [0, 0]], nilpotent) the full
    tensor gives the simple-shear reduction: sigma_xy = int s G,
    sigma_xx = int 2 s gamma G, sigma_yy = 0."""
    s = _shear_history(live, 61)
    k = np.zeros((live, 2, 2))
    k[:, 0, 1] = s
    r = np.abs(s)
    G, tau, gc = 1e-3, 30.0, 0.05
    sxx, sxy, syy = oracle.finger_sum(n_hist, k, G, tau, gc)
    # reduced path: strain gamma_k = sum of s over ages 1..k
    dg = np.concatenate([[0.0], np.cumsum(s[1:])])
    want_xy, want_xx = oracle.history_sum(n_hist, s, r, dg, G, tau, gc, n_live=live)
    assert abs(sxy - want_xy) <= 1e-15 * abs(want_xy) + 1e-22
    assert abs(sxx - want_xx) <= 1e-13 * abs(want_xx) + 1e-24
    assert abs(syy) <= 1e-24


@pytest.mark.parametrize("eps", [3e-4, -2e-3])
def test_finger_planar_extension_closed_form(eps):
    """Constant planar extension kappa = diag(eps, -eps): E_k = diag(e^{eps k},
    e^{-eps k}), so sigma_xx = G sum_k w_k 2 eps e^{2 eps k} D_k and
    sigma_yy = -G sum_k w_k 2 eps e^{-2 eps k} D_k with the damping
    D_k = e^{-k (1/tau + 2|eps|/gamma_c)} -- geometric sums in closed form
    (trapezoid weights 1/2 at both ends of the window)."""
    n_hist, G, tau, gc = 80, 1e-3, 25.0, 0.1
    k = np.tile(np.diag([eps, -eps]), (n_hist, 1, 1))
    sxx, sxy, syy = oracle.finger_sum(n_hist, k, G, tau, gc)
    lam = 1 / tau + 2 * abs(eps) / gc
    n = n_hist - 1

    def trap(x):  # sum_{k=0}^{n} w_k x^k
        return (1 - x ** (n + 1)) / (1 - x) - 0.5 - 0.5 * x ** n

    want_xx = G * 2 * eps * trap(math.exp(2 * eps - lam))
    want_yy = -G * 2 * eps * trap(math.exp(-2 * eps - lam))
    assert abs(sxx / want_xx - 1) <= 1e-13
    assert abs(syy / want_yy - 1) <= 1e-13
    assert abs(sxy) <= 1e-22


def test_finger_rigid_rotation_is_stress_free():
    """kappa = [[0, w], [-w, 0]] is a rigid rotation: E is a rotation that
    commutes with kappa, E kappa E^T = kappa is antisymmetric, and the
    stress vanishes (frame indifference)."""
    w = 3e-3
    k = np.tile(np.array([[0.0, w], [-w, 0.0]]), (60, 1, 1))
    out = oracle.finger_sum(60, k, 1e-3, 40.0, 0.1)
    assert max(abs(v) for v in out) <= 1e-20


def test_finger_rotates_with_the_frame():
    """Rotating every velocity gradient by a fixed Q rotates the stress:
    sigma' = Q sigma Q^T (|gamma_dot| is invariant)."""
    rng = np.random.default_rng(workloads.BASE_SEED + 62)
    k = rng.uniform(-2e-3, 2e-3, size=(70, 2, 2))
    th = 0.7
    Q = np.array([[math.cos(th), -math.sin(th)], [math.sin(th), math.cos(th)]])
    kq = np.einsum("ab,kbc,dc->kad", Q, k, Q)
    a = oracle.finger_sum(70, k, 1e-3, 30.0, 0.08)
    b = oracle.finger_sum(70, kq, 1e-3, 30.0, 0.08)
    S = np.array([[a[0], a[1]], [a[1], a[2]]])
    Sq = Q @ S @ Q.T
    np.testing.assert_allclose([b[0], b[1], b[2]], [Sq[0, 0], Sq[0, 1], Sq[1, 1]],
                               rtol=0, atol=1e-13 * np.abs(S).max())


def test_finger_channel_equals_reduced_channel_in_unidirectional_flow():
    """A unidirectional channel gives the same run with the full tensor and
    with the simple-shear reduction (sigma_yy stays zero)."""
    ch = workloads.plain_f64().channels[0].replace(lx=1, ly=12, n_hist=120, tau_m=30.0,
                                                   gx=5e-5)
    wl = workloads.Workload("u", [ch], "f64", steps_on=300, steps_off=100, sample_every=50)
    a = oracle.run_workload(wl)[0]
    b = oracle.run_workload(workloads.Workload("u", [ch.replace(finger=True)], "f64",
                                               steps_on=300, steps_off=100,
                                               sample_every=50))[0]
    # the reduced path takes strains as differences of the growing prefix
    # Gamma, the full tensor as products: N1 (second order in the strain)
    # differs by the prefix's cancellation, ~1e-12
    for key, tol in (("ux", 1e-13), ("sxy", 1e-13), ("n1", 1e-11)):
        assert np.abs(a[key] - b[key]).max() <= tol * np.abs(a[key]).max(), key


def test_finger_product_order_rotation_after_shear():
    """Order of the factors in Eq. eeval (newest on the left): shear for the
    older ages, then a rigid rotation for the K - 1 newest.  The rotation
    adds no stress of its own and turns the shear's stress with it:
    sigma = R sigma_shear R^T, R = exp(kappa_rot (K - 1)), where sigma_shear
    is the same history with zero gradient in place of the rotation.  The
    reversed product order would instead rotate the shear rate before it
    is deformed."""
    K, H, w = 15, 90, 0.02
    s = _shear_history(H, 63, scale=3e-3) + 4e-3
    hist = np.zeros((H, 2, 2))
    hist[K:, 0, 1] = s[K:]
    rot = hist.copy()
    rot[1:K] = np.array([[0.0, w], [-w, 0.0]])
    G, tau, gc = 1e-3, 40.0, 0.1
    a = oracle.finger_sum(H, hist, G, tau, gc)
    b = oracle.finger_sum(H, rot, G, tau, gc)
    R = oracle.expm2(np.array([[0.0, w], [-w, 0.0]]) * (K - 1))
    S = np.array([[a[0], a[1]], [a[1], a[2]]])
    want = R @ S @ R.T
    got = np.array([[b[0], b[1]], [b[1], b[2]]])
    assert np.abs(got - want).max() <= 1e-13 * np.abs(S).max()
    assert np.abs(got - S).max() > 1e-3 * np.abs(S).max()   # the rotation matters


# --------------------------------------------------------------------------
# The paper's own stress coupling (Eq. bodyforce with d_t delta rho)
# --------------------------------------------------------------------------

@pytest.mark.parametrize("seed", range(4))
def test_paper_forcing_moments(seed):
    """Moments of Eq. bodyforce on D2Q9 (4th-order isotropy of the weights):
    sum F = (1 - 1/2tau) dr, sum c F = (1 - 1/2tau) f,
    sum c c F = -sbar/tau + (1 - 1/2tau) (cs2 dr I - dr u u + u f + f u)."""
    rng = np.random.default_rng(workloads.BASE_SEED + 70 + seed)
    tau = rng.uniform(0.6, 2.0)
    u, f = rng.uniform(-0.05, 0.05, 2), rng.uniform(-1e-4, 1e-4, 2)
    a, b = rng.uniform(-1e-3, 1e-3, 2)
    sbar = np.array([a, b, -a])
    dr = rng.uniform(-1e-5, 1e-5)
    F = oracle.force_term_paper(tau, u[0], u[1], f[0], f[1], sbar, dr)
    cx, cy, _, _ = oracle.lattice()
    c = np.stack([cx, cy], 1).astype(float)
    pre = 1 - 1 / (2 * tau)
    S = np.array([[a, b], [b, -a]])
    A = -dr * np.outer(u, u) + np.outer(u, f) + np.outer(f, u)
    assert abs(F.sum() - pre * dr) < 1e-18
    np.testing.assert_allclose(c.T @ F, pre * f, rtol=0, atol=1e-18)
    want2 = -S / tau + pre * (dr / 3 * np.eye(2) + A)
    np.testing.assert_allclose(np.einsum("i,ia,ib->ab", F, c, c), want2, rtol=0, atol=1e-17)


def test_paper_coupling_newtonian_equals_body_force():
    """Without stress (G = 0) both couplings are the same scheme."""
    ch = workloads.large_2d(lx=6, ly=10, n_hist=16).channels[0].replace(g_inf=0.0, gx=2e-5)
    wl = lambda c: workloads.Workload("n", [c], "f64", steps_on=200, sample_every=50)
    a = oracle.run_workload(wl(ch))[0]
    b = oracle.run_workload(wl(ch.replace(paper_coupling=True)))[0]
    for key in ("ux", "uy", "rho"):
        np.testing.assert_allclose(b[key], a[key], rtol=0, atol=1e-15 * np.abs(a[key]).max())


@pytest.mark.parametrize("finger", [False, True])
def test_paper_coupling_mass_and_pressure(finger):
    """Every node gains d_t delta rho of mass per step, so the total mass
    plus 1.5 sum tr sigma^{t-2} (the density carrying the non-Newtonian
    pressure -tr sigma / 2 = cs2 delta rho) is conserved exactly."""
    ch = workloads.large_2d(lx=8, ly=12, n_hist=64).channels[0]
    ch = ch.replace(u0=ch.u0 * 50.0, tau_m=30.0, paper_coupling=True, finger=finger)
    oc = oracle.OracleChannel(ch)
    m0 = oc.mass()
    oc.step(300)
    tr = oc.trace_prev()
    assert np.abs(tr).max() > 1e-8          # the trace is not trivially zero
    assert abs(oc.mass() + 1.5 * tr.sum() - m0) / m0 < 1e-13


def test_paper_coupling_ucm_steady_centreline():
    """With the paper's coupling the UCM channel reaches the same steady
    state as with the body force: centreline g ly^2 / (8 nu_eff) at second
    order in 1/ly (nu_eff = nu + the discrete Maxwell viscosity)."""
    errs = []
    for ly in (12, 24):
        g, tau, Gm = 1e-6, 15.0, 5e-3
        ch = workloads.Channel(lx=1, ly=ly, tau_lb=1.0, g_inf=Gm, tau_m=tau,
                               gamma_c=math.inf, n_hist=600, gx=g, paper_coupling=True)
        oc = oracle.OracleChannel(ch)
        nu = 0.5 / 3
        eta_s = Gm * 0.5 / math.tanh(0.5 / tau) * (1 - math.exp(-599 / tau))
        nu_eff = nu + eta_s
        t_wall = ly * ly / (math.pi ** 2 * nu_eff)
        oc.step(int(25 * t_wall) + 1000)
        _, ux, _ = oc.fields()
        uc = 0.5 * (ux[ly // 2, 0] + ux[ly // 2 - 1, 0])
        y = ly / 2 - 0.5
        want = g / (2 * nu_eff) * (y + 0.5) * (ly - 0.5 - y)
        errs.append(abs(uc / want - 1))
    assert errs[0] < 0.05
    assert errs[1] < errs[0] / 3


# --------------------------------------------------------------------------
# Alternative laws: accumulated-strain damping (Sec. II) and the
# instantaneous law (Eq. inlM)
# --------------------------------------------------------------------------

def test_strain_damping_equals_nlm_for_constant_shear():
    """Under constant shear the accumulated strain from t' to t is (t - t')|s|,
    exactly the rate term of Eq. nlmax: both laws give the same sums."""
    H, t = 300, 180
    for s in (2e-4, -7e-4):
        s_age = np.where(np.arange(H) <= t, s, 0.0)
        r_age = np.abs(s_age)
        dg = np.concatenate([[0.0], np.cumsum(s_age[1:])])
        a = oracle.history_sum(H, s_age, r_age, dg, 1e-3, 40.0, 0.05)
        b = oracle.history_sum_wm(H, s_age, r_age, dg, 1e-3, 40.0, 0.05)
        np.testing.assert_allclose(b, a, rtol=1e-13)


def test_strain_damping_one_step_recursion():
    """The damping factorises over time, so the shear stress obeys the
    one-step update A(t+1) = s_{t+1}/2 + l_t (A(t) + s_t/2) with
    l_t = exp(-1/tau - r_t/gamma_c) while nothing leaves the window
    (trapezoid weight 1/2 at age 0, 1 beyond)."""
    rng = np.random.default_rng(workloads.BASE_SEED + 80)
    T, H, tau, gc, G = 150, 400, 30.0, 0.02, 1.0
    s = rng.uniform(-1e-3, 1e-3, T)
    r = np.abs(s) * rng.uniform(0.5, 1.5, T)       # |gamma_dot| from the full II_D
    A = []
    for t in range(T):
        s_age = s[t::-1]
        r_age = r[t::-1]
        A.append(oracle.history_sum_wm(H, s_age, r_age, np.zeros(t + 1), G, tau, gc,
                                       n_live=t + 1)[0])
    for t in range(T - 1):
        lam = math.exp(-1 / tau - r[t] / gc)
        want = 0.5 * s[t + 1] + lam * (A[t] + 0.5 * s[t])
        assert abs(A[t + 1] - want) <= 1e-13 * max(abs(want), 1e-3)


def test_strain_damping_differs_from_nlm_for_varying_shear():
    rng = np.random.default_rng(workloads.BASE_SEED + 81)
    H = 200
    s_age = rng.uniform(-1e-3, 1e-3, H)
    r_age = np.abs(s_age)
    dg = np.concatenate([[0.0], np.cumsum(s_age[1:])])
    a = oracle.history_sum(H, s_age, r_age, dg, 1e-3, 40.0, 0.01)
    b = oracle.history_sum_wm(H, s_age, r_age, dg, 1e-3, 40.0, 0.01)
    assert abs(a[0] - b[0]) > 1e-3 * abs(a[0])


def test_instantaneous_law_is_the_steady_limit_of_the_history_sum():
    """Long-time constant shear: the integral model tends to the
    instantaneous law within its trapezoid factors 1 + O(lam^2)."""
    n_hist = 20000
    for s in (1e-5, 3e-4, 2e-3):
        s_age = np.full(n_hist, s)
        a = oracle.history_sum_ages(s_age, np.abs(s_age), G, TAU, GC)
        b = oracle.instantaneous(s, abs(s), G, TAU, GC)
        lam = 1.0 / TAU + s / GC
        assert abs(a[0] / b[0] - 1) < lam ** 2 / 11
        assert abs(a[1] / b[1] - 1) < lam ** 2 / 11


def test_instantaneous_channel_reaches_the_integral_steady_state():
    """Fig. steadystate's claim: the instantaneous and the integral model
    reach the same steady channel flow (up to the O(lam^2) quadrature factor
    of the integral model and its truncated window)."""
    base = workloads.Channel(lx=1, ly=14, tau_lb=1.0, g_inf=4e-3, tau_m=12.0, gamma_c=0.05,
                             n_hist=500, gx=2e-5)
    outs = []
    for law in ("nlm", "instantaneous"):
        oc = oracle.OracleChannel(base.replace(law=law))
        oc.step(6000)
        outs.append(oc.fields()[1][:, 0])
        sxy, _ = oc.stress()
    a, b = outs
    assert np.abs(a).max() > 1e-4
    # quadrature factor 1 + lam^2/12 at the largest rate lam = 1/tau + |s|/gamma_c
    s_max = np.abs(np.diff(a)).max() * 1.5
    lam = 1 / base.tau_m + s_max / base.gamma_c
    assert np.abs(a - b).max() <= lam ** 2 / 12 * np.abs(a).max()
