"""CPU checks of the test helpers the GPU studies rely on: the UCM channel
flow's modal solution (tests/closed_forms.py) against facts it must reproduce
on its own, and the input recipes of the Sec. IV and appendix channels
(workloads.py) against the dimensionless numbers they are built from."""
import math

import numpy as np
import pytest

import workloads
from closed_forms import channel_node_positions, maxwell_channel_startup


@pytest.mark.parametrize("g_inf,tau", [(0.0, 1.0), (1e-3, 50.0), (2e-2, 400.0)])
def test_modal_solution_reaches_the_poiseuille_profile(g_inf, tau):
    """Long after startup the flow is the parabola g (H^2 - y^2) / (2 eta)
    with the total viscosity eta = eta_s + G tau (Sec. I: eta = G tau)."""
    half, eta_s, g = 8.0, 0.1, 1e-6
    y = np.linspace(-half, half, 33)
    u = maxwell_channel_startup(y, [1e9], half, 1.0, eta_s, g_inf, tau, g)[0]
    want = g * (half * half - y * y) / (2.0 * (eta_s + g_inf * tau))
    assert np.abs(u - want).max() <= 1e-9 * want.max()


def test_modal_solution_starts_from_rest_and_accelerates_with_the_force():
    """At t = 0 the fluid is at rest; away from the walls it first
    accelerates freely, u = g t, before momentum diffusion reaches it."""
    half, eta_s, g = 16.0, 0.05, 1e-6
    y = np.array([0.0, 4.0])
    u0, u1 = maxwell_channel_startup(y, [0.0, 5.0], half, 1.0, eta_s, 0.0, 1.0, g)
    assert np.abs(u0).max() <= 1e-12 * g
    assert np.abs(u1 - g * 5.0).max() <= 1e-6 * g * 5.0


def test_modal_solution_oscillates_for_an_elastic_fluid():
    """Small retardation, large relaxation time (the appendix's regime):
    the centre velocity overshoots its steady value; with the same total
    viscosity and no elasticity (Newtonian) it does not."""
    half, g = 32.0, 1e-6
    t = np.linspace(0, 20000, 401)
    elastic = maxwell_channel_startup([0.0], t, half, 1.0, 0.01, 1e-2, 1000.0, g)[:, 0]
    viscous = maxwell_channel_startup([0.0], t, half, 1.0, 10.01, 0.0, 1.0, g)[:, 0]
    steady = g * half * half / (2 * 10.01)
    assert elastic.max() > 2.0 * steady
    assert viscous.max() <= steady * (1 + 1e-9)


def test_node_positions_put_the_halfway_walls_at_plus_minus_h():
    y = channel_node_positions(32)
    assert y[0] == -15.5 and y[-1] == 15.5 and abs(y.mean()) < 1e-15


@pytest.mark.parametrize("ratio", [0.1, 1.0, 8.0])
@pytest.mark.parametrize("model", workloads.SEC4_MODELS)
def test_sec4_channels_carry_their_dimensionless_numbers(ratio, model):
    ch = workloads.sec4_channel(ratio, 10.0, model)
    eta = (ch.tau_lb - 0.5) / 3.0
    half = ch.ly / 2
    nlm = workloads.sec4_channel(ratio, 10.0, "nlm")
    tau0 = eta / nlm.g_inf
    assert ch.lx == 1 and ch.ly == 2 * workloads.SEC4_HALF_WIDTH and ch.tau_lb == 0.9
    assert math.isclose(workloads.sec4_wall_time() / tau0, ratio, rel_tol=1e-12)
    assert math.isclose(4 * half * half / (math.pi ** 2 * eta), workloads.sec4_wall_time())
    assert math.isclose(nlm.tau_m, 10.0 * tau0, rel_tol=1e-12)
    assert math.isclose(ch.gx, nlm.g_inf / (2 * half), rel_tol=1e-12)
    if model == "nlm":
        assert ch.n_hist == math.ceil(6 * ch.tau_m) and ch.gamma_c == 0.1
        # the plug of the steady flow: |sigma_xy| = g |y| below G gamma_c
        assert math.isclose(ch.g_inf * ch.gamma_c / ch.gx / half, 2 * ch.gamma_c)
    elif model == "ucm":
        assert math.isinf(ch.gamma_c) and ch.n_hist == math.ceil(10 * ch.tau_m)
    elif model == "instantaneous":
        assert ch.law == "instantaneous"
    else:
        assert ch.g_inf == 0.0


@pytest.mark.parametrize("width,theta,s2", [(128, 400.0, 0.05), (512, 2000.0, 0.01)])
def test_appendix_channels_carry_their_dimensionless_numbers(width, theta, s2):
    ch = workloads.appendix_ucm_channel(width, theta, s2)
    eta = (ch.tau_lb - 0.5) / 3.0
    tau0 = eta / ch.g_inf
    eta_max = ch.g_inf * (ch.tau_m + tau0)
    assert math.isclose(ch.tau_m / tau0, theta, rel_tol=1e-12)
    assert math.isclose(eta_max * tau0 / width ** 2, s2, rel_tol=1e-12)
    assert math.isclose(eta_max * ch.tau_m / width ** 2, s2 * theta, rel_tol=1e-12)
    assert math.isclose(ch.gx * (width / 2) ** 2 / (2 * eta_max), 1e-5, rel_tol=1e-12)
    assert math.isinf(ch.gamma_c) and ch.n_hist == math.ceil(10 * ch.tau_m)
