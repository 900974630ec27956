"""Closed-form results the tests hold the oracle and the GPU path to.

Test infrastructure only: nothing here imports the oracle or the GPU path.

Startup of pressure-driven channel flow of a Maxwell fluid with a background
viscosity (the UCM of the paper's appendix, Fig. UCM: the problem Waters and
King solved; gamma_c = inf makes Eq. nlmax linear).  Between no-slip walls at
y = -H and y = H (y from the channel centre), with density rho, background
viscosity eta_s, polymer stress sigma_p(t) = int_0^inf G e^{-s/tau} kappa(t - s)
ds, and a force density rho g switched on at t = 0 from rest:

    rho du/dt = d/dy (eta_s du/dy + sigma_p) + rho g.

The modes cos(k_n y), k_n = (2n + 1) pi / (2H), vanish at the walls; the
constant force has the coefficients c_n = 4 (-1)^n / ((2n + 1) pi).  With
u = sum a_n cos(k_n y) and sigma_p = -sum b_n k_n sin(k_n y), each mode obeys

    a_n' = -(k_n^2 / rho) (eta_s a_n + b_n) + g c_n,    b_n' = G a_n - b_n / tau,

a linear system x' = A x + f from x(0) = 0, so x(t) = x_ss - e^{At} x_ss with
x_ss = -A^{-1} f; e^{At} of the 2 x 2 matrix comes from Sylvester's formula
with its two eigenvalues (complex for oscillating modes).  By linearity the
flow after the force is removed at time T is u_on(T + t) - u_on(t).
"""
import math

import numpy as np


def maxwell_channel_startup(y, t, half_width, rho, eta_s, g_inf, tau, g, n_modes=2000):
    """u(y, t) [len(t)][len(y)] of the startup flow above (t in steps, y from
    the centre in lattice units)."""
    n = np.arange(n_modes)
    k = (2 * n + 1) * math.pi / (2.0 * half_width)
    c = 4.0 * (-1.0) ** n / ((2 * n + 1) * math.pi)
    a11 = -k * k * eta_s / rho
    a12 = -k * k / rho
    a21 = np.full_like(k, g_inf)
    a22 = np.full_like(k, -1.0 / tau)
    f1 = g * c
    det = a11 * a22 - a12 * a21
    a_ss = -a22 * f1 / det
    b_ss = a21 * f1 / det
    tr = a11 + a22
    root = np.sqrt((tr * tr - 4.0 * det).astype(complex))
    l1, l2 = (tr + root) / 2.0, (tr - root) / 2.0
    tt = np.asarray(t, dtype=float)[:, None]
    e1, e2 = np.exp(l1 * tt), np.exp(l2 * tt)
    p = (l1 * e2 - l2 * e1) / (l1 - l2)
    q = (e1 - e2) / (l1 - l2)
    a_t = (a_ss - (p * a_ss + q * (a11 * a_ss + a12 * b_ss))).real
    return a_t @ np.cos(np.outer(k, np.asarray(y, dtype=float)))


def channel_node_positions(ly):
    """y of the lattice nodes from the centre (halfway walls at +-ly/2)."""
    return np.arange(ly) - (ly - 1) / 2.0
