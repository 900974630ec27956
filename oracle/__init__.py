"""FP64 CPU oracle of the hybrid lattice-Boltzmann / integral nonlinear Maxwell
scheme (arXiv:1504.06123).

TEST INFRASTRUCTURE ONLY: imported by the test suite, the smoke check and the
benchmark's CPU-baseline leg, never by the product package.  It shares no code
with the GPU path; the only common import is the seeded input module
``workloads``.
"""
from .oracle import (  # noqa: F401
    OracleChannel, QGrid, lattice, equilibrium, force_term, collide,
    density_momentum, velocity_gradient, shear_rate, stress_divergence,
    stream, history_sum, history_sum_ages, run_workload, load, expm2, finger_sum,
    force_term_paper, history_sum_wm, instantaneous, LAWS,
)
