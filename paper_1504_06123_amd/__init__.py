"""MI355X-native hybrid lattice-Boltzmann engine with the integral nonlinear
Maxwell constitutive equation (Papenkort & Voigtmann, arXiv:1504.06123).

The computation lives in liblbmax.so (HIP kernels for gfx950 behind the C
interface in include/lbmax.h); this package is its Python binding.
"""
from ._lib import LBError, load  # noqa: F401
from .solver import (MachWarning, Solver, make_descs, pack_state_header,  # noqa: F401
                     state_layout, workspace_bytes)

__all__ = ["Solver", "LBError", "MachWarning", "load", "make_descs", "pack_state_header",
           "state_layout", "workspace_bytes"]
