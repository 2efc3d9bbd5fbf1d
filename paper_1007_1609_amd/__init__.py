"""Chebyshev-BdG on MI355X: the batched Chebyshev recursion of the rescaled
Nambu BdG operator, local moments, the T = 0 gap equation and the LDOS, with
reverse-mode derivatives (Covaci, Peeters, Berciu, arXiv:1007.1609).

The compute lives in libcbdg.so (HIP for gfx950, C ABI in include/cbdg.h);
this package marshals torch tensors and streams into it and drives the
self-consistency loop.  Importing the package loads the library and raises
ImportError when it has not been built.
"""
from . import _lib
from ._lib import (CbdgError, CBDG_FP64, CBDG_FP32_ACC64, CBDG_REAL, CBDG_COMPLEX,
                   CBDG_BC_OPEN, CBDG_BC_PERIODIC, CBDG_ALG_AUTO, CBDG_ALG_DIRECT,
                   CBDG_ALG_DOUBLING, CBDG_QTY_GAP, CBDG_QTY_DENSITY)

_lib.load()

from .api import (Operator, Bounds, weights, chebyshev_moments, check_moments,  # noqa: E402
                  gap_update, ldos, gap_update_backward, ldos_backward,
                  chebyshev_moments_backward, moments_workspace_bytes,
                  backward_workspace_bytes, workspace, sum_coefficients, density, density_backward,
                  chebyshev_moments_nb, bond_gap_update, bond_current, chebyshev_moments_resident,
                  resident_workspace_bytes, REVERSIBLE, reversible_supported,
                  chebyshev_moments_jacobian, jacobian_matvec)

__all__ = [
    "CbdgError", "CBDG_FP64", "CBDG_FP32_ACC64", "CBDG_REAL", "CBDG_COMPLEX", "CBDG_BC_OPEN",
    "CBDG_BC_PERIODIC", "CBDG_ALG_AUTO", "CBDG_ALG_DIRECT", "CBDG_ALG_DOUBLING", "Operator", "Bounds", "weights", "chebyshev_moments", "check_moments",
    "gap_update", "ldos", "gap_update_backward", "ldos_backward", "chebyshev_moments_backward",
    "moments_workspace_bytes", "backward_workspace_bytes", "workspace", "CBDG_QTY_GAP",
    "CBDG_QTY_DENSITY", "sum_coefficients", "density", "density_backward", "chebyshev_moments_nb",
    "bond_gap_update", "bond_current", "chebyshev_moments_resident", "resident_workspace_bytes",
    "REVERSIBLE", "reversible_supported", "chebyshev_moments_jacobian", "jacobian_matvec",
]
