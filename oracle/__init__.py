"""Plain, slow, obviously correct CPU oracle of the Chebyshev-BdG hot path.

TEST INFRASTRUCTURE.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import or call anything here.  The
product library never does, and this package never imports the product
package: the two share no code.  Inputs come from the seeded generators in
``workloads``, which hold none of the method's arithmetic.

Parts (each function cites the passage of the paper it follows):
  core.py   explicit sparse Hamiltonian of eq. (hamil2), the vector recursion
            of eq. (ref2) and its adjoint, in plain C (cbdg_oracle.c)
  kpm.py    kernel factors, energy weights (T = 0 closed forms, finite-T
            quadrature), the gap equation eq. (op1), the LDOS eq. (ldos) and
            the electron density, in NumPy FP64
  scf.py    the self-consistency loop (plain mixing)
  offdiag.py  moments between a start site and its neighbours, the bond order
            parameter and the bond current

Readings of passages the paper leaves open are listed with the code that
uses them.
"""
from .core import (build_csr, bounds, moments, moments_backward, workload_csr, workload_bounds,
                   workload_moments, max_threads, ensure_built)
from .kpm import (jackson, lorentz, sign_coefficients, sign_weight_coefficients, gap_weights, gap_map,
                  ldos, ldos_weights, chebyshev_T, thermal_coefficients, thermal_gap_weights, density, gap_map_thermal)
from .scf import scf_plain
from .offdiag import neighbour_site, neighbour_moments, bond_gap_map, bond_current

__all__ = [
    "build_csr", "bounds", "moments", "moments_backward", "workload_csr", "workload_bounds",
    "workload_moments", "max_threads", "ensure_built", "jackson", "lorentz",
    "sign_coefficients", "sign_weight_coefficients", "gap_weights", "gap_map", "ldos", "ldos_weights",
    "chebyshev_T", "scf_plain", "thermal_coefficients", "thermal_gap_weights", "density", "gap_map_thermal",
    "neighbour_site", "neighbour_moments", "bond_gap_map", "bond_current",
]
