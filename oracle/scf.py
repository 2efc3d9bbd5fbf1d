"""Self-consistency loop of the oracle (paragraph after the current density:
each grid point's Green's function is computed with the current order
parameter profile, the order parameter is updated in the Hamiltonian, and the
procedure is repeated).  Test infrastructure only.

Readings: plain mixing Delta <- (1 - alpha) Delta + alpha Delta^new with
alpha = 1 by default; stop when max_i |Delta^new_i - Delta_i| < tol; the
spectral bounds (a, b) are computed once from the initial Delta with the cap
U/2 and then held fixed.
"""
from __future__ import annotations

import numpy as np

from .core import workload_bounds, workload_csr, moments
from .kpm import gap_map, gap_map_thermal, thermal_gap_weights


def scf_plain(w, tol=1e-6, alpha=1.0, max_iter=200, n_threads=0, bounds=None, history=None, T=0.0):
    """T > 0: the gap weight tanh(E/2T) of eq. (op1) (coefficients computed once)."""
    if bounds is None:
        _, _, a, b = workload_bounds(w)
    else:
        a, b = bounds
    wts = thermal_gap_weights(w.N, a, b, T) if T > 0 else None
    delta = np.array(w.delta, dtype=np.complex128 if w.scalar == "complex" else np.float64)
    sites = np.arange(w.L2, dtype=np.int32)
    for it in range(1, max_iter + 1):
        H = workload_csr(w, a, b, delta)
        _, mu_he = moments(H, sites, w.N, n_threads=n_threads)
        new = gap_map(mu_he, w.U) if T == 0 else gap_map_thermal(mu_he, w.U, a, b, T, weights=wts)
        if w.scalar != "complex":
            new = new.real
        r = float(np.max(np.abs(new - delta)))
        delta = (1.0 - alpha) * delta + alpha * new
        if history is not None:
            history.append(r)
        if r < tol:
            return delta, it, r, (a, b)
    return delta, max_iter, r, (a, b)
