"""Self-consistency loop on the device (the paper's iteration: compute every
grid point's Green's function with the current order parameter, update the
order parameter in the Hamiltonian, repeat -- the paragraph after the current
density).

The loop body is three library calls -- cbdg_chebyshev_moments over all
sites, cbdg_gap_update (gap equation, mixing, residual) and
cbdg_op_update_delta -- and one scalar copied to the host per iteration to
test convergence.  The spectral bounds (a, b) stay frozen at the values the
operator was built with.
"""
from __future__ import annotations

import time
from dataclasses import dataclass, field
from typing import List, Optional

import torch

from . import _lib as L
from .api import Operator, chebyshev_moments, gap_update, moments_workspace_bytes, workspace


@dataclass
class ScfResult:
    delta: torch.Tensor
    iterations: int
    residual: float
    history: List[float] = field(default_factory=list)
    seconds: float = 0.0
    moment_passes: int = 0


def plain_mixing(op: Operator, U: float, delta0: torch.Tensor, N: int, tile: int,
                 precision: int = L.CBDG_FP64, alpha: float = 1.0, tol: float = 1e-6,
                 max_iter: int = 200, kernel: str = "jackson", E_c: float = 0.0,
                 sites: Optional[torch.Tensor] = None, callback=None) -> ScfResult:
    """Delta <- (1 - alpha) Delta + alpha F(Delta) until max|F(Delta) - Delta| < tol."""
    dev = delta0.device
    if sites is None:
        sites = torch.arange(op.L2, dtype=torch.int32, device=dev)
    w = op.weights(kernel, E_c=E_c)
    ws = workspace(moments_workspace_bytes(op, min(tile, sites.numel()), precision), dev)
    n = sites.numel()
    mu_ee = torch.empty((n, N), dtype=torch.float64, device=dev)
    mu_he = torch.empty((n, N), dtype=delta0.dtype, device=dev)
    delta = delta0.clone()
    nxt = torch.empty_like(delta)
    resid = torch.empty(1, dtype=torch.float64, device=dev)
    hist: List[float] = []
    t0 = time.perf_counter()
    op.update_delta(delta)
    r = float("inf")
    it = 0
    for it in range(1, max_iter + 1):
        chebyshev_moments(op, sites, N, tile, precision, ws=ws, out=(mu_ee, mu_he))
        gap_update(mu_he, w, U, delta, alpha, delta_out=nxt, resid=resid)
        r = float(resid.item())
        hist.append(r)
        delta, nxt = nxt, delta
        op.update_delta(delta)
        if callback is not None:
            callback(it, r)
        if not (r == r):
            raise L.CbdgError(L.CBDG_EBOUNDS, "scf", "non-finite residual at iteration %d" % it)
        if r < tol:
            break
    torch.cuda.synchronize()
    return ScfResult(delta, it, r, hist, time.perf_counter() - t0, it)
