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
from .api import (Operator, bond_gap_update, chebyshev_moments, chebyshev_moments_nb, gap_update,
                  moments_workspace_bytes, sum_coefficients, workspace)


@dataclass
class ScfResult:
    delta: torch.Tensor
    iterations: int
    residual: float
    history: List[float] = field(default_factory=list)
    seconds: float = 0.0
    moment_passes: int = 0
    fast_passes: int = 0      # passes evaluated in the reduced recursion precision
    warmup_passes: int = 0    # passes with the reduced warm-up moment count


class _PrecisionSchedule:
    """Recursion precision of each gap-map evaluation: `fast` (if given) until
    the residual falls below switch_tol or stops falling (the reduced
    precision's own error floor), `final` afterwards.  Stopping is allowed
    only after an evaluation in `final`."""

    def __init__(self, final: int, fast: Optional[int], switch_tol: Optional[float], tol: float):
        self.final = final
        self.fast = fast if fast is not None and fast != final else None
        self.current = self.fast if self.fast is not None else final
        self.switch_tol = switch_tol if switch_tol is not None else max(0.5 * tol, 1e-7)
        self.tol = tol
        self.fast_evaluations = 0
        self._last = float("inf")

    def workspace_bytes(self, op: Operator, tile: int) -> int:
        precs = [self.final] + ([self.fast] if self.fast is not None else [])
        return max(moments_workspace_bytes(op, tile, p) for p in precs)

    def done(self, r: float) -> bool:
        """Records an evaluation with residual r; True once converged."""
        if self.current != self.final:
            self.fast_evaluations += 1
            if r < self.switch_tol or (r < 1e-4 and r > 0.9 * self._last):
                self.current = self.final
            self._last = r
            return False
        return r < self.tol


def plain_mixing(op: Operator, U: float, delta0: torch.Tensor, N: int, tile: int,
                 precision: int = L.CBDG_FP64, alpha: float = 1.0, tol: float = 1e-6,
                 max_iter: int = 200, kernel: str = "jackson", E_c: float = 0.0,
                 sites: Optional[torch.Tensor] = None, callback=None, T: float = 0.0,
                 fast_precision: Optional[int] = None, switch_tol: Optional[float] = None) -> ScfResult:
    """Delta <- (1 - alpha) Delta + alpha F(Delta) until max|F(Delta) - Delta| < tol
    (temperature T: the gap weight tanh(E/2T), coefficients computed once).
    fast_precision: evaluate F with that recursion precision (CBDG_FP32_ACC64)
    until the residual falls below switch_tol (default max(tol/2, 1e-7)), then
    with `precision`; only an evaluation in `precision` can end the loop."""
    dev = delta0.device
    if sites is None:
        sites = torch.arange(op.L2, dtype=torch.int32, device=dev)
    w = op.weights(kernel, E_c=E_c, T=T)
    coeff = sum_coefficients(w, N, L.CBDG_QTY_GAP, dev) if T > 0 else None
    sched = _PrecisionSchedule(precision, fast_precision, switch_tol, tol)
    ws = workspace(sched.workspace_bytes(op, min(tile, sites.numel())), dev)
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
        chebyshev_moments(op, sites, N, tile, sched.current, ws=ws, out=(mu_ee, mu_he))
        gap_update(mu_he, w, U, delta, alpha, delta_out=nxt, resid=resid, coeff=coeff)
        r = float(resid.item())
        hist.append(r)
        delta, nxt = nxt, delta
        op.update_delta(delta)
        if callback is not None:
            callback(it, r)
        if not (r == r):
            raise L.CbdgError(L.CBDG_EBOUNDS, "scf", "non-finite residual at iteration %d" % it)
        if sched.done(r):
            break
    torch.cuda.synchronize()
    return ScfResult(delta, it, r, hist, time.perf_counter() - t0, it, sched.fast_evaluations)


def bond_plain_mixing(op: Operator, U: float, delta: torch.Tensor, delta_bond0: torch.Tensor, N: int,
                      tile: int, alpha: float = 1.0, tol: float = 1e-6, max_iter: int = 200,
                      kernel: str = "jackson", T: float = 0.0, callback=None) -> ScfResult:
    """Self-consistency of the bond order parameter (on-site Delta held at
    `delta`): neighbour moments of every site, the symmetrised bond gap map
    with mixing, cbdg_op_update_delta with the new bonds, until
    max|Delta_new - Delta| < tol.  The result's delta is the [2 * L2] bond array."""
    dev = delta_bond0.device
    sites = torch.arange(op.L2, dtype=torch.int32, device=dev)
    w = op.weights(kernel, T=T)
    coeff = sum_coefficients(w, N, L.CBDG_QTY_GAP, dev) if T > 0 else None
    ws = workspace(moments_workspace_bytes(op, min(tile, op.L2), L.CBDG_FP64, L.CBDG_ALG_DIRECT), dev)
    db = delta_bond0.clone()
    nxt = torch.empty_like(db)
    resid = torch.empty(1, dtype=torch.float64, device=dev)
    hist: List[float] = []
    t0 = time.perf_counter()
    op.update_delta(delta, db)
    r = float("inf")
    it = 0
    for it in range(1, max_iter + 1):
        _, _, _, nb_he = chebyshev_moments_nb(op, sites, N, tile, ws=ws)
        bond_gap_update(nb_he, op, w, U, db, alpha, delta_bond_out=nxt, resid=resid, coeff=coeff)
        r = float(resid.item())
        hist.append(r)
        db, nxt = nxt, db
        op.update_delta(delta, db)
        if callback is not None:
            callback(it, r)
        if not (r == r):
            raise L.CbdgError(L.CBDG_EBOUNDS, "scf", "non-finite residual at iteration %d" % it)
        if r < tol:
            break
    torch.cuda.synchronize()
    return ScfResult(db, it, r, hist, time.perf_counter() - t0, it)


def _gmres(matvec, rhs, tol, restart=30, maxiter=60):
    """Restarted GMRES (modified Gram-Schmidt Arnoldi, Givens rotations) on
    host FP64 vectors of the size of Delta; matvec runs on the device."""
    import numpy as np
    n = rhs.size
    x = np.zeros(n)
    bnorm = np.linalg.norm(rhs)
    if bnorm == 0.0:
        return x, 0
    used = 0
    r = rhs.copy()
    while used < maxiter:
        beta = np.linalg.norm(r)
        if beta <= tol * bnorm:
            break
        m = min(restart, maxiter - used)
        V = np.zeros((m + 1, n))
        H = np.zeros((m + 1, m))
        cs, sn = np.zeros(m), np.zeros(m)
        g = np.zeros(m + 1)
        g[0] = beta
        V[0] = r / beta
        k_used = 0
        for k in range(m):
            w = matvec(V[k])
            used += 1
            for i in range(k + 1):
                H[i, k] = np.dot(V[i], w)
                w = w - H[i, k] * V[i]
            H[k + 1, k] = np.linalg.norm(w)
            if H[k + 1, k] > 0:
                V[k + 1] = w / H[k + 1, k]
            for i in range(k):
                t = cs[i] * H[i, k] + sn[i] * H[i + 1, k]
                H[i + 1, k] = -sn[i] * H[i, k] + cs[i] * H[i + 1, k]
                H[i, k] = t
            den = np.hypot(H[k, k], H[k + 1, k])
            cs[k], sn[k] = (1.0, 0.0) if den == 0 else (H[k, k] / den, H[k + 1, k] / den)
            H[k, k] = cs[k] * H[k, k] + sn[k] * H[k + 1, k]
            H[k + 1, k] = 0.0
            g[k + 1] = -sn[k] * g[k]
            g[k] = cs[k] * g[k]
            k_used = k + 1
            if abs(g[k + 1]) <= tol * bnorm or H[k, k] == 0:
                break
        y = np.linalg.solve(np.triu(H[:k_used, :k_used]), g[:k_used])
        x = x + V[:k_used].T @ y
        if abs(g[k_used]) <= tol * bnorm:
            break
        r = rhs - matvec(x)
        used += 1
    return x, used


def anderson_mixing(op: Operator, U: float, delta0: torch.Tensor, N: int, tile: int,
                    precision: int = L.CBDG_FP64, depth: int = 5, beta: float = 1.0, tol: float = 1e-6,
                    max_iter: int = 200, kernel: str = "jackson", E_c: float = 0.0, T: float = 0.0,
                    warmup_tol: float = 1e-2, callback=None, fast_precision: Optional[int] = None,
                    switch_tol: Optional[float] = None, warmup_N: int = 0) -> ScfResult:
    """The fixed point Delta = F(Delta) of the plain-mixing loop, accelerated by
    Anderson mixing: with g_k = F(Delta_k) - Delta_k and the differences of the
    last `depth` iterates (dX) and residuals (dG),
        gamma = argmin ||g_k - dG gamma||,
        Delta_{k+1} = Delta_k + beta g_k - (dX + beta dG) gamma.
    The gap map also has the trivial fixed point Delta = 0 (and -Delta), so
    plain-mixing steps come first until max|F - Delta| < warmup_tol, as for
    Newton-Krylov; the history restarts when a step raises the residual.
    One gap-map evaluation per iteration, as plain mixing; the stopping test is
    the same max|F(Delta) - Delta| < tol.  Real order parameters.
    fast_precision / switch_tol: as for plain_mixing; the history is kept
    across the switch (the two evaluations of F differ by far less than tol).
    warmup_N (0 < warmup_N < N): the plain-mixing warm-up steps evaluate the
    gap map with warmup_N moments; the first evaluation below warmup_tol
    switches to N for good (and, as any residual jump, restarts the history)."""
    dev = delta0.device
    sites = torch.arange(op.L2, dtype=torch.int32, device=dev)
    w = op.weights(kernel, E_c=E_c, T=T)
    sched = _PrecisionSchedule(precision, fast_precision, switch_tol, tol)
    ws = workspace(sched.workspace_bytes(op, min(tile, op.L2)), dev)
    Nw = warmup_N if 0 < warmup_N < N else N
    bufs = {}
    for n_mom in {N, Nw}:
        bufs[n_mom] = (torch.empty((op.L2, n_mom), dtype=torch.float64, device=dev),
                       torch.empty((op.L2, n_mom), dtype=delta0.dtype, device=dev),
                       sum_coefficients(w, n_mom, L.CBDG_QTY_GAP, dev) if T > 0 else None)
    n_cur = Nw
    warm = 0
    resid = torch.empty(1, dtype=torch.float64, device=dev)
    hist: List[float] = []
    t0 = time.perf_counter()
    x = delta0.clone()
    xs, gs = [], []
    r = float("inf")
    it = 0
    for it in range(1, max_iter + 1):
        op.update_delta(x)
        mu_ee, mu_he, coeff = bufs[n_cur]
        chebyshev_moments(op, sites, n_cur, tile, sched.current, ws=ws, out=(mu_ee, mu_he))
        fx, _ = gap_update(mu_he, w, U, x, 1.0, resid=resid, coeff=coeff)
        g = fx - x
        r = float(resid.item())
        hist.append(r)
        if callback is not None:
            callback(it, r)
        if not (r == r):
            raise L.CbdgError(L.CBDG_EBOUNDS, "scf", "non-finite residual at iteration %d" % it)
        if n_cur != N:
            # reduced-N warm-up: plain steps only, never the end of the loop
            warm += 1
            sched.fast_evaluations += sched.current != sched.final
            x = fx
            if r < warmup_tol:
                n_cur = N
            continue
        if sched.done(r):
            x = fx
            break
        if r >= max(tol, warmup_tol) or (len(hist) > 1 and r > 2.0 * hist[-2]):
            xs, gs = [], []
            x = fx  # plain step
            continue
        xs.append(x)
        gs.append(g)
        if len(xs) > depth + 1:
            xs.pop(0)
            gs.pop(0)
        if len(xs) == 1:
            x = x + beta * g
            continue
        dX = torch.stack([xs[i + 1] - xs[i] for i in range(len(xs) - 1)], dim=1)
        dG = torch.stack([gs[i + 1] - gs[i] for i in range(len(gs) - 1)], dim=1)
        gamma = torch.linalg.lstsq(dG.cpu(), g.cpu().unsqueeze(1)).solution.to(dev).squeeze(1)
        x = x + beta * g - (dX + beta * dG) @ gamma
    torch.cuda.synchronize()
    return ScfResult(x, it, r, hist, time.perf_counter() - t0, it, sched.fast_evaluations, warm)


def newton_krylov(op: Operator, U: float, delta0: torch.Tensor, N: int, tile: int,
                  tol: float = 1e-6, max_newton: int = 30, jv: str = "vjp", fd_step: float = 1e-7,
                  gmres_tol: float = 1e-2, warmup_tol: float = 1e-2, max_warmup: int = 100,
                  kernel: str = "jackson", callback=None, T: float = 0.0,
                  rebuild_jacobian: bool = True) -> ScfResult:
    """Solve F(Delta) = Delta with inexact Newton steps (J_F - I) d = -(F - Delta).

    The gap map has more than one fixed point (Delta -> -Delta, and the
    trivial Delta = 0), so the solve first runs plain-mixing iterations until
    max|F - Delta| < warmup_tol, which keeps it on the branch plain mixing
    selects, then takes Newton steps with a backtracking line search on
    ||F(Delta) - Delta||_2.

    J_F v is one reverse pass (the gap map's Jacobian is symmetric for a real
    operator with uniform U, so the vector-Jacobian product J_F^T v equals
    J_F v; it takes the checkpoint-free reverse passes where the operator
    allows them), or a forward finite difference (jv="fd"), or, with
    jv="jacobian", a product with the whole Jacobian J_F, built by one
    checkpoint-free reverse sweep whose per-start-vector gradients are its
    rows (cbdg_chebyshev_moments_jacobian; L2 x L2 FP64 on the device) and
    applied by the library's matrix-vector kernel; rebuild_jacobian=False
    keeps the first Newton step's matrix for the later steps (a chord
    iteration).  The residual test is the one of plain mixing:
    max|F(Delta) - Delta| < tol.  counts["F"] is the number of gap-map
    evaluations, counts["J"] the Jacobian products, counts["jacobian"] the
    matrices built.
    """
    import numpy as np
    from .api import (REVERSIBLE, backward_workspace_bytes, chebyshev_moments_backward, chebyshev_moments_jacobian,
                      gap_update_backward, jacobian_matvec, reversible_supported)
    if jv not in ("vjp", "fd", "jacobian"):
        raise ValueError("jv must be 'vjp', 'fd' or 'jacobian'")
    if op.is_complex:
        raise L.CbdgError(L.CBDG_EUNSUPPORTED, "newton_krylov", "real operators only")
    dev = delta0.device
    sites = torch.arange(op.L2, dtype=torch.int32, device=dev)
    w = op.weights(kernel, T=T)
    coeff = sum_coefficients(w, N, L.CBDG_QTY_GAP, dev) if T > 0 else None
    ws = workspace(moments_workspace_bytes(op, min(tile, op.L2), L.CBDG_FP64), dev)
    mu_ee = torch.empty((op.L2, N), dtype=torch.float64, device=dev)
    mu_he = torch.empty((op.L2, N), dtype=torch.float64, device=dev)
    resid = torch.empty(1, dtype=torch.float64, device=dev)
    counts = {"F": 0, "J": 0, "warmup": 0, "newton": 0, "jacobian": 0}
    bw_ws = {}
    jac = {}

    def F(delta_t):
        op.update_delta(delta_t)
        chebyshev_moments(op, sites, N, tile, L.CBDG_FP64, ws=ws, out=(mu_ee, mu_he))
        new, _ = gap_update(mu_he, w, U, delta_t, 1.0, resid=resid, coeff=coeff)
        counts["F"] += 1
        return new

    t0 = time.perf_counter()
    delta = delta0.clone()
    hist: List[float] = []
    Fd = F(delta)
    g = Fd - delta
    r = float(torch.max(torch.abs(g)).item())
    hist.append(r)
    # plain mixing into the basin of the branch it converges to
    while r >= max(tol, warmup_tol) and counts["warmup"] < max_warmup:
        delta = Fd
        Fd = F(delta)
        g = Fd - delta
        r = float(torch.max(torch.abs(g)).item())
        hist.append(r)
        counts["warmup"] += 1
    for _ in range(max_newton):
        if callback is not None:
            callback(len(hist), r)
        if not (r == r):
            raise L.CbdgError(L.CBDG_EBOUNDS, "newton_krylov", "non-finite residual")
        if r < tol:
            break
        counts["newton"] += 1
        op.update_delta(delta)
        if jv != "fd" and "ws" not in bw_ws:
            # the checkpoint-free reverse passes where the operator allows them
            bw_ws["stride"] = REVERSIBLE if reversible_supported(op, min(tile, op.L2), N) else 0
            if jv == "jacobian" and bw_ws["stride"] != REVERSIBLE:
                raise L.CbdgError(L.CBDG_EUNSUPPORTED, "newton_krylov",
                                  "the whole Jacobian needs the checkpoint-free reverse passes")
            bw_ws["ws"] = workspace(backward_workspace_bytes(op, min(tile, op.L2), N, bw_ws["stride"]), dev)
        if jv == "jacobian" and (rebuild_jacobian or "J" not in jac):
            # row k: d F_k / d Delta (the gap update's cotangent of its own moments, one reverse sweep)
            d_mu, _ = gap_update_backward(torch.ones(op.L2, dtype=torch.float64, device=dev), N, w, U, 1.0,
                                          want_delta_in=False, coeff=coeff)
            _, jac["J"] = chebyshev_moments_jacobian(op, sites, N, tile, None, d_mu, jac_delta=jac.get("J"),
                                                     ws=bw_ws["ws"])
            counts["jacobian"] += 1
        Fd_now, delta_now = Fd, delta

        def matvec(v_np):
            v = torch.as_tensor(v_np, dtype=torch.float64, device=dev)
            counts["J"] += 1
            if jv == "fd":
                h = fd_step / max(1e-300, float(np.max(np.abs(v_np))))
                Fp = F(delta_now + h * v)
                counts["F"] -= 1
                jvv = (Fp - Fd_now) / h
            elif jv == "jacobian":
                jvv = jacobian_matvec(jac["J"], v)
            else:
                d_mu, _ = gap_update_backward(v, N, w, U, 1.0, want_delta_in=False, coeff=coeff)
                _, jvv = chebyshev_moments_backward(op, sites, N, tile, None, d_mu, bw_ws["stride"], ws=bw_ws["ws"])
            return (jvv - v).cpu().numpy()

        d_np, _ = _gmres(matvec, -g.cpu().numpy(), gmres_tol)
        d = torch.as_tensor(d_np, dtype=torch.float64, device=dev)
        g2 = float(torch.linalg.norm(g).item())
        lam = 1.0
        while True:
            trial = delta + lam * d
            Ft = F(trial)
            gt = Ft - trial
            if float(torch.linalg.norm(gt).item()) <= (1.0 - 1e-4 * lam) * g2 or lam < 1.0 / 64:
                break
            lam *= 0.5
        delta, Fd, g = trial, Ft, gt
        r = float(torch.max(torch.abs(g)).item())
        hist.append(r)
    torch.cuda.synchronize()
    res = ScfResult(delta, len(hist), r, hist, time.perf_counter() - t0, counts["F"] + counts["J"])
    res.counts = dict(counts)
    return res
