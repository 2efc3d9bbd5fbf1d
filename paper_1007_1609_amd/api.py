"""Torch-facing helpers over the C ABI.

PyTorch supplies device memory and the current HIP stream; every number is
computed by libcbdg.so.  Inputs must already be contiguous device tensors of
the documented dtype (float64, complex128 for complex Delta, int32 sites);
nothing is converted silently.
"""
from __future__ import annotations

import ctypes as C
from dataclasses import dataclass
from typing import Optional, Tuple

import torch

from . import _lib as L


def _stream() -> int:
    return torch.cuda.current_stream().cuda_stream


def _ptr(t: Optional[torch.Tensor], dtype=None, name="tensor"):
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("%s must be a device tensor" % name)
    if not t.is_contiguous():
        raise ValueError("%s must be contiguous" % name)
    if dtype is not None and t.dtype != dtype:
        raise ValueError("%s must have dtype %s, got %s" % (name, dtype, t.dtype))
    return t.data_ptr()


def _need(t: Optional[torch.Tensor], numel: int, name: str) -> None:
    """Caller-supplied arrays must hold at least what the call writes or reads."""
    if t is not None and t.numel() < numel:
        raise ValueError("%s has %d elements, the call needs %d" % (name, t.numel(), numel))


def weights(a: float, b: float, kernel: str = "jackson", lam: float = 0.0, T: float = 0.0,
            E_c: float = 0.0) -> L.cbdg_weights:
    k = {"jackson": L.CBDG_KERNEL_JACKSON, "lorentz": L.CBDG_KERNEL_LORENTZ}[kernel]
    return L.cbdg_weights(k, float(lam), float(T), float(E_c), float(a), float(b))


@dataclass
class Bounds:
    E_min: float
    E_max: float
    a: float
    b: float


class Operator:
    """Handle of a rescaled BdG operator (cbdg_build_bdg / cbdg_op_destroy)."""

    def __init__(self, Lx, Ly, t, mu_c, eps, delta, delta_bond=None, peierls=None, *,
                 bc_x=0, bc_y=0, complex_=False, fixed: Optional[Tuple[float, float]] = None,
                 delta_cap=0.0, eta=0.01):
        L.load()
        self.Lx, self.Ly = int(Lx), int(Ly)
        self.bc_x, self.bc_y = int(bc_x), int(bc_y)
        self.scalar = L.CBDG_COMPLEX if complex_ else L.CBDG_REAL
        ddt = torch.complex128 if complex_ else torch.float64
        lat = L.cbdg_lattice(self.Lx, self.Ly, int(bc_x), int(bc_y), self.scalar)
        fb = None
        if fixed is not None:
            a, b = fixed
            fb = L.cbdg_bounds(b - a, b + a, float(a), float(b))
        out = L.cbdg_bounds()
        h = C.c_void_p()
        L.cbdg_build_bdg(C.byref(lat), float(t), float(mu_c), _ptr(eps, torch.float64, "eps"),
                         _ptr(delta, ddt, "delta"), _ptr(delta_bond, ddt, "delta_bond"),
                         _ptr(peierls, torch.float64, "peierls"),
                         C.byref(fb) if fb is not None else None, float(delta_cap), float(eta),
                         _stream(), C.byref(h), C.byref(out))
        self._handle = h
        self.bounds = Bounds(out.E_min, out.E_max, out.a, out.b)
        self.has_bond = delta_bond is not None
        self._alive = True

    @classmethod
    def from_workload(cls, w, device="cuda", delta=None, fixed=None):
        cplx = w.scalar == "complex"
        ddt = torch.complex128 if cplx else torch.float64
        eps = torch.as_tensor(w.eps, dtype=torch.float64, device=device).contiguous()
        dl = torch.as_tensor(w.delta if delta is None else delta, dtype=ddt, device=device).contiguous()
        db = None if w.delta_bond is None else torch.as_tensor(
            w.delta_bond.reshape(-1) if cplx else w.delta_bond.real.reshape(-1), dtype=ddt,
            device=device).contiguous()
        ph = None if w.peierls is None else torch.as_tensor(
            w.peierls.reshape(-1), dtype=torch.float64, device=device).contiguous()
        return cls(w.Lx, w.Ly, w.t, w.mu_c, eps, dl, db, ph, bc_x=w.bc_x, bc_y=w.bc_y,
                   complex_=cplx, fixed=fixed, delta_cap=w.delta_cap, eta=w.eta)

    @property
    def handle(self):
        """The library handle; a closed operator raises instead of handing out
        the released pointer."""
        if not getattr(self, "_alive", False):
            raise ValueError("operator has been closed")
        return self._handle

    @property
    def L2(self):
        return self.Lx * self.Ly

    @property
    def is_complex(self):
        return self.scalar == L.CBDG_COMPLEX

    def update_delta(self, delta: torch.Tensor, delta_bond: Optional[torch.Tensor] = None):
        h = self.handle
        ddt = torch.complex128 if self.is_complex else torch.float64
        L.cbdg_op_update_delta(h, _ptr(delta, ddt, "delta"),
                               _ptr(delta_bond, ddt, "delta_bond"), _stream())

    def weights(self, kernel="jackson", lam=0.0, E_c=0.0, T=0.0):
        return weights(self.bounds.a, self.bounds.b, kernel, lam, T, E_c)

    def close(self):
        if getattr(self, "_alive", False):
            h, self._handle, self._alive = self._handle, None, False
            L.cbdg_op_destroy(h)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def moments_workspace_bytes(op: Operator, tile: int, precision: int = L.CBDG_FP64,
                            algorithm: int = L.CBDG_ALG_AUTO) -> int:
    n = C.c_size_t()
    L.cbdg_moments_workspace_size(op.handle, int(tile), int(precision), int(algorithm), C.byref(n))
    return n.value


def workspace(nbytes: int, device="cuda") -> torch.Tensor:
    return torch.empty(max(int(nbytes), 1), dtype=torch.uint8, device=device)


def chebyshev_moments(op: Operator, sites: torch.Tensor, N: int, tile: int,
                      precision: int = L.CBDG_FP64, ws: Optional[torch.Tensor] = None,
                      out: Optional[Tuple[torch.Tensor, torch.Tensor]] = None,
                      algorithm: int = L.CBDG_ALG_AUTO):
    """mu_ee [n, N] float64 and mu_he [n, N] (float64 or complex128)."""
    n = int(sites.numel())
    eff = max(1, min(int(tile), n))
    need = moments_workspace_bytes(op, eff, precision, algorithm)
    if ws is None or ws.numel() < need:
        ws = workspace(need, sites.device)
    if out is None:
        mu_ee = torch.empty((n, N), dtype=torch.float64, device=sites.device)
        mu_he = torch.empty((n, N), dtype=torch.complex128 if op.is_complex else torch.float64,
                            device=sites.device)
    else:
        mu_ee, mu_he = out
        _need(mu_ee, n * int(N), "mu_ee")
        _need(mu_he, n * int(N), "mu_he")
    L.cbdg_chebyshev_moments(op.handle, _ptr(sites, torch.int32, "sites"), n, int(N), int(tile),
                             int(precision), int(algorithm), _ptr(ws, None, "workspace"), ws.numel(),
                             _ptr(mu_ee, torch.float64, "mu_ee"),
                             _ptr(mu_he, torch.complex128 if op.is_complex else torch.float64, "mu_he"),
                             _stream())
    return mu_ee, mu_he


def resident_workspace_bytes(op: Operator, tile: int, precision: int = L.CBDG_FP64) -> int:
    n = C.c_size_t()
    L.cbdg_resident_workspace_size(op.handle, int(tile), int(precision), C.byref(n))
    return n.value


def chebyshev_moments_resident(op: Operator, sites: torch.Tensor, N: int, tile: int,
                               precision: int = L.CBDG_FP64, ws: Optional[torch.Tensor] = None,
                               out: Optional[Tuple[torch.Tensor, torch.Tensor]] = None,
                               spin_limit: int = 0):
    """Moments by doubling with every recursion step of a tile in one
    persistent launch (tiles of at most 256 vectors whose buffers fit the
    Infinity Cache); mu_ee, mu_he [n, N] float64."""
    n = int(sites.numel())
    eff = max(1, min(int(tile), n))
    need = resident_workspace_bytes(op, eff, precision)
    if ws is None or ws.numel() < need:
        ws = workspace(need, sites.device)
    if out is None:
        mu_ee = torch.empty((n, N), dtype=torch.float64, device=sites.device)
        mu_he = torch.empty((n, N), dtype=torch.float64, device=sites.device)
    else:
        mu_ee, mu_he = out
        _need(mu_ee, n * int(N), "mu_ee")
        _need(mu_he, n * int(N), "mu_he")
    L.cbdg_chebyshev_moments_resident(op.handle, _ptr(sites, torch.int32, "sites"), n, int(N), int(tile),
                                      int(precision), int(spin_limit), _ptr(ws, None, "workspace"), ws.numel(),
                                      _ptr(mu_ee, torch.float64, "mu_ee"), _ptr(mu_he, torch.float64, "mu_he"),
                                      _stream())
    return mu_ee, mu_he


def chebyshev_moments_nb(op: Operator, sites: torch.Tensor, N: int, tile: int,
                         precision: int = L.CBDG_FP64, ws: Optional[torch.Tensor] = None):
    """Direct moments plus the neighbour moments nb_ee, nb_he [n, 4, N]
    (neighbours +x, -x, +y, -y; complex128 for complex operators)."""
    n = int(sites.numel())
    eff = max(1, min(int(tile), n))
    need = moments_workspace_bytes(op, eff, precision, L.CBDG_ALG_DIRECT)
    if ws is None or ws.numel() < need:
        ws = workspace(need, sites.device)
    cdt = torch.complex128 if op.is_complex else torch.float64
    mu_ee = torch.empty((n, N), dtype=torch.float64, device=sites.device)
    mu_he = torch.empty((n, N), dtype=cdt, device=sites.device)
    nb_ee = torch.empty((n, 4, N), dtype=cdt, device=sites.device)
    nb_he = torch.empty((n, 4, N), dtype=cdt, device=sites.device)
    L.cbdg_chebyshev_moments_nb(op.handle, _ptr(sites, torch.int32, "sites"), n, int(N), int(tile), int(precision),
                                _ptr(ws, None, "workspace"), ws.numel(), _ptr(mu_ee, torch.float64, "mu_ee"),
                                _ptr(mu_he, None, "mu_he"), _ptr(nb_ee, None, "nb_ee"), _ptr(nb_he, None, "nb_he"),
                                _stream())
    return mu_ee, mu_he, nb_ee, nb_he


def bond_gap_update(nb_he: torch.Tensor, op: Operator, w: L.cbdg_weights, U: float,
                    delta_bond_in: torch.Tensor, alpha: float = 1.0,
                    delta_bond_out: Optional[torch.Tensor] = None, resid: Optional[torch.Tensor] = None,
                    coeff: Optional[torch.Tensor] = None):
    """Symmetrised bond order parameter [2 * L2] from the neighbour moments of
    every site of op's lattice (rows in site order)."""
    N = nb_he.shape[-1]
    coeff = _coeff_for(w, N, L.CBDG_QTY_GAP, coeff, nb_he.device)
    _need(nb_he, op.L2 * 4 * N, "nb_he")
    _need(delta_bond_in, 2 * op.L2, "delta_bond_in")
    _need(delta_bond_out, 2 * op.L2, "delta_bond_out")
    _need(coeff, N, "coeff")
    if delta_bond_out is None:
        delta_bond_out = torch.empty_like(delta_bond_in)
    if resid is None:
        resid = torch.empty(1, dtype=torch.float64, device=nb_he.device)
    ddt = torch.complex128 if op.is_complex else torch.float64
    L.cbdg_bond_gap_update(_ptr(nb_he, ddt, "nb_he"), op.Lx, op.Ly, op.bc_x, op.bc_y, int(N), op.scalar, C.byref(w),
                           _ptr(coeff, torch.float64, "coeff"), float(U), _ptr(delta_bond_in, ddt, "delta_bond_in"),
                           float(alpha), _ptr(delta_bond_out, ddt, "delta_bond_out"),
                           _ptr(resid, torch.float64, "resid"), _stream())
    return delta_bond_out, resid


def bond_current(op: Operator, nb_ee: torch.Tensor, w: L.cbdg_weights,
                 coeff: Optional[torch.Tensor] = None) -> torch.Tensor:
    """Particle current [2, L2] along the +x and +y bond of every site."""
    N = nb_ee.shape[-1]
    _need(nb_ee, op.L2 * 4 * N, "nb_ee")
    if coeff is None:
        coeff = sum_coefficients(w, N, L.CBDG_QTY_DENSITY, nb_ee.device)
    _need(coeff, N, "coeff")
    out = torch.empty((2, op.L2), dtype=torch.float64, device=nb_ee.device)
    ddt = torch.complex128 if op.is_complex else torch.float64
    L.cbdg_bond_current(op.handle, _ptr(nb_ee, ddt, "nb_ee"), int(N), C.byref(w), _ptr(coeff, torch.float64, "coeff"),
                        _ptr(out, torch.float64, "current"), _stream())
    return out


def check_moments(mu_ee: torch.Tensor, mu_he: torch.Tensor, tol: float = 1e-9) -> bool:
    """True when every moment is finite with |mu| <= 1 + tol (synchronises)."""
    flag = torch.empty(1, dtype=torch.int32, device=mu_ee.device)
    n, N = mu_ee.shape
    L.cbdg_check_moments(_ptr(mu_ee, torch.float64, "mu_ee"), _ptr(mu_he, None, "mu_he"), n, N,
                         L.CBDG_COMPLEX if mu_he.is_complex() else L.CBDG_REAL, float(tol),
                         _ptr(flag), _stream())
    return int(flag.item()) == 0


def sum_coefficients(w: L.cbdg_weights, N: int, quantity: int = L.CBDG_QTY_GAP,
                     device="cuda") -> torch.Tensor:
    """Damped Chebyshev coefficients g_n c_n of the gap (tanh(E/2T) on
    |E| < E_c) or density (f(E)) weight at the weights' temperature."""
    out = torch.empty(int(N), dtype=torch.float64, device=device)
    L.cbdg_sum_coefficients(C.byref(w), int(N), int(quantity), _ptr(out, torch.float64, "coeff"), _stream())
    return out


def _coeff_for(w, N, quantity, coeff, device):
    if coeff is None and w.T > 0.0:
        coeff = sum_coefficients(w, N, quantity, device)
    return coeff


def gap_update(mu_he: torch.Tensor, w: L.cbdg_weights, U: float, delta_in: torch.Tensor,
               alpha: float = 1.0, U_rows: Optional[torch.Tensor] = None,
               delta_out: Optional[torch.Tensor] = None, resid: Optional[torch.Tensor] = None,
               coeff: Optional[torch.Tensor] = None):
    """coeff: g_n c_n of the gap weight (computed here when T > 0 and not given)."""
    n, N = mu_he.shape
    cplx = mu_he.is_complex()
    coeff = _coeff_for(w, N, L.CBDG_QTY_GAP, coeff, mu_he.device)
    for t, name in ((delta_in, "delta_in"), (delta_out, "delta_out"), (U_rows, "U_rows")):
        _need(t, n, name)
    _need(coeff, N, "coeff")
    if delta_out is None:
        delta_out = torch.empty_like(delta_in)
    if resid is None:
        resid = torch.empty(1, dtype=torch.float64, device=mu_he.device)
    ddt = torch.complex128 if cplx else torch.float64
    L.cbdg_gap_update(_ptr(mu_he, ddt, "mu_he"), n, N, L.CBDG_COMPLEX if cplx else L.CBDG_REAL,
                      C.byref(w), _ptr(coeff, torch.float64, "coeff"), float(U),
                      _ptr(U_rows, torch.float64, "U_rows"),
                      _ptr(delta_in, ddt, "delta_in"), float(alpha), _ptr(delta_out, ddt, "delta_out"),
                      _ptr(resid, torch.float64, "resid"), _stream())
    return delta_out, resid


def ldos(mu_ee: torch.Tensor, w: L.cbdg_weights, energies: torch.Tensor,
         out: Optional[torch.Tensor] = None):
    n, N = mu_ee.shape
    nE = int(energies.numel())
    _need(out, n * nE, "ldos out")
    if out is None:
        out = torch.empty((n, nE), dtype=torch.float64, device=mu_ee.device)
    L.cbdg_ldos(_ptr(mu_ee, torch.float64, "mu_ee"), n, N, C.byref(w),
                _ptr(energies, torch.float64, "energies"), nE, _ptr(out, torch.float64, "ldos"),
                _stream())
    return out


def gap_update_backward(d_delta_out: torch.Tensor, N: int, w: L.cbdg_weights, U: float,
                        alpha: float = 1.0, U_rows: Optional[torch.Tensor] = None,
                        want_delta_in: bool = True, coeff: Optional[torch.Tensor] = None):
    n = int(d_delta_out.numel())
    d_mu = torch.empty((n, N), dtype=torch.float64, device=d_delta_out.device)
    d_in = torch.empty_like(d_delta_out) if want_delta_in else None
    coeff = _coeff_for(w, N, L.CBDG_QTY_GAP, coeff, d_delta_out.device)
    _need(U_rows, n, "U_rows")
    _need(coeff, N, "coeff")
    L.cbdg_gap_update_backward(_ptr(d_delta_out, torch.float64, "d_delta_out"), n, int(N), C.byref(w),
                               _ptr(coeff, torch.float64, "coeff"), float(U), _ptr(U_rows, torch.float64, "U_rows"), float(alpha),
                               _ptr(d_mu, torch.float64, "d_mu_he"), _ptr(d_in, torch.float64, "d_delta_in"),
                               _stream())
    return d_mu, d_in


def density(mu_ee: torch.Tensor, w: L.cbdg_weights, coeff: Optional[torch.Tensor] = None,
            out: Optional[torch.Tensor] = None) -> torch.Tensor:
    """Electron density per site, 2 sum_n g_n c_n mu_ee_n (f(E) weight)."""
    n, N = mu_ee.shape
    coeff = _coeff_for(w, N, L.CBDG_QTY_DENSITY, coeff, mu_ee.device)
    _need(coeff, N, "coeff")
    _need(out, n, "density out")
    if out is None:
        out = torch.empty(n, dtype=torch.float64, device=mu_ee.device)
    L.cbdg_density(_ptr(mu_ee, torch.float64, "mu_ee"), n, N, C.byref(w), _ptr(coeff, torch.float64, "coeff"),
                   _ptr(out, torch.float64, "density"), _stream())
    return out


def density_backward(d_density: torch.Tensor, N: int, w: L.cbdg_weights,
                     coeff: Optional[torch.Tensor] = None) -> torch.Tensor:
    n = int(d_density.numel())
    coeff = _coeff_for(w, N, L.CBDG_QTY_DENSITY, coeff, d_density.device)
    _need(coeff, N, "coeff")
    d_mu = torch.empty((n, N), dtype=torch.float64, device=d_density.device)
    L.cbdg_density_backward(_ptr(d_density, torch.float64, "d_density"), n, int(N), C.byref(w),
                            _ptr(coeff, torch.float64, "coeff"), _ptr(d_mu, torch.float64, "d_mu_ee"), _stream())
    return d_mu


def ldos_backward(d_ldos: torch.Tensor, N: int, w: L.cbdg_weights, energies: torch.Tensor):
    n, nE = d_ldos.shape
    _need(energies, nE, "energies")
    d_mu = torch.empty((n, N), dtype=torch.float64, device=d_ldos.device)
    L.cbdg_ldos_backward(_ptr(d_ldos, torch.float64, "d_ldos"), n, int(N), C.byref(w),
                         _ptr(energies, torch.float64, "energies"), nE, _ptr(d_mu, torch.float64, "d_mu_ee"),
                         _stream())
    return d_mu


def backward_workspace_bytes(op: Operator, tile: int, N: int, ckpt_stride: int = 0,
                             algorithm: int = L.CBDG_ALG_AUTO) -> int:
    n = C.c_size_t()
    L.cbdg_backward_workspace_size(op.handle, int(tile), int(N), int(ckpt_stride), int(algorithm), C.byref(n))
    return n.value


# ckpt_stride of the reverse passes that regenerate the forward vectors
# backwards instead of storing checkpoints (doubling, real operators with
# uniform hopping, Lx = 64 W)
REVERSIBLE = -1


def reversible_supported(op: Operator, tile: int, N: int) -> bool:
    """Whether the checkpoint-free reverse passes apply to this operator."""
    try:
        backward_workspace_bytes(op, max(1, int(tile)), N, REVERSIBLE, L.CBDG_ALG_DOUBLING)
        return True
    except L.CbdgError:
        return False


def chebyshev_moments_jacobian(op: Operator, sites: torch.Tensor, N: int, tile: int,
                               dmu_ee: Optional[torch.Tensor], dmu_he: Optional[torch.Tensor],
                               jac_eps: Optional[torch.Tensor] = None, jac_delta: Optional[torch.Tensor] = None,
                               want_eps: bool = False, ws: Optional[torch.Tensor] = None):
    """Per-start-vector rows of the moments' reverse-mode derivative
    (cbdg_chebyshev_moments_jacobian): row k of the returned [n_start, L2]
    matrices is the gradient of sum_n dmu[k][n] mu[k][n] with respect to eps
    and Delta.  jac_eps is filled only when given or want_eps."""
    n = int(sites.numel())
    eff = max(1, min(int(tile), n))
    need = backward_workspace_bytes(op, eff, N, REVERSIBLE, L.CBDG_ALG_DOUBLING)
    if ws is None or ws.numel() < need:
        ws = workspace(need, sites.device)
    _need(dmu_ee, n * int(N), "dmu_ee")
    _need(dmu_he, n * int(N), "dmu_he")
    _need(jac_eps, n * op.L2, "jac_eps")
    _need(jac_delta, n * op.L2, "jac_delta")
    if jac_delta is None:
        jac_delta = torch.empty((n, op.L2), dtype=torch.float64, device=sites.device)
    if jac_eps is None and want_eps:
        jac_eps = torch.empty((n, op.L2), dtype=torch.float64, device=sites.device)
    L.cbdg_chebyshev_moments_jacobian(op.handle, _ptr(sites, torch.int32, "sites"), n, int(N), int(tile),
                                      _ptr(dmu_ee, torch.float64, "dmu_ee"),
                                      _ptr(dmu_he, torch.float64, "dmu_he"),
                                      _ptr(ws, None, "workspace"), ws.numel(),
                                      _ptr(jac_eps, torch.float64, "jac_eps"),
                                      _ptr(jac_delta, torch.float64, "jac_delta"), op.L2, _stream())
    return jac_eps, jac_delta


def jacobian_matvec(A: torch.Tensor, x: torch.Tensor, out: Optional[torch.Tensor] = None) -> torch.Tensor:
    """y = A x for a dense row-major FP64 matrix on the device
    (cbdg_jacobian_matvec; fixed summation order)."""
    if A.dim() != 2 or not A.is_contiguous():
        raise ValueError("A must be a contiguous 2-D tensor")
    rows, cols = A.shape
    _need(x, cols, "x")
    if out is None:
        out = torch.empty(rows, dtype=torch.float64, device=A.device)
    _need(out, rows, "out")
    L.cbdg_jacobian_matvec(_ptr(A, torch.float64, "A"), rows, cols, cols, _ptr(x, torch.float64, "x"),
                           _ptr(out, torch.float64, "out"), _stream())
    return out


def chebyshev_moments_backward(op: Operator, sites: torch.Tensor, N: int, tile: int,
                               dmu_ee: Optional[torch.Tensor], dmu_he: Optional[torch.Tensor],
                               ckpt_stride: int = 0, grad_eps: Optional[torch.Tensor] = None,
                               grad_delta: Optional[torch.Tensor] = None,
                               ws: Optional[torch.Tensor] = None, algorithm: int = L.CBDG_ALG_AUTO):
    n = int(sites.numel())
    eff = max(1, min(int(tile), n))
    need = backward_workspace_bytes(op, eff, N, ckpt_stride, algorithm)
    if ws is None or ws.numel() < need:
        ws = workspace(need, sites.device)
    _need(dmu_ee, n * int(N), "dmu_ee")
    _need(dmu_he, n * int(N), "dmu_he")
    _need(grad_eps, op.L2, "grad_eps")
    _need(grad_delta, op.L2, "grad_delta")
    if grad_eps is None:
        grad_eps = torch.zeros(op.L2, dtype=torch.float64, device=sites.device)
    if grad_delta is None:
        grad_delta = torch.zeros(op.L2, dtype=torch.float64, device=sites.device)
    L.cbdg_chebyshev_moments_backward(op.handle, _ptr(sites, torch.int32, "sites"), n, int(N),
                                      int(tile), int(ckpt_stride), int(algorithm),
                                      _ptr(dmu_ee, torch.float64, "dmu_ee"),
                                      _ptr(dmu_he, torch.float64, "dmu_he"),
                                      _ptr(ws, None, "workspace"), ws.numel(),
                                      _ptr(grad_eps, torch.float64, "grad_eps"),
                                      _ptr(grad_delta, torch.float64, "grad_delta"), _stream())
    return grad_eps, grad_delta
