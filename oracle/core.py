"""ctypes front end of the C oracle (cbdg_oracle.c).  Test infrastructure only.

The shared object is built from the single C file with gcc; ``ensure_built``
compiles it when it is missing or older than its source.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from typing import Optional, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "cbdg_oracle.c")
_LIB = os.path.join(_HERE, "libcbdg_oracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (plain IEEE FP64: no fast-math)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared",
                               _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def ensure_built():
    global _lib
    if _lib is None:
        build(force=False)
        lib = C.CDLL(_LIB)
        i64p = C.POINTER(C.c_int64)
        i32p = C.POINTER(C.c_int32)
        dp = C.POINTER(C.c_double)
        lib.ora_csr_nnz_bound.restype = C.c_int64
        lib.ora_csr_nnz_bound.argtypes = [C.c_int, C.c_int]
        lib.ora_build_csr.restype = C.c_int64
        lib.ora_build_csr.argtypes = [C.c_int, C.c_int, C.c_int, C.c_int, C.c_double, C.c_double,
                                      dp, dp, dp, dp, C.c_double, C.c_double, i64p, i32p, dp]
        lib.ora_moments.restype = C.c_int
        lib.ora_moments.argtypes = [C.c_int64, i64p, i32p, dp, C.c_int, i32p, C.c_int64,
                                    C.c_int, dp, dp, C.c_int]
        lib.ora_moments_backward.restype = C.c_int
        lib.ora_moments_backward.argtypes = [C.c_int64, i64p, i32p, dp, i32p, C.c_int64, C.c_int,
                                             C.c_double, dp, dp, dp, dp, C.c_int]
        lib.ora_max_threads.restype = C.c_int
        _lib = lib
    return _lib


def _p(arr, ct):
    return arr.ctypes.data_as(C.POINTER(ct)) if arr is not None else None


def max_threads() -> int:
    return int(ensure_built().ora_max_threads())


class CSR:
    """Explicit sparse matrix in the interleaved Nambu basis r = 2*s + alpha."""

    def __init__(self, rowptr, col, val, D, a, b):
        self.rowptr, self.col, self.val = rowptr, col, val
        self.D, self.a, self.b = D, a, b

    @property
    def is_real(self) -> bool:
        return bool(np.all(self.val.imag == 0.0))

    def to_scipy(self):
        import scipy.sparse as sp
        return sp.csr_matrix((self.val, self.col, self.rowptr), shape=(self.D, self.D))


def build_csr(Lx, Ly, bc_x, bc_y, t, mu_c, eps, delta, delta_bond=None, peierls=None,
              a=1.0, b=0.0) -> CSR:
    """(H - b)/a of eq. (hamil2) as an explicit CSR (a=1, b=0 gives H itself)."""
    lib = ensure_built()
    L2 = Lx * Ly
    eps = np.ascontiguousarray(eps, dtype=np.float64)
    dl = np.ascontiguousarray(np.asarray(delta, dtype=np.complex128).reshape(L2))
    db = None if delta_bond is None else np.ascontiguousarray(
        np.asarray(delta_bond, dtype=np.complex128).reshape(2, L2))
    ph = None if peierls is None else np.ascontiguousarray(
        np.asarray(peierls, dtype=np.float64).reshape(2, L2))
    nb = lib.ora_csr_nnz_bound(Lx, Ly)
    rowptr = np.zeros(2 * L2 + 1, dtype=np.int64)
    col = np.zeros(nb, dtype=np.int32)
    val = np.zeros(nb, dtype=np.complex128)
    nnz = lib.ora_build_csr(Lx, Ly, bc_x, bc_y, t, mu_c, _p(eps, C.c_double),
                            dl.view(np.float64).ctypes.data_as(C.POINTER(C.c_double)),
                            None if db is None else db.view(np.float64).ctypes.data_as(C.POINTER(C.c_double)),
                            _p(ph, C.c_double), float(a), float(b),
                            _p(rowptr, C.c_int64), _p(col, C.c_int32),
                            val.view(np.float64).ctypes.data_as(C.POINTER(C.c_double)))
    if nnz < 0:
        raise ValueError("oracle: bad lattice arguments")
    return CSR(rowptr, col[:nnz].copy(), val[:nnz].copy(), 2 * L2, float(a), float(b))


def bounds(Lx, Ly, bc_x, bc_y, t, mu_c, eps, delta, delta_bond=None, peierls=None,
           delta_cap=0.0, eta=0.01) -> Tuple[float, float, float, float]:
    """Spectral bounds and rescaling of the paragraph after eq. (rec).

    Reading: the paper asks only for approximate E_min, E_max ("not essential to
    have accurate bounds").  The oracle takes the Gershgorin disc bound of the
    unscaled H -- the largest absolute row sum -- with every |Delta_i| raised to
    at least delta_cap so the bound holds for every iterate of the gap map.
    Particle-hole symmetry makes the bound symmetric: E_max = -E_min = R, b = 0,
    a = (E_max - E_min)/(2 - eta).  Returns (E_min, E_max, a, b).
    """
    dl = np.asarray(delta, dtype=np.complex128).reshape(-1)
    mag = np.maximum(np.abs(dl), delta_cap)
    capped = np.where(np.abs(dl) > 0, dl / np.where(np.abs(dl) > 0, np.abs(dl), 1.0), 1.0) * mag
    H = build_csr(Lx, Ly, bc_x, bc_y, t, mu_c, eps, capped, delta_bond, peierls, 1.0, 0.0)
    rows = np.add.reduceat(np.abs(H.val), H.rowptr[:-1]) if H.val.size else np.zeros(H.D)
    R = float(np.max(rows))
    e_min, e_max = -R, R
    a = (e_max - e_min) / (2.0 - eta)
    b = 0.5 * (e_max + e_min)
    return e_min, e_max, a, b


def workload_csr(w, a: float, b: float, delta=None) -> CSR:
    return build_csr(w.Lx, w.Ly, w.bc_x, w.bc_y, w.t, w.mu_c, w.eps,
                     w.delta if delta is None else delta, w.delta_bond, w.peierls, a, b)


def workload_bounds(w, delta=None):
    return bounds(w.Lx, w.Ly, w.bc_x, w.bc_y, w.t, w.mu_c, w.eps,
                  w.delta if delta is None else delta, w.delta_bond, w.peierls,
                  delta_cap=w.delta_cap, eta=w.eta)


def moments(H: CSR, sites, N: int, n_threads: int = 0, force_complex: Optional[bool] = None):
    """mu_ee[k, n] = <s,e|T_n(Ht)|s,e>, mu_he[k, n] = <s,h|T_n(Ht)|s,e>, s = sites[k].

    Eq. (ref2) with the moments of eqs. (coeff1)/(coeff2) taken without the
    1/(1 + delta_{0n}) factor.  mu_ee is real (a diagonal element of a
    Hermitian matrix function); mu_he is complex, real for a real operator.
    """
    lib = ensure_built()
    sites = np.ascontiguousarray(sites, dtype=np.int32)
    n = sites.size
    is_complex = (not H.is_real) if force_complex is None else bool(force_complex)
    mu_ee = np.zeros((n, N), dtype=np.float64)
    mu_he = np.zeros((n, N), dtype=np.complex128)
    rc = lib.ora_moments(H.D, _p(H.rowptr, C.c_int64), _p(H.col, C.c_int32),
                         H.val.view(np.float64).ctypes.data_as(C.POINTER(C.c_double)),
                         int(is_complex), _p(sites, C.c_int32), n, int(N),
                         _p(mu_ee, C.c_double),
                         mu_he.view(np.float64).ctypes.data_as(C.POINTER(C.c_double)),
                         int(n_threads))
    if rc != 0:
        raise ValueError("oracle: moments failed (bad sites, N, or complex values on the real path)")
    if not is_complex:
        return mu_ee, mu_he.real.copy()
    return mu_ee, mu_he


def workload_moments(w, a, b, sites=None, N=None, delta=None, n_threads=0):
    H = workload_csr(w, a, b, delta)
    return moments(H, w.start_sites if sites is None else sites, w.N if N is None else N,
                   n_threads=n_threads)


def moments_backward(H: CSR, sites, N: int, dmu_ee, dmu_he, n_threads: int = 0):
    """Gradient of L = sum(dmu_ee*mu_ee + dmu_he*mu_he) w.r.t. eps_j and a real
    Delta_j, for a real operator with (a, b) held fixed.  Returns
    (grad_eps, grad_delta), each of length L2."""
    lib = ensure_built()
    if not H.is_real:
        raise ValueError("oracle: the backward pass is defined for a real operator")
    sites = np.ascontiguousarray(sites, dtype=np.int32)
    n = sites.size
    dmu_ee = np.ascontiguousarray(np.broadcast_to(dmu_ee, (n, N)), dtype=np.float64)
    dmu_he = np.ascontiguousarray(np.broadcast_to(dmu_he, (n, N)), dtype=np.float64)
    L2 = H.D // 2
    ge = np.zeros(L2)
    gd = np.zeros(L2)
    rc = lib.ora_moments_backward(H.D, _p(H.rowptr, C.c_int64), _p(H.col, C.c_int32),
                                  H.val.view(np.float64).ctypes.data_as(C.POINTER(C.c_double)),
                                  _p(sites, C.c_int32), n, int(N), float(H.a),
                                  _p(dmu_ee, C.c_double), _p(dmu_he, C.c_double),
                                  _p(ge, C.c_double), _p(gd, C.c_double), int(n_threads))
    if rc != 0:
        raise ValueError("oracle: backward failed")
    return ge, gd
