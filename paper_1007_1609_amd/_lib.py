"""ctypes mirror of include/cbdg.h: same function names, same argument order.

Argument marshalling only.  Loading fails loudly when libcbdg.so has not been
built: there is no other implementation behind these names.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libcbdg.so")

CBDG_OK = 0
CBDG_EINVAL = -1
CBDG_ENOMEM = -2
CBDG_EHIP = -3
CBDG_EBOUNDS = -4
CBDG_EUNSUPPORTED = -5

CBDG_BC_OPEN, CBDG_BC_PERIODIC = 0, 1
CBDG_REAL, CBDG_COMPLEX = 0, 1
CBDG_FP64, CBDG_FP32_ACC64 = 0, 1
CBDG_KERNEL_JACKSON, CBDG_KERNEL_LORENTZ = 0, 1
CBDG_ALG_AUTO, CBDG_ALG_DIRECT, CBDG_ALG_DOUBLING = 0, 1, 2
CBDG_QTY_GAP, CBDG_QTY_DENSITY = 0, 1

_NAMES = {CBDG_EINVAL: "EINVAL", CBDG_ENOMEM: "ENOMEM", CBDG_EHIP: "EHIP",
          CBDG_EBOUNDS: "EBOUNDS", CBDG_EUNSUPPORTED: "EUNSUPPORTED"}


class cbdg_lattice(C.Structure):
    _fields_ = [("Lx", C.c_int32), ("Ly", C.c_int32), ("bc_x", C.c_int32),
                ("bc_y", C.c_int32), ("scalar", C.c_int32)]


class cbdg_bounds(C.Structure):
    _fields_ = [("E_min", C.c_double), ("E_max", C.c_double), ("a", C.c_double), ("b", C.c_double)]


class cbdg_weights(C.Structure):
    _fields_ = [("kernel", C.c_int32), ("lambda_", C.c_double), ("T", C.c_double),
                ("E_c", C.c_double), ("a", C.c_double), ("b", C.c_double)]


class CbdgError(RuntimeError):
    def __init__(self, code: int, where: str, message: str):
        super().__init__("%s: %s (%s)" % (where, message, _NAMES.get(code, str(code))))
        self.code = code


_vp = C.c_void_p
_i32, _i64, _f64, _sz = C.c_int32, C.c_int64, C.c_double, C.c_size_t

# (name, argtypes) exactly as declared in include/cbdg.h
SIGNATURES = {
    "cbdg_build_bdg": [C.POINTER(cbdg_lattice), _f64, _f64, _vp, _vp, _vp, _vp,
                       C.POINTER(cbdg_bounds), _f64, _f64, _vp, C.POINTER(_vp),
                       C.POINTER(cbdg_bounds)],
    "cbdg_op_update_delta": [_vp, _vp, _vp, _vp],
    "cbdg_op_destroy": [_vp],
    "cbdg_op_bounds": [_vp, C.POINTER(cbdg_bounds)],
    "cbdg_moments_workspace_size": [_vp, _i32, _i32, _i32, C.POINTER(_sz)],
    "cbdg_chebyshev_moments": [_vp, _vp, _i64, _i32, _i32, _i32, _i32, _vp, _sz, _vp, _vp, _vp],
    "cbdg_resident_workspace_size": [_vp, _i32, _i32, C.POINTER(_sz)],
    "cbdg_chebyshev_moments_resident": [_vp, _vp, _i64, _i32, _i32, _i32, _i64, _vp, _sz, _vp, _vp, _vp],
    "cbdg_chebyshev_moments_static": [_vp, _vp, _i64, _i32, _i32, _i32, _i32, _vp, _vp, _vp],
    "cbdg_chebyshev_moments_nb": [_vp, _vp, _i64, _i32, _i32, _i32, _vp, _sz, _vp, _vp, _vp, _vp, _vp],
    "cbdg_check_moments": [_vp, _vp, _i64, _i32, _i32, _f64, _vp, _vp],
    "cbdg_bond_gap_update": [_vp, _i32, _i32, _i32, _i32, _i32, _i32, C.POINTER(cbdg_weights), _vp, _f64,
                             _vp, _f64, _vp, _vp, _vp],
    "cbdg_bond_current": [_vp, _vp, _i32, C.POINTER(cbdg_weights), _vp, _vp, _vp],
    "cbdg_sum_coefficients": [C.POINTER(cbdg_weights), _i32, _i32, _vp, _vp],
    "cbdg_gap_update": [_vp, _i64, _i32, _i32, C.POINTER(cbdg_weights), _vp, _f64, _vp, _vp,
                        _f64, _vp, _vp, _vp],
    "cbdg_density": [_vp, _i64, _i32, C.POINTER(cbdg_weights), _vp, _vp, _vp],
    "cbdg_density_backward": [_vp, _i64, _i32, C.POINTER(cbdg_weights), _vp, _vp, _vp],
    "cbdg_ldos": [_vp, _i64, _i32, C.POINTER(cbdg_weights), _vp, _i32, _vp, _vp],
    "cbdg_gap_update_backward": [_vp, _i64, _i32, C.POINTER(cbdg_weights), _vp, _f64, _vp, _f64,
                                 _vp, _vp, _vp],
    "cbdg_ldos_backward": [_vp, _i64, _i32, C.POINTER(cbdg_weights), _vp, _i32, _vp, _vp],
    "cbdg_backward_workspace_size": [_vp, _i32, _i32, _i32, _i32, C.POINTER(_sz)],
    "cbdg_chebyshev_moments_backward": [_vp, _vp, _i64, _i32, _i32, _i32, _i32, _vp, _vp, _vp, _sz,
                                        _vp, _vp, _vp],
    "cbdg_chebyshev_moments_jacobian": [_vp, _vp, _i64, _i32, _i32, _vp, _vp, _vp, _sz, _vp, _vp, _i64, _vp],
    "cbdg_jacobian_matvec": [_vp, _i64, _i64, _i64, _vp, _vp, _vp],
}

_lib = None


def load():
    """Load libcbdg.so and declare every entry point; raises if it is absent."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(
            "libcbdg.so is not built (expected at %s); run `python paper_1007_1609_amd/build.py` "
            "or __graft_entry__.build()" % LIB_PATH)
    lib = C.CDLL(LIB_PATH)
    for name, argtypes in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.argtypes = argtypes
        fn.restype = C.c_int
    lib.cbdg_last_error.argtypes = []
    lib.cbdg_last_error.restype = C.c_char_p
    lib.cbdg_static_scratch_bytes.argtypes = []
    lib.cbdg_static_scratch_bytes.restype = C.c_size_t
    _lib = lib
    return lib


def check(rc: int, where: str):
    if rc != CBDG_OK:
        msg = load().cbdg_last_error().decode(errors="replace")
        raise CbdgError(rc, where, msg)


def _call(name):
    def f(*args):
        lib = load()
        rc = getattr(lib, name)(*args)
        check(rc, name)
        return rc
    f.__name__ = name
    return f


# Python entry points with the C names (raise CbdgError on a non-zero status).
cbdg_build_bdg = _call("cbdg_build_bdg")
cbdg_op_update_delta = _call("cbdg_op_update_delta")
cbdg_op_destroy = _call("cbdg_op_destroy")
cbdg_op_bounds = _call("cbdg_op_bounds")
cbdg_moments_workspace_size = _call("cbdg_moments_workspace_size")
cbdg_chebyshev_moments = _call("cbdg_chebyshev_moments")
cbdg_chebyshev_moments_static = _call("cbdg_chebyshev_moments_static")
cbdg_resident_workspace_size = _call("cbdg_resident_workspace_size")
cbdg_chebyshev_moments_resident = _call("cbdg_chebyshev_moments_resident")
cbdg_check_moments = _call("cbdg_check_moments")
cbdg_sum_coefficients = _call("cbdg_sum_coefficients")
cbdg_density = _call("cbdg_density")
cbdg_density_backward = _call("cbdg_density_backward")
cbdg_chebyshev_moments_nb = _call("cbdg_chebyshev_moments_nb")
cbdg_bond_gap_update = _call("cbdg_bond_gap_update")
cbdg_bond_current = _call("cbdg_bond_current")
cbdg_gap_update = _call("cbdg_gap_update")
cbdg_ldos = _call("cbdg_ldos")
cbdg_gap_update_backward = _call("cbdg_gap_update_backward")
cbdg_ldos_backward = _call("cbdg_ldos_backward")
cbdg_backward_workspace_size = _call("cbdg_backward_workspace_size")
cbdg_chebyshev_moments_backward = _call("cbdg_chebyshev_moments_backward")
cbdg_chebyshev_moments_jacobian = _call("cbdg_chebyshev_moments_jacobian")
cbdg_jacobian_matvec = _call("cbdg_jacobian_matvec")


def cbdg_last_error() -> str:
    return load().cbdg_last_error().decode(errors="replace")


def cbdg_static_scratch_bytes() -> int:
    return int(load().cbdg_static_scratch_bytes())
