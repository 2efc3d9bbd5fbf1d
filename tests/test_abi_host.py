"""Host-side checks of the C ABI that need no GPU: the library loads, exports
every entry point include/cbdg.h declares with the argument count the
binding uses, and rejects bad arguments on the host before touching HIP."""
import ctypes as C
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "cbdg.h")
LIBSO = os.path.join(ROOT, "paper_1007_1609_amd", "libcbdg.so")


def _ensure_lib():
    if not os.path.exists(LIBSO):
        subprocess.check_call(["python", os.path.join(ROOT, "paper_1007_1609_amd", "build.py")])
    from paper_1007_1609_amd import _lib
    return _lib


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    decls = {}
    for m in re.finditer(r"(?:int|const char \*)\s*(cbdg_\w+)\s*\(([^)]*)\)\s*;", text):
        args = m.group(2).strip()
        n = 0 if args in ("", "void") else args.count(",") + 1
        decls[m.group(1)] = n
    return decls


def test_header_declares_the_boundary_calls():
    d = _declared()
    for name in ("cbdg_build_bdg", "cbdg_op_update_delta", "cbdg_op_destroy", "cbdg_chebyshev_moments",
                 "cbdg_gap_update", "cbdg_ldos", "cbdg_chebyshev_moments_backward",
                 "cbdg_gap_update_backward", "cbdg_ldos_backward", "cbdg_last_error",
                 "cbdg_chebyshev_moments_jacobian", "cbdg_jacobian_matvec"):
        assert name in d, name


def test_library_exports_every_declared_symbol():
    L = _ensure_lib()
    out = subprocess.run(["nm", "-D", "--defined-only", LIBSO], capture_output=True, text=True).stdout
    exported = set(re.findall(r" T (cbdg_\w+)", out))
    for name in _declared():
        assert name in exported, name
    lib = L.load()
    for name in _declared():
        assert hasattr(lib, name)


def test_binding_argument_counts_match_header():
    L = _ensure_lib()
    d = _declared()
    for name, argtypes in L.SIGNATURES.items():
        assert d[name] == len(argtypes), name
    assert set(L.SIGNATURES) | {"cbdg_last_error"} == set(d)


def test_host_validation_without_gpu():
    L = _ensure_lib()
    lib = L.load()
    # build: NULL lattice, empty lattice, periodic too short, Peierls on a real operator
    assert lib.cbdg_build_bdg(None, 1.0, 0.0, None, None, None, None, None, 0.0, 0.01, None, None, None) == L.CBDG_EINVAL
    h = C.c_void_p()
    lat = L.cbdg_lattice(0, 4, 0, 0, 0)
    assert lib.cbdg_build_bdg(C.byref(lat), 1.0, 0.0, 8, 8, None, None, None, 0.0, 0.01, None, C.byref(h), None) == L.CBDG_EINVAL
    assert "empty" in L.cbdg_last_error()
    lat = L.cbdg_lattice(2, 4, 1, 0, 0)
    assert lib.cbdg_build_bdg(C.byref(lat), 1.0, 0.0, 8, 8, None, None, None, 0.0, 0.01, None, C.byref(h), None) == L.CBDG_EINVAL
    assert "periodic" in L.cbdg_last_error()
    lat = L.cbdg_lattice(4, 4, 0, 0, L.CBDG_REAL)
    assert lib.cbdg_build_bdg(C.byref(lat), 1.0, 0.0, 8, 8, None, 8, None, 0.0, 0.01, None, C.byref(h), None) == L.CBDG_EINVAL
    assert "COMPLEX" in L.cbdg_last_error()
    lat = L.cbdg_lattice(4, 4, 0, 0, L.CBDG_REAL)
    assert lib.cbdg_build_bdg(C.byref(lat), 1.0, 0.0, 8, 8, None, None, None, 0.0, 1.5, None, C.byref(h), None) == L.CBDG_EINVAL
    assert "eta" in L.cbdg_last_error()
    # moments: NULL op, bad N
    n = C.c_size_t()
    assert lib.cbdg_moments_workspace_size(None, 64, 0, 0, C.byref(n)) == L.CBDG_EINVAL
    assert lib.cbdg_chebyshev_moments(None, None, 0, 8, 8, 0, 0, None, 0, None, None, None) == L.CBDG_EINVAL
    # gap update: bad N, bad kernel, finite temperature without coefficients,
    # E = 0 outside the interval
    w = L.cbdg_weights(0, 0.0, 0.0, 0.0, 2.0, 0.0)
    assert lib.cbdg_gap_update(None, 4, 0, 0, C.byref(w), None, 1.0, None, None, 1.0, None, 8, None) == L.CBDG_EINVAL
    bad = L.cbdg_weights(7, 0.0, 0.0, 0.0, 2.0, 0.0)
    assert lib.cbdg_gap_update(8, 4, 8, 0, C.byref(bad), None, 1.0, None, 8, 1.0, 8, 8, None) == L.CBDG_EINVAL
    hot = L.cbdg_weights(0, 0.0, 0.1, 0.0, 2.0, 0.0)
    assert lib.cbdg_gap_update(8, 4, 8, 0, C.byref(hot), None, 1.0, None, 8, 1.0, 8, 8, None) == L.CBDG_EINVAL
    assert "cbdg_sum_coefficients" in L.cbdg_last_error()
    neg = L.cbdg_weights(0, 0.0, -0.1, 0.0, 2.0, 0.0)
    assert lib.cbdg_gap_update(8, 4, 8, 0, C.byref(neg), 8, 1.0, None, 8, 1.0, 8, 8, None) == L.CBDG_EINVAL
    off = L.cbdg_weights(0, 0.0, 0.0, 0.0, 2.0, 5.0)
    assert lib.cbdg_gap_update(8, 4, 8, 0, C.byref(off), None, 1.0, None, 8, 1.0, 8, 8, None) == L.CBDG_EINVAL
    # coefficients: bad quantity, NULL output, E = 0 outside; density without coefficients at T > 0
    assert lib.cbdg_sum_coefficients(C.byref(hot), 16, 5, 8, None) == L.CBDG_EINVAL
    assert lib.cbdg_sum_coefficients(C.byref(hot), 16, 0, None, None) == L.CBDG_EINVAL
    assert lib.cbdg_sum_coefficients(C.byref(off), 16, 1, 8, None) == L.CBDG_EINVAL
    assert lib.cbdg_density(8, 4, 8, C.byref(hot), None, 8, None) == L.CBDG_EINVAL
    assert lib.cbdg_density_backward(8, 4, 8, C.byref(hot), None, 8, None) == L.CBDG_EINVAL
    lor = L.cbdg_weights(1, 0.0, 0.0, 0.0, 2.0, 0.0)
    assert lib.cbdg_ldos(8, 4, 8, C.byref(lor), 8, 4, 8, None) == L.CBDG_EINVAL
    assert lib.cbdg_check_moments(None, None, 4, 8, 0, 1e-9, None, None) == L.CBDG_EINVAL
    assert lib.cbdg_op_destroy(None) == L.CBDG_OK


def test_python_errors_carry_message():
    L = _ensure_lib()
    with pytest.raises(L.CbdgError) as e:
        L.cbdg_moments_workspace_size(None, 0, 0, 0, None)
    assert e.value.code == L.CBDG_EINVAL and "moments_workspace_size" in str(e.value)


def test_native_runner_links_the_library_and_checks_its_arguments():
    """The native runner (host code over the C ABI) is built beside the library,
    resolves libcbdg.so from its own folder, and rejects bad arguments before
    any HIP call."""
    runner = os.path.join(ROOT, "paper_1007_1609_amd", "cbdg_moments_run")
    if not os.path.exists(runner):
        sys_path = os.path.join(ROOT, "paper_1007_1609_amd")
        subprocess.check_call(["python", "-c", "import build; build.build_runner()"], cwd=sys_path)
    out = subprocess.run(["ldd", runner], capture_output=True, text=True).stdout
    assert re.search(r"libcbdg\.so => %s" % re.escape(os.path.join(ROOT, "paper_1007_1609_amd")), out), out
    for args in ([], ["256", "256", "1024", "1024", "0", "fp64"], ["64", "4", "16", "8", "300", "fp64"],
                 ["64", "4", "16", "8", "10", "bf16"]):
        r = subprocess.run([runner, *args], capture_output=True, text=True)
        assert r.returncode == 2, (args, r.stdout, r.stderr)
