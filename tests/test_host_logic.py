"""Host-side pieces of the product that need no GPU."""
import numpy as np
import pytest


def test_gmres_solves_nonsymmetric_system():
    from paper_1007_1609_amd.scf import _gmres
    rng = np.random.default_rng(0)
    n = 60
    A = np.eye(n) * 3 + rng.normal(size=(n, n)) / np.sqrt(n)
    b = rng.normal(size=n)
    calls = []

    def mv(v):
        calls.append(1)
        return A @ v

    x, used = _gmres(mv, b, 1e-12, restart=15, maxiter=400)
    assert np.linalg.norm(A @ x - b) <= 1e-10 * np.linalg.norm(b)
    assert used == len(calls)


def test_gmres_zero_rhs():
    from paper_1007_1609_amd.scf import _gmres
    x, used = _gmres(lambda v: v, np.zeros(5), 1e-8)
    assert used == 0 and np.all(x == 0)


def _schedule(fast=1, switch_tol=None, tol=1e-6):
    from paper_1007_1609_amd.scf import _PrecisionSchedule
    return _PrecisionSchedule(0, fast, switch_tol, tol)


def test_precision_schedule_without_a_fast_precision_is_the_plain_test():
    s = _schedule(fast=None)
    assert s.current == 0
    assert not s.done(2e-6) and s.done(5e-7)
    assert s.fast_evaluations == 0
    # the same precision given twice is no schedule either
    assert _schedule(fast=0).current == 0


def test_precision_schedule_switches_below_half_the_tolerance():
    s = _schedule()
    assert s.switch_tol == 5e-7
    assert s.current == 1
    # a reduced-precision residual below tol does not end the loop
    for r in (1e-1, 1e-3, 8e-7):
        assert not s.done(r) and s.current == 1
    assert not s.done(4e-7)          # below switch_tol: next evaluation in FP64
    assert s.current == 0 and s.fast_evaluations == 4
    assert not s.done(3e-6)          # FP64 above tol: keep going in FP64
    assert s.done(9e-7) and s.current == 0


def test_precision_schedule_switches_when_the_residual_stalls():
    s = _schedule(switch_tol=1e-12, tol=1e-9)
    for r in (1e-2, 1e-3, 5e-5, 3e-6):
        assert not s.done(r) and s.current == 1
    assert not s.done(2.9e-6)        # below 1e-4 and not falling: the FP32 floor
    assert s.current == 0
    # above 1e-4 a slow phase is not taken for the floor
    s = _schedule(switch_tol=1e-12, tol=1e-9)
    assert not s.done(1e-2) and not s.done(0.95e-2) and s.current == 1


def test_precision_schedule_default_switch_is_floored():
    assert _schedule(tol=1e-9).switch_tol == 1e-7
    assert _schedule(tol=1e-4).switch_tol == 5e-5


def test_reverse_pass_accounting_matches_the_library_plan():
    """Launch and vector-stream counts of the doubling-form reverse pass for
    the 128x128, N = 512 workload (M = 256).  Default checkpoint stride 18
    (ceil(sqrt(257)) = 17 rounded up to a multiple of 3), 15 segments: the
    forward is 1 step + 85 three-step passes; 14 segments are recomputed by
    8 two-step passes each, the last (a_254 .. a_256) by a pair and a single
    step; 256 adjoint steps follow."""
    import bench_forms
    streams, launches = bench_forms.adjoint_traffic(512, 128 * 128)
    assert launches == (1 + 85) + (14 * 8 + 2) + 256
    fwd = 1 + 2 + 85 * 4
    rec = 14 * 8 * 4 + 4 + 3
    adj = 254 * 5 + 4 + 3
    assert streams == fwd + rec + adj
    # stride 17 (not a multiple of 3): two-step forward, 1 + 127 passes + 1
    s17, l17 = bench_forms.adjoint_traffic(512, 128 * 128, ckpt=17)
    assert l17 == (1 + 127 + 1) + 15 * (7 + 1) + 256
    assert s17 == (1 + 2 + 127 * 4 + 3) + 15 * (7 * 4 + 3) + adj
    # stride 1 stores every vector: no recomputation, two-step forward
    s1, l1 = bench_forms.adjoint_traffic(512, 128 * 128, ckpt=1)
    assert l1 == 129 + 256 and s1 == (1 + 2 + 127 * 4 + 3) + adj
    # small tiles: two-step forward at stride 18
    s64, l64 = bench_forms.adjoint_traffic(512, 128 * 128, tile=64)
    assert l64 == (1 + 127 + 1) + (14 * 8 + 2) + 256


def _diamond_brute(x, y, Lx, Ly, bcx, bcy, R):
    X, Y = np.meshgrid(np.arange(Lx), np.arange(Ly))
    tot = 0
    for xi, yi in zip(x, y):
        dx, dy = np.abs(X - xi), np.abs(Y - yi)
        if bcx:
            dx = np.minimum(dx, Lx - dx)
        if bcy:
            dy = np.minimum(dy, Ly - dy)
        tot += int(((dx + dy) <= R).sum())
    return tot


@pytest.mark.parametrize("Lx,Ly", [(7, 5), (16, 9), (64, 3), (10, 10), (8, 8)])
@pytest.mark.parametrize("bcx,bcy", [(0, 0), (1, 0), (0, 1), (1, 1)])
def test_light_cone_site_count_is_exact(Lx, Ly, bcx, bcy):
    """The closed form (open lattice) and the row sums (periodic directions)
    of the sites within lattice distance R of each start site, against a
    brute-force count, for radii from 0 to past the lattice's diameter."""
    import bench_forms
    rng = np.random.default_rng(Lx * Ly + 2 * bcx + bcy)
    x, y = rng.integers(0, Lx, 7), rng.integers(0, Ly, 7)
    for R in (0, 1, 2, 3, 4, 5, 8, 13, 30):
        assert bench_forms.diamond_sites(x, y, Lx, Ly, bcx, bcy, R) == _diamond_brute(x, y, Lx, Ly, bcx, bcy, R)


def test_vector_contiguous_pass_schedule():
    """N/2 steps as the first step, passes of K steps from step 2, the
    remainder in one shorter pass (two or more steps) or a single step; bytes
    per pass = cones of a_{n-2}, a_{n-1} read and of the last two written."""
    import bench_forms
    L, sites = 256, np.array([0, 300, 65535])
    for N, K, passes, tail, singles in ((1024, 7, 73, 0, 0), (2048, 7, 146, 0, 1), (1024, 6, 85, 0, 1),
                                        (512, 7, 36, 3, 0), (14, 6, 1, 0, 0), (12, 6, 0, 5, 0), (6, 3, 0, 2, 0)):
        launches, moved, streamed = bench_forms.vc_traffic(sites, L, L, 0, 0, N // 2, K)
        assert launches == 1 + passes + (tail > 0) + singles
        assert streamed == 3 * L * L * (N // 2) * 3

        def D(R):
            return bench_forms.diamond_sites(sites % L, sites // L, L, L, 0, 0, R)
        want = D(0) + D(1)
        n = 2
        for _ in range(passes):
            want += D(n - 2) + D(n - 1) + D(n + K - 2) + D(n + K - 1)
            n += K
        if tail:
            want += D(n - 2) + D(n - 1) + D(n + tail - 2) + D(n + tail - 1)
            n += tail
        for _ in range(singles):
            want += D(n - 2) + D(n - 1) + D(n)
            n += 1
        assert n == N // 2 + 1 and moved == want


def test_closed_operator_raises_before_any_library_call():
    # a released operator hands out no pointer: every wrapper that needs the
    # handle raises on the host instead of passing freed memory to the library
    import pytest
    import paper_1007_1609_amd as P
    op = object.__new__(P.Operator)
    op._handle, op._alive = None, False
    with pytest.raises(ValueError, match="closed"):
        P.moments_workspace_bytes(op, 64)
    with pytest.raises(ValueError, match="closed"):
        P.backward_workspace_bytes(op, 64, 16)
    with pytest.raises(ValueError, match="closed"):
        op.update_delta(None)
    op.close()   # closing twice is a no-op


def test_newton_krylov_rejects_an_unknown_product_before_any_library_call():
    from paper_1007_1609_amd import scf
    with pytest.raises(ValueError):
        scf.newton_krylov(None, 2.0, None, 64, 64, jv="hessian")


def test_jacobian_matvec_checks_its_operands_on_the_host():
    import torch
    import paper_1007_1609_amd as P
    with pytest.raises(ValueError):
        P.jacobian_matvec(torch.zeros(3, 4, dtype=torch.float64).t(), torch.zeros(3, dtype=torch.float64))
    with pytest.raises(ValueError):
        P.jacobian_matvec(torch.zeros(3, 4, dtype=torch.float64), torch.zeros(2, dtype=torch.float64))
    with pytest.raises(ValueError):  # host tensors never reach the library
        P.jacobian_matvec(torch.zeros(3, 4, dtype=torch.float64), torch.zeros(4, dtype=torch.float64))


def test_bench_refuses_more_than_one_gpu():
    """bench.py runs on one GPU; --gpus N > 1 exits with a message before
    anything touches a device."""
    import os
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120, cwd=root)
    assert r.returncode == 2 and "one GPU" in r.stderr and r.stdout == ""
