"""The cache-resident recursion (every step of a tile in one persistent launch
with grid barriers) against the oracle's recursion of eq. (ref2) and against
the HBM-streaming path of cbdg_chebyshev_moments; its size limits and the
bounded barrier."""
import numpy as np
import pytest
import torch

import oracle
import workloads as W
from tests.gpu_common import DEV, TOL_MOMENT, maxdiff

pytestmark = pytest.mark.gpu
TOL_FP32 = 2e-5


def _P():
    import paper_1007_1609_amd as P
    return P


def _resident(w, N, tile, prec=0, sites=None, spin_limit=0, fixed=None):
    P = _P()
    op = P.Operator.from_workload(w, DEV, fixed=fixed)
    s = torch.as_tensor(w.start_sites if sites is None else sites, dtype=torch.int32, device=DEV)
    r_ee, r_he = P.chebyshev_moments_resident(op, s, N, tile, prec, spin_limit=spin_limit)
    h_ee, h_he = P.chebyshev_moments(op, s, N, tile, prec, algorithm=P.CBDG_ALG_DOUBLING if N >= 3 else 0)
    torch.cuda.synchronize()
    a, b = op.bounds.a, op.bounds.b
    op.close()
    return (r_ee.cpu().numpy(), r_he.cpu().numpy(), h_ee.cpu().numpy(), h_he.cpu().numpy(), a, b)


@pytest.mark.parametrize("prec,tol", [(0, TOL_MOMENT), (1, TOL_FP32)], ids=["fp64", "fp32"])
@pytest.mark.parametrize("Lx,Ly,bc,tile,N", [
    (12, 10, 0, 37, 41),     # ragged tiles, odd N, strips of 2
    (9, 13, 0, 64, 40),      # odd width: strips of 1
    (8, 8, 1, 64, 33),       # periodic
    (20, 18, 0, 256, 64),    # one region per workgroup pass
    (16, 40, 0, 100, 30),    # several row segments per strip
    (6, 7, 0, 5, 3),         # N = 3: one doubling step after the first
])
def test_resident_matches_oracle_and_streaming_path(Lx, Ly, bc, tile, N, prec, tol):
    w = W.small_random(Lx, Ly, N=N, seed=Lx * Ly + N, bc_x=bc, bc_y=bc)
    r_ee, r_he, h_ee, h_he, a, b = _resident(w, N, tile, prec)
    o_ee, o_he = oracle.workload_moments(w, a, b)
    print("resident %dx%d N=%d tile %d: |diff| vs oracle ee %.2e he %.2e" % (
        Lx, Ly, N, tile, maxdiff(r_ee, o_ee), maxdiff(r_he, o_he)))
    assert maxdiff(r_ee, o_ee) <= tol and maxdiff(r_he, o_he) <= tol
    # same recursion vectors, dot products summed over other regions
    assert maxdiff(r_ee, h_ee) <= (1e-13 if prec == 0 else 1e-6)
    assert maxdiff(r_he, h_he) <= (1e-13 if prec == 0 else 1e-6)


@pytest.mark.parametrize("N", [1, 2])
def test_resident_few_moments(N):
    w = W.small_random(10, 9, N=N, seed=5)
    r_ee, r_he, _, _, a, b = _resident(w, N, 64)
    o_ee, o_he = oracle.workload_moments(w, a, b, N=N)
    assert maxdiff(r_ee, o_ee) <= TOL_MOMENT and maxdiff(r_he, o_he) <= TOL_MOMENT


def test_resident_invalid_and_duplicate_sites():
    w = W.small_random(10, 8, N=24, seed=7)
    sites = np.array([3, -1, 80, 3, 79, 0], np.int32)
    r_ee, r_he, _, _, a, b = _resident(w, 24, 4, sites=sites)
    assert np.all(np.isnan(r_ee[[1, 2]])) and np.all(np.isnan(r_he[[1, 2]]))
    ok = [0, 3, 4, 5]
    o_ee, o_he = oracle.workload_moments(w, a, b, sites=sites[ok], N=24)
    assert maxdiff(r_ee[ok], o_ee) <= TOL_MOMENT and maxdiff(r_he[ok], o_he) <= TOL_MOMENT
    assert np.array_equal(r_ee[0], r_ee[3])


@pytest.mark.parametrize("prec,tol", [(0, TOL_MOMENT), (1, TOL_FP32)], ids=["fp64", "fp32"])
def test_config4_resident_tiles_at_full_size(prec, tol):
    """128x128, N = 512, tiles of 128 vectors (two 32 MiB FP64 buffers, well
    inside the Infinity Cache): sampled lanes against the oracle, every row
    against the streaming path."""
    w = W.config4()
    _, _, a, b = oracle.workload_bounds(w)
    sites = np.arange(1024, dtype=np.int32) * 97 % w.L2
    r_ee, r_he, h_ee, h_he, a, b = _resident(w, w.N, 128, prec, sites=sites, fixed=(a, b))
    pick = [0, 1, 127, 128, 500, 1023]
    o_ee, o_he = oracle.workload_moments(w, a, b, sites=sites[pick])
    print("config4 resident: |diff| vs oracle ee %.2e he %.2e; vs streaming %.2e" % (
        maxdiff(r_ee[pick], o_ee), maxdiff(r_he[pick], o_he), maxdiff(r_ee, h_ee)))
    assert maxdiff(r_ee[pick], o_ee) <= tol and maxdiff(r_he[pick], o_he) <= tol
    assert maxdiff(r_ee, h_ee) <= (1e-12 if prec == 0 else 1e-6)
    assert maxdiff(r_he, h_he) <= (1e-12 if prec == 0 else 1e-6)


def test_resident_barrier_gives_up_and_the_gpu_stays_usable():
    """A spin limit of one poll makes the first grid barrier give up: every
    workgroup leaves the kernel, the call reports EHIP, and the next call with
    the default limit gives the right moments."""
    P = _P()
    w = W.small_random(24, 20, N=32, seed=3)
    op = P.Operator.from_workload(w, DEV)
    s = torch.as_tensor(w.start_sites, dtype=torch.int32, device=DEV)
    with pytest.raises(P.CbdgError) as e:
        P.chebyshev_moments_resident(op, s, 32, 128, spin_limit=1)
    assert e.value.code == P._lib.CBDG_EHIP and "barrier" in str(e.value)
    r_ee, r_he = P.chebyshev_moments_resident(op, s, 32, 128)
    torch.cuda.synchronize()
    o_ee, o_he = oracle.workload_moments(w, op.bounds.a, op.bounds.b, N=32)
    op.close()
    assert maxdiff(r_ee.cpu().numpy(), o_ee) <= TOL_MOMENT and maxdiff(r_he.cpu().numpy(), o_he) <= TOL_MOMENT


def test_resident_refuses_what_it_does_not_hold():
    P = _P()
    w = W.config1(L=256, N=16)
    op = P.Operator.from_workload(w, DEV)
    with pytest.raises(P.CbdgError) as e:           # 2 x 65536 x 256 x 16 B > 200 MiB
        P.resident_workspace_bytes(op, 256)
    assert e.value.code == P._lib.CBDG_EINVAL and "Infinity Cache" in str(e.value)
    assert P.resident_workspace_bytes(op, 64) > 0   # 2 x 65536 x 64 x 16 B = 128 MiB
    with pytest.raises(P.CbdgError) as e:
        P.resident_workspace_bytes(op, 300)
    assert e.value.code == P._lib.CBDG_EINVAL
    op.close()
    wc = W.small_random(8, 8, N=16, seed=1, complex_=True)
    opc = P.Operator.from_workload(wc, DEV)
    with pytest.raises(P.CbdgError) as e:
        P.resident_workspace_bytes(opc, 64)
    assert e.value.code == P._lib.CBDG_EUNSUPPORTED
    opc.close()
    ws = W.small_random(8, 8, N=16, seed=1)
    ops = P.Operator.from_workload(ws, DEV, fixed=(6.0, 0.25))
    with pytest.raises(P.CbdgError) as e:
        P.resident_workspace_bytes(ops, 64)
    assert e.value.code == P._lib.CBDG_EINVAL
    ops.close()
