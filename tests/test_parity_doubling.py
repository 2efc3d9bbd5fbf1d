"""Moment doubling (ceil((N-1)/2) recursion steps, moments 2n-1 and 2n from
the FP64 dot products of a_n with itself and with a_{n-1}) against the
oracle's direct moments and against the GPU's own direct path, across the
operator variants, ragged tiles, odd and even N, the edge cases, FP32 and
the full 256x256 launch shape."""
import numpy as np
import pytest
import torch

import oracle
import workloads as W
from tests.gpu_common import DEV, TOL_MOMENT, gpu_moments, maxdiff

pytestmark = pytest.mark.gpu

AUTO, DIRECT, DOUBLING = 0, 1, 2


def _both(w, N=None, tile=None, sites=None, precision=0, fixed=None):
    op, d_ee, d_he = gpu_moments(w, sites=sites, N=N, tile=tile, precision=precision, fixed=fixed,
                                 algorithm=DIRECT)
    op.close()
    op, m_ee, m_he = gpu_moments(w, sites=sites, N=N, tile=tile, precision=precision, fixed=fixed,
                                 algorithm=DOUBLING)
    a, b = op.bounds.a, op.bounds.b
    op.close()
    return (d_ee, d_he), (m_ee, m_he), a, b


@pytest.mark.parametrize("case", [
    dict(),
    dict(bc_x=W.PERIODIC, bc_y=W.PERIODIC),
    dict(bond=True, bc_y=W.PERIODIC),
    dict(complex_=True, flux=0.3),
    dict(complex_=True, bond=True, flux=0.25, bc_x=W.PERIODIC, bc_y=W.PERIODIC),
])
@pytest.mark.parametrize("N", [3, 4, 65, 96])
def test_doubling_matches_oracle_and_direct(case, N):
    w = W.small_random(11, 35, N=N, seed=N + 7, **case)
    direct, dbl, a, b = _both(w, tile=128)
    o_ee, o_he = oracle.workload_moments(w, a, b)
    assert b == 0.0
    assert maxdiff(dbl[0], o_ee) <= TOL_MOMENT and maxdiff(dbl[1], o_he) <= TOL_MOMENT
    assert maxdiff(dbl[0], direct[0]) <= 1e-12 and maxdiff(dbl[1], direct[1]) <= 1e-12
    # mu_he of even order vanishes exactly under doubling
    assert np.all(dbl[1][:, 0::2] == 0)


@pytest.mark.parametrize("Lx,Ly,tile,n_sites", [
    (13, 37, 100, 160),
    (40, 70, 300, 300),
    (9, 5, 7, 45),
    (64, 48, 520, 520),    # W = 8 strips, three 256-lane chunks
])
def test_doubling_ragged_shapes(Lx, Ly, tile, n_sites):
    w = W.small_random(Lx, Ly, N=97, seed=Lx + Ly, n_sites=n_sites)
    _, dbl, a, b = _both(w, tile=tile)
    o_ee, o_he = oracle.workload_moments(w, a, b)
    assert maxdiff(dbl[0], o_ee) <= TOL_MOMENT and maxdiff(dbl[1], o_he) <= TOL_MOMENT


@pytest.mark.parametrize("N", [1, 2])
def test_doubling_with_one_or_two_moments_is_direct(N):
    w = W.small_random(6, 7, N=N, seed=2)
    direct, dbl, _, _ = _both(w)
    assert np.array_equal(direct[0], dbl[0]) and np.array_equal(direct[1], dbl[1])


def test_doubling_refuses_uncentred_rescaling():
    import paper_1007_1609_amd as P
    w = W.small_random(10, 9, N=64, seed=3)
    op = P.Operator.from_workload(w, DEV, fixed=(6.25, 0.31))
    with pytest.raises(P.CbdgError) as e:
        P.moments_workspace_bytes(op, 64, 0, DOUBLING)
    assert e.value.code == -1 and "b = 0" in str(e.value)
    st = torch.as_tensor(w.start_sites, device=DEV)
    ws = P.workspace(P.moments_workspace_bytes(op, 64, 0, DIRECT), DEV)
    with pytest.raises(P.CbdgError) as e:
        P.chebyshev_moments(op, st, 64, 64, ws=ws, algorithm=DOUBLING)
    assert e.value.code == -1
    # AUTO takes the direct path and matches the oracle
    mu_ee, mu_he = P.chebyshev_moments(op, st, 64, 64, ws=ws, algorithm=AUTO)
    o_ee, o_he = oracle.workload_moments(w, 6.25, 0.31)
    assert maxdiff(mu_ee.cpu().numpy(), o_ee) <= TOL_MOMENT
    assert maxdiff(mu_he.cpu().numpy(), o_he) <= TOL_MOMENT
    op.close()


def test_doubling_workspace_is_checked():
    import paper_1007_1609_amd as P
    w = W.small_random(16, 16, N=20, seed=5)
    op = P.Operator.from_workload(w, DEV)
    st = torch.as_tensor(w.start_sites, device=DEV)
    from paper_1007_1609_amd import _lib as L
    n = st.numel()
    small = P.moments_workspace_bytes(op, n, 0, DIRECT)
    assert P.moments_workspace_bytes(op, n, 0, DOUBLING) > small
    ws = P.workspace(small, DEV)
    mu_ee = torch.empty((n, 20), dtype=torch.float64, device=DEV)
    mu_he = torch.empty((n, 20), dtype=torch.float64, device=DEV)
    args = (op.handle, st.data_ptr(), n, 20, n, 0)
    tail = (ws.data_ptr(), small, mu_ee.data_ptr(), mu_he.data_ptr(), torch.cuda.current_stream().cuda_stream)
    with pytest.raises(P.CbdgError) as e:
        L.cbdg_chebyshev_moments(*args, DOUBLING, *tail)
    assert e.value.code == -1 and "workspace" in str(e.value)
    L.cbdg_chebyshev_moments(*args, DIRECT, *tail)
    torch.cuda.synchronize()
    o_ee, _ = oracle.workload_moments(w, op.bounds.a, op.bounds.b, N=20)
    op.close()
    assert maxdiff(mu_ee.cpu().numpy(), o_ee) <= TOL_MOMENT


def test_doubling_invalid_sites_keep_nan_rows():
    w = W.small_random(6, 6, N=12, seed=1)
    op, g_ee, g_he = gpu_moments(w, sites=np.array([3, -1, 36, 7], np.int32), tile=4, algorithm=DOUBLING)
    assert np.all(np.isnan(g_ee[1])) and np.all(np.isnan(g_ee[2])) and np.all(np.isnan(g_he[1]))
    o_ee, o_he = oracle.workload_moments(w, op.bounds.a, op.bounds.b, sites=[3, 7], N=12)
    op.close()
    assert maxdiff(g_ee[[0, 3]], o_ee) <= TOL_MOMENT and maxdiff(g_he[[0, 3]], o_he) <= TOL_MOMENT


def test_doubling_duplicate_sites_and_tiny_tiles():
    w = W.small_random(12, 10, N=50, seed=2)
    sites = np.array([5, 5, 119, 0, 64, 5, 33], dtype=np.int32)
    _, dbl, a, b = _both(w, sites=sites, tile=3)
    o_ee, o_he = oracle.workload_moments(w, a, b, sites=sites)
    assert maxdiff(dbl[0], o_ee) <= TOL_MOMENT and maxdiff(dbl[1], o_he) <= TOL_MOMENT


def test_doubling_bits_are_reproducible():
    w = W.small_random(24, 20, N=64, seed=9)
    _, d1, _, _ = _both(w, tile=128)
    _, d2, _, _ = _both(w, tile=128)
    assert np.array_equal(d1[0], d2[0]) and np.array_equal(d1[1], d2[1])


@pytest.mark.parametrize("complex_", [False, True])
def test_doubling_fp32(complex_):
    """FP32 vectors, FP64 dot products: error against the FP64 oracle within
    the bar of the direct FP32 path (2e-5 at these N)."""
    kw = dict(complex_=True, bond=True, flux=0.1) if complex_ else {}
    w = W.small_random(48, 40, N=512 if not complex_ else 256, seed=14, n_sites=64, **kw)
    direct, dbl, a, b = _both(w, tile=64, precision=1)
    o_ee, o_he = oracle.workload_moments(w, a, b)
    e_d = max(maxdiff(direct[0], o_ee), maxdiff(direct[1], o_he))
    e_m = max(maxdiff(dbl[0], o_ee), maxdiff(dbl[1], o_he))
    print("fp32 %s: max error direct %.2e, doubling %.2e" % ("complex" if complex_ else "real", e_d, e_m))
    assert e_m < 2e-5 and e_d < 2e-5


def test_doubling_full_size_launch_shape():
    """256x256, one tile of 1024 vectors, N = 1024: doubling against the
    GPU's direct path on every moment, and sampled rows against the oracle."""
    w = W.config1()
    sites = np.arange(1024, dtype=np.int32) * 61 % w.L2
    direct, dbl, a, b = _both(w, sites=sites, tile=1024)
    dd = max(maxdiff(direct[0], dbl[0]), maxdiff(direct[1], dbl[1]))
    pick = [0, 255, 256, 1023]
    o_ee, o_he = oracle.workload_moments(w, a, b, sites=sites[pick])
    do = max(maxdiff(dbl[0][pick], o_ee), maxdiff(dbl[1][pick], o_he))
    print("256x256 N=1024: doubling vs direct %.2e, vs oracle %.2e" % (dd, do))
    assert dd <= TOL_MOMENT and do <= TOL_MOMENT
