"""The moments entry point that allocates nothing (cbdg_chebyshev_moments_static)
against cbdg_chebyshev_moments with a caller workspace, called through the C
ABI: two calls in a row on one GPU, the second with a smaller input, each
bitwise equal to the workspace call and within 1e-10 of the oracle."""
import ctypes as C

import numpy as np
import pytest
import torch

import oracle
import workloads as W
from tests.gpu_common import DEV, TOL_MOMENT, maxdiff

pytestmark = pytest.mark.gpu


def _static(op, sites, N, tile, prec, alg):
    import paper_1007_1609_amd as P
    L = P._lib
    n = sites.numel()
    mu_ee = torch.full((n, N), 7.0, dtype=torch.float64, device=DEV)
    mu_he = torch.full((n, N), 7.0, dtype=torch.float64, device=DEV)
    L.cbdg_chebyshev_moments_static(op.handle, C.c_void_p(sites.data_ptr()), n, N, tile, prec, alg,
                                    C.c_void_p(mu_ee.data_ptr()), C.c_void_p(mu_he.data_ptr()),
                                    C.c_void_p(torch.cuda.current_stream().cuda_stream))
    return mu_ee, mu_he


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("alg", [0, 1])
def test_static_scratch_moments_equal_workspace_moments(prec, alg):
    import paper_1007_1609_amd as P
    assert P._lib.cbdg_static_scratch_bytes() == 64 << 20
    cases = [
        (W.config0(), 256, 256),                          # 16x16, all sites, one tile
        (W.small_random(12, 10, N=64, seed=3), 37, 64),   # smaller: ragged tiles of 37
    ]
    for w, tile, N in cases:
        op = P.Operator.from_workload(w, DEV)
        sites = torch.as_tensor(w.start_sites, dtype=torch.int32, device=DEV)
        s_ee, s_he = _static(op, sites, N, tile, prec, alg)
        r_ee, r_he = P.chebyshev_moments(op, sites, N, tile, prec, algorithm=alg)
        torch.cuda.synchronize()
        assert torch.equal(s_ee, r_ee) and torch.equal(s_he, r_he)
        o_ee, o_he = oracle.workload_moments(w, op.bounds.a, op.bounds.b, N=N)
        tol = TOL_MOMENT if prec == 0 else 2e-5
        assert maxdiff(s_ee.cpu().numpy(), o_ee) <= tol and maxdiff(s_he.cpu().numpy(), o_he) <= tol
        op.close()


def test_static_scratch_rejects_tiles_beyond_the_array():
    import paper_1007_1609_amd as P
    w = W.config1(L=64, N=16)
    op = P.Operator.from_workload(w, DEV)
    sites = torch.arange(1024, dtype=torch.int32, device=DEV)
    with pytest.raises(P.CbdgError) as e:
        _static(op, sites, 16, 1024, 0, 0)
    assert e.value.code == P._lib.CBDG_EINVAL and "static scratch" in str(e.value)
    # tiles small enough for the array run
    s_ee, _ = _static(op, sites[:64], 16, 16, 0, 0)
    r_ee, _ = P.chebyshev_moments(op, sites[:64], 16, 16)
    torch.cuda.synchronize()
    assert torch.equal(s_ee, r_ee)
    op.close()
