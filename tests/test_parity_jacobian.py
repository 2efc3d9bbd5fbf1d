"""Per-start-vector rows of the moments' reverse-mode derivative
(cbdg_chebyshev_moments_jacobian), the library's matrix-vector product, and
the Newton solve that uses the whole Jacobian of the gap map.  Each row is
checked against the CPU oracle's full-storage adjoint run on that start site
alone; the rows' weighted sum against the summed reverse pass; the Newton
fixed point against plain mixing and against the oracle's gap map."""
import numpy as np
import pytest
import torch

import oracle
import workloads as W
from tests.gpu_common import DEV

pytestmark = pytest.mark.gpu

REV = -1
DOUBLING = 2


def _P():
    import paper_1007_1609_amd as P
    return P


def _rel(x, ref):
    return float(np.max(np.abs(np.asarray(x) - np.asarray(ref))) / max(np.max(np.abs(ref)), 1e-300))


def _rows(w, N, dee, dhe, tile, sites=None):
    P = _P()
    op = P.Operator.from_workload(w, DEV)
    s = torch.as_tensor(w.start_sites if sites is None else sites, dtype=torch.int32, device=DEV)
    je, jd = P.chebyshev_moments_jacobian(op, s, N, tile, None if dee is None else torch.as_tensor(dee, device=DEV),
                                          None if dhe is None else torch.as_tensor(dhe, device=DEV), want_eps=True)
    torch.cuda.synchronize()
    a, b = op.bounds.a, op.bounds.b
    op.close()
    return je.cpu().numpy(), jd.cpu().numpy(), a, b


@pytest.mark.parametrize("Lx,Ly,bcx,bcy,N,tile", [
    (64, 6, 0, 0, 20, 100),     # W = 1, ragged tiles
    (128, 5, 1, 0, 25, 300),    # W = 2, periodic x, one tile
    (256, 4, 0, 1, 18, 400),    # W = 4, periodic y, two tiles
])
def test_rows_match_the_oracle_one_start_site_at_a_time(Lx, Ly, bcx, bcy, N, tile):
    w = W.small_random(Lx, Ly, N=N, seed=Lx + Ly + N, bc_x=bcx, bc_y=bcy)
    n = len(w.start_sites)
    rng = np.random.default_rng(n + N)
    dee, dhe = rng.normal(size=(n, N)), rng.normal(size=(n, N))
    je, jd, a, b = _rows(w, N, dee, dhe, tile)
    csr = oracle.workload_csr(w, a, b)
    for k in sorted({0, 1, Lx - 1, Lx, n // 2, n - 1}):
        oe, od = oracle.moments_backward(csr, w.start_sites[k:k + 1], N, dee[k:k + 1], dhe[k:k + 1])
        assert _rel(je[k], oe) < 1e-10 and _rel(jd[k], od) < 1e-10, k


@pytest.mark.parametrize("Lx,Ly,bc,N,tile", [(64, 9, 0, 24, 37), (128, 6, 1, 33, 200), (256, 5, 0, 20, 512)])
def test_weighted_rows_sum_to_the_reverse_pass(Lx, Ly, bc, N, tile):
    """sum_k v_k row_k equals the summed gradient with cotangents v_k dmu[k]."""
    P = _P()
    w = W.small_random(Lx, Ly, N=N, seed=3 * Lx + N, bc_x=bc, bc_y=bc)
    n = len(w.start_sites)
    rng = np.random.default_rng(N)
    dee, dhe = rng.normal(size=(n, N)), rng.normal(size=(n, N))
    v = rng.normal(size=n)
    je, jd, _, _ = _rows(w, N, dee, dhe, tile)
    op = P.Operator.from_workload(w, DEV)
    s = torch.as_tensor(w.start_sites, dtype=torch.int32, device=DEV)
    ge, gd = P.chebyshev_moments_backward(op, s, N, tile, torch.as_tensor(dee * v[:, None], device=DEV),
                                          torch.as_tensor(dhe * v[:, None], device=DEV), REV, algorithm=DOUBLING)
    op.close()
    assert _rel(v @ je, ge.cpu().numpy()) < 1e-12 and _rel(v @ jd, gd.cpu().numpy()) < 1e-12


def test_invalid_start_sites_give_zero_rows():
    w = W.small_random(64, 7, N=16, seed=5)
    sites = np.array([3, -1, 64 * 7, 3, 200], np.int32)
    rng = np.random.default_rng(2)
    dhe = rng.normal(size=(5, 16))
    je, jd, a, b = _rows(w, 16, None, dhe, 4, sites=sites)
    assert not np.any(je[[1, 2]]) and not np.any(jd[[1, 2]])
    assert np.all(np.isfinite(je)) and np.all(np.isfinite(jd))
    csr = oracle.workload_csr(w, a, b)
    # rows 0 and 3: the same start site with different cotangents, each the oracle's
    for k in (0, 3, 4):
        oe, od = oracle.moments_backward(csr, sites[[k]], 16, np.zeros((1, 16)), dhe[[k]])
        assert _rel(jd[k], od) < 1e-10 and _rel(je[k], oe) < 1e-10, k


def test_unsupported_cases_are_refused():
    P = _P()
    for w, N in ((W.small_random(12, 10, N=16, seed=1), 16), (W.small_random(64, 4, N=2, seed=1), 2)):
        op = P.Operator.from_workload(w, DEV)
        s = torch.as_tensor(w.start_sites, dtype=torch.int32, device=DEV)
        dhe = torch.ones((len(w.start_sites), N), dtype=torch.float64, device=DEV)
        with pytest.raises(P.CbdgError) as e:
            P.chebyshev_moments_jacobian(op, s, N, 64, None, dhe)
        assert "EUNSUPPORTED" in str(e.value)
        op.close()


@pytest.mark.parametrize("rows,cols", [(1, 1), (37, 1000), (1000, 64), (4096, 4096)])
def test_matvec_matches_numpy_and_repeats_bit_for_bit(rows, cols):
    P = _P()
    rng = np.random.default_rng(rows + cols)
    A = rng.normal(size=(rows, cols))
    x = rng.normal(size=cols)
    At, xt = torch.as_tensor(A, device=DEV), torch.as_tensor(x, device=DEV)
    y1 = P.jacobian_matvec(At, xt).cpu().numpy()
    y2 = P.jacobian_matvec(At, xt).cpu().numpy()
    ref = A @ x
    assert np.array_equal(y1, y2)
    assert np.max(np.abs(y1 - ref)) <= 1e-13 * max(1.0, float(np.max(np.abs(A) @ np.abs(x))))


def _swave64(N=160, n_imp=9):
    w = W.config4(L=64, N=N, tile=512)
    rng = np.random.default_rng(4)
    eps = np.zeros(64 * 64)
    eps[rng.choice(64 * 64, n_imp, replace=False)] = rng.uniform(0, 4, n_imp)
    return w.with_(eps=eps)


@pytest.mark.parametrize("rebuild", [True, False], ids=["newton", "chord"])
def test_newton_with_the_whole_jacobian_reaches_the_plain_mixing_fixed_point(rebuild):
    P = _P()
    from paper_1007_1609_amd import scf
    w = _swave64()
    d0 = torch.as_tensor(w.delta, device=DEV)
    op = P.Operator.from_workload(w, DEV)
    plain = scf.plain_mixing(op, w.U, d0, w.N, w.tile, tol=1e-9, max_iter=400)
    op.close()
    op = P.Operator.from_workload(w, DEV)
    nk = scf.newton_krylov(op, w.U, d0, w.N, w.tile, tol=1e-9, jv="jacobian", rebuild_jacobian=rebuild)
    op.close()
    print("64x64: plain mixing %d passes, Newton with the whole Jacobian %s" % (plain.moment_passes, nk.counts))
    assert plain.residual < 1e-9 and nk.residual < 1e-9
    assert float(np.max(np.abs(plain.delta.cpu().numpy() - nk.delta.cpu().numpy()))) < 2e-8
    assert nk.counts["jacobian"] >= 1


def test_jacobian_is_symmetric_for_the_gap_map():
    """For a real operator with uniform U the gap map's Jacobian is symmetric
    (the second derivative of one functional); the rows built one start
    vector at a time show it to rounding."""
    P = _P()
    w = _swave64(N=96)
    op = P.Operator.from_workload(w, DEV)
    wts = op.weights("jackson")
    d_mu, _ = P.gap_update_backward(torch.ones(op.L2, dtype=torch.float64, device=DEV), w.N, wts, w.U, 1.0,
                                    want_delta_in=False)
    s = torch.arange(op.L2, dtype=torch.int32, device=DEV)
    _, J = P.chebyshev_moments_jacobian(op, s, w.N, 512, None, d_mu)
    op.close()
    Jn = J.cpu().numpy()
    assert np.max(np.abs(Jn - Jn.T)) <= 1e-12 * np.max(np.abs(Jn))
