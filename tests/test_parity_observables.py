"""GPU gap update, LDOS and the self-consistency loop vs the CPU oracle."""
import numpy as np
import pytest
import torch

import oracle
import workloads as W
from tests.gpu_common import DEV, maxdiff

pytestmark = pytest.mark.gpu


def _P():
    import paper_1007_1609_amd as P
    return P


def _rand_moments(n, N, cplx, seed):
    rng = np.random.default_rng(seed)
    mu = rng.uniform(-1, 1, (n, N)) / np.sqrt(1 + np.arange(N))
    if cplx:
        mu = mu + 1j * rng.uniform(-1, 1, (n, N)) / np.sqrt(1 + np.arange(N))
    return mu


@pytest.mark.parametrize("cplx", [False, True])
@pytest.mark.parametrize("kernel,lam", [("jackson", 0.0), ("lorentz", 3.0)])
@pytest.mark.parametrize("a,b,E_c", [(7.0, 0.0, 0.0), (5.5, 0.3, 0.0), (6.0, -0.2, 2.5)])
def test_gap_update_matches_oracle(cplx, kernel, lam, a, b, E_c):
    P = _P()
    n, N, U, alpha = 333, 257, 2.5, 0.7
    mu = _rand_moments(n, N, cplx, 1)
    rng = np.random.default_rng(2)
    din = rng.uniform(0, 0.3, n) + (1j * rng.uniform(-0.1, 0.1, n) if cplx else 0)
    ref_new = oracle.gap_map(mu, U, kernel=kernel, lam=lam, a=a, b=b, E_c=E_c)
    if not cplx:
        ref_new = ref_new.real
    ref_out = (1 - alpha) * din + alpha * ref_new
    ref_r = np.max(np.abs(ref_new - din))
    w = P.weights(a, b, kernel, lam, 0.0, E_c)
    mu_t = torch.as_tensor(mu, device=DEV)
    din_t = torch.as_tensor(din, device=DEV)
    out, r = P.gap_update(mu_t, w, U, din_t, alpha)
    assert maxdiff(out.cpu().numpy(), ref_out) <= 1e-12
    assert abs(float(r.item()) - ref_r) <= 1e-12


def test_gap_update_per_row_coupling_and_alias():
    P = _P()
    n, N = 70, 64
    mu = _rand_moments(n, N, False, 3)
    U = np.random.default_rng(4).uniform(1, 3, n)
    din = np.full(n, 0.1)
    ref = oracle.gap_map(mu, U, a=4.0).real
    d = torch.as_tensor(din, device=DEV)
    out, r = P.gap_update(torch.as_tensor(mu, device=DEV), P.weights(4.0, 0.0), 0.0, d, 1.0,
                          U_rows=torch.as_tensor(U, device=DEV), delta_out=d)
    assert out.data_ptr() == d.data_ptr()
    assert maxdiff(d.cpu().numpy(), ref) <= 1e-12


def test_gap_update_empty_rows_sets_zero_residual():
    P = _P()
    r = torch.full((1,), 5.0, dtype=torch.float64, device=DEV)
    P.gap_update(torch.zeros((0, 8), dtype=torch.float64, device=DEV), P.weights(3.0, 0.0), 1.0,
                 torch.zeros(0, dtype=torch.float64, device=DEV), resid=r)
    assert float(r.item()) == 0.0


def test_gap_update_nan_propagates_to_residual():
    P = _P()
    mu = _rand_moments(10, 16, False, 5)
    mu[3, 4] = np.nan
    _, r = P.gap_update(torch.as_tensor(mu, device=DEV), P.weights(3.0, 0.0), 1.0,
                        torch.zeros(10, dtype=torch.float64, device=DEV))
    assert np.isnan(float(r.item()))


@pytest.mark.parametrize("kernel,lam", [("jackson", 0.0), ("lorentz", 4.0)])
def test_ldos_matches_oracle(kernel, lam):
    P = _P()
    n, N, a, b = 45, 300, 5.0, 0.2
    mu = _rand_moments(n, N, False, 6)
    E = np.linspace(-4.5, 4.9, 601)
    ref = oracle.ldos(mu, E, a, b, kernel, lam)
    got = P.ldos(torch.as_tensor(mu, device=DEV), P.weights(a, b, kernel, lam),
                 torch.as_tensor(E, device=DEV)).cpu().numpy()
    assert maxdiff(got, ref) <= 1e-10 * np.max(np.abs(ref))


def test_ldos_outside_interval_is_nan():
    P = _P()
    mu = _rand_moments(2, 8, False, 7)
    E = np.array([-3.0, 0.0, 2.0, 2.5])
    got = P.ldos(torch.as_tensor(mu, device=DEV), P.weights(2.0, 0.0), torch.as_tensor(E, device=DEV)).cpu().numpy()
    assert np.all(np.isnan(got[:, [0, 2, 3]])) and np.all(np.isfinite(got[:, 1]))


def test_config0_one_gap_update_and_ldos_end_to_end():
    P = _P()
    w = W.config0()
    op = P.Operator.from_workload(w, DEV)
    a, b = op.bounds.a, op.bounds.b
    sites = torch.as_tensor(w.start_sites, device=DEV)
    mu_ee, mu_he = P.chebyshev_moments(op, sites, w.N, w.tile)
    wt = op.weights()
    new, r = P.gap_update(mu_he, wt, w.U, torch.as_tensor(w.delta, device=DEV))
    E = torch.linspace(-2, 2, 101, dtype=torch.float64, device=DEV)
    ld = P.ldos(mu_ee, wt, E)
    o_ee, o_he = oracle.workload_moments(w, a, b)
    o_new = oracle.gap_map(o_he, w.U).real
    o_ld = oracle.ldos(o_ee, E.cpu().numpy(), a, b)
    op.close()
    print("config0: one-step Delta err %.2e, LDOS rel err %.2e" % (
        maxdiff(new.cpu().numpy(), o_new), maxdiff(ld.cpu().numpy(), o_ld) / np.max(np.abs(o_ld))))
    assert maxdiff(new.cpu().numpy(), o_new) <= 1e-10
    assert abs(float(r.item()) - np.max(np.abs(o_new - w.delta))) <= 1e-10
    assert maxdiff(ld.cpu().numpy(), o_ld) <= 1e-10 * np.max(np.abs(o_ld))


def test_config0_scf_matches_oracle_scf():
    """Same number of plain-mixing iterations on both sides, then compare."""
    P = _P()
    from paper_1007_1609_amd import scf
    w = W.config0()
    o_delta, o_it, o_r, _ = oracle.scf_plain(w, tol=1e-9, max_iter=300)
    op = P.Operator.from_workload(w, DEV)
    res = scf.plain_mixing(op, w.U, torch.as_tensor(w.delta, device=DEV), w.N, w.tile, tol=0.0,
                           max_iter=o_it)
    op.close()
    err = maxdiff(res.delta.cpu().numpy(), o_delta)
    print("config0 SCF: %d iterations, residual %.2e, max |Delta_gpu - Delta_oracle| = %.2e" % (
        o_it, res.residual, err))
    assert res.iterations == o_it and abs(res.residual - o_r) < 1e-12
    assert err <= 1e-10


def test_scf_fixed_point_under_oracle_map():
    """The GPU's self-consistent Delta is a fixed point of the oracle's gap map."""
    P = _P()
    from paper_1007_1609_amd import scf
    w = W.small_random(20, 18, N=256, seed=31)
    w = w.with_(delta=np.full(w.L2, 0.1), U=2.2)
    op = P.Operator.from_workload(w, DEV)
    res = scf.plain_mixing(op, w.U, torch.as_tensor(w.delta, device=DEV), w.N, 512, tol=1e-8, max_iter=400)
    d = res.delta.cpu().numpy()
    _, o_he = oracle.workload_moments(w, op.bounds.a, op.bounds.b, delta=d)
    op.close()
    assert res.residual < 1e-8
    assert maxdiff(oracle.gap_map(o_he, w.U).real, d) < 2e-8
