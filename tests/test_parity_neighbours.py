"""Neighbour moments <j,alpha|T_n|i,e> of the four lattice neighbours of each
start site, the bond order parameter and the bond current, against the
oracle's recursion, the Bloch closed form of a uniform d-wave lattice, and a
bond self-consistency loop written with the oracle."""
import numpy as np
import pytest
import torch

import oracle
import workloads as W
from tests.gpu_common import DEV, TOL_MOMENT, maxdiff

pytestmark = pytest.mark.gpu


def _P():
    import paper_1007_1609_amd as P
    return P


def _gpu_nb(w, sites=None, tile=None, precision=0, fixed=None):
    P = _P()
    op = P.Operator.from_workload(w, DEV, fixed=fixed)
    s = torch.as_tensor(w.start_sites if sites is None else sites, dtype=torch.int32, device=DEV)
    out = P.chebyshev_moments_nb(op, s, w.N, w.tile if tile is None else tile, precision)
    torch.cuda.synchronize()
    return op, [o.cpu().numpy() for o in out]


@pytest.mark.parametrize("case,tile", [
    (dict(), 64),
    (dict(bc_x=W.PERIODIC, bc_y=W.PERIODIC), 37),
    (dict(bond=True, bc_y=W.PERIODIC), 128),
    (dict(complex_=True, bond=True, flux=0.2, bc_x=W.PERIODIC), 50),
    (dict(complex_=True, flux=0.3), 300),
])
def test_neighbour_moments_match_oracle(case, tile):
    w = W.small_random(11, 13, N=70, seed=51, **case)
    op, (mee, mhe, nee, nhe) = _gpu_nb(w, tile=tile)
    a, b = op.bounds.a, op.bounds.b
    op.close()
    H = oracle.workload_csr(w, a, b)
    oee, ohe = oracle.neighbour_moments(H, w.Lx, w.Ly, w.bc_x, w.bc_y, w.start_sites, w.N)
    if w.scalar != "complex":
        oee, ohe = oee.real, ohe.real
    print("neighbour moments %s: max |diff| ee %.2e he %.2e" % (case, maxdiff(nee, oee), maxdiff(nhe, ohe)))
    assert maxdiff(nee, oee) <= TOL_MOMENT and maxdiff(nhe, ohe) <= TOL_MOMENT
    lee, lhe = oracle.workload_moments(w, a, b)
    assert maxdiff(mee, lee) <= TOL_MOMENT and maxdiff(mhe, lhe) <= TOL_MOMENT


def test_neighbour_moments_fp32_and_invalid_sites():
    w = W.small_random(16, 9, N=120, seed=52)
    sites = np.array([3, -2, 100, 144, 143], dtype=np.int32)     # 144 = L2: invalid
    op, (mee, mhe, nee, nhe) = _gpu_nb(w, sites=sites, tile=4, precision=1)
    a, b = op.bounds.a, op.bounds.b
    op.close()
    assert np.all(np.isnan(nee[1])) and np.all(np.isnan(nhe[3])) and np.all(np.isnan(mee[3]))
    ok = [0, 2, 4]
    oee, ohe = oracle.neighbour_moments(oracle.workload_csr(w, a, b), w.Lx, w.Ly, 0, 0, sites[ok], w.N)
    assert maxdiff(nee[ok], oee.real) < 2e-5 and maxdiff(nhe[ok], ohe.real) < 2e-5
    # site 143 is the last corner: its +x and +y neighbours are missing rows of zeros
    assert np.all(nee[4, 0] == 0) and np.all(nee[4, 2] == 0)


def test_bond_gap_update_matches_oracle():
    P = _P()
    w = W.small_random(10, 12, N=90, seed=53, complex_=True, bond=True, flux=0.1, bc_y=W.PERIODIC)
    op, (_, _, _, nhe) = _gpu_nb(w)
    a, b = op.bounds.a, op.bounds.b
    db_in = torch.as_tensor(w.delta_bond.reshape(-1), device=DEV)
    new, r = P.bond_gap_update(torch.as_tensor(nhe, device=DEV), op, op.weights(), 1.3, db_in, 0.6)
    op.close()
    H = oracle.workload_csr(w, a, b)
    _, ohe = oracle.neighbour_moments(H, w.Lx, w.Ly, w.bc_x, w.bc_y, w.start_sites, w.N)
    ref = oracle.bond_gap_map(ohe, 1.3, w.Lx, w.Ly, w.bc_x, w.bc_y, oracle.gap_weights(w.N))
    mixed = 0.4 * w.delta_bond + 0.6 * ref
    assert maxdiff(new.cpu().numpy(), mixed.reshape(-1)) < 1e-10
    assert abs(float(r.item()) - np.max(np.abs(ref - w.delta_bond))) < 1e-10


def test_bond_gap_bloch_closed_form_at_64x64():
    """Uniform d-wave bonds on a periodic 64x64 lattice: the map must give
    (U/4)(conj S_+ + conj S_-) with S from the Bloch sum, and Delta_y = -Delta_x."""
    P = _P()
    L, t, mu, D0, U, N = 64, 1.0, -0.3, 0.15, 1.7, 128
    L2 = L * L
    db = np.zeros((2, L2), dtype=np.complex128)
    db[0], db[1] = D0, -D0
    w = W.Workload("dwave64", L, L, W.PERIODIC, W.PERIODIC, t, mu, U, np.zeros(L2), np.zeros(L2), db, None, N,
                   np.arange(L2, dtype=np.int32), 1024, scalar="complex", pairing="bond")
    a = 6.3
    op, (_, _, _, nhe) = _gpu_nb(w, fixed=(a, 0.0))
    new, _ = P.bond_gap_update(torch.as_tensor(nhe, device=DEV), op, op.weights(), U,
                               torch.as_tensor(db.reshape(-1), device=DEV), 1.0)
    op.close()
    new = new.cpu().numpy().reshape(2, L2)
    k = 2 * np.pi * np.arange(L) / L
    kx, ky = np.meshgrid(k, k, indexing="ij")
    xi = -2 * t * (np.cos(kx) + np.cos(ky)) - mu
    Dk = 2 * D0 * (np.cos(kx) - np.cos(ky))
    E = np.sqrt(xi ** 2 + Dk ** 2)
    p = np.polynomial.chebyshev.chebval(E / a, oracle.gap_weights(N))
    Sx = np.mean(np.exp(-1j * kx) * Dk * p / E)
    Sxm = np.mean(np.exp(1j * kx) * Dk * p / E)
    ref_x = 0.25 * U * (np.conj(Sx) + np.conj(Sxm))
    print("d-wave 64x64: Delta_x new %.6f, closed form %.6f" % (new[0].real.mean(), ref_x.real))
    assert maxdiff(new[0], ref_x) < 1e-12 and maxdiff(new[1], -ref_x) < 1e-12


@pytest.mark.parametrize("pairing", [False, True])
def test_bond_current_matches_oracle(pairing):
    P = _P()
    w = W.small_random(9, 8, N=150, seed=54, complex_=True, flux=0.17, bc_x=W.PERIODIC)
    if not pairing:
        w = w.with_(delta=np.zeros(w.L2, dtype=np.complex128))
    op, (_, _, nee, _) = _gpu_nb(w)
    a, b = op.bounds.a, op.bounds.b
    wt = op.weights(T=0.08)
    J = P.bond_current(op, torch.as_tensor(nee, device=DEV), wt).cpu().numpy()
    op.close()
    H = oracle.workload_csr(w, a, b)
    oee, _ = oracle.neighbour_moments(H, w.Lx, w.Ly, w.bc_x, w.bc_y, w.start_sites, w.N)
    wf = oracle.jackson(w.N) * oracle.thermal_coefficients(w.N, a, b, 0.08, quantity="density")
    ref = oracle.bond_current(oee, w.t, w.peierls, w.Lx, w.Ly, w.bc_x, w.bc_y, wf)
    print("bond current (pairing=%s): max |J| %.3e, max |diff| %.2e" % (pairing, np.abs(ref).max(), maxdiff(J, ref)))
    assert np.abs(ref).max() > 1e-4
    assert maxdiff(J, ref) < 1e-10


def test_dwave_bond_self_consistency_matches_oracle_loop():
    """Plain mixing of the bond order parameter on a periodic 8x8 lattice from
    a d-wave guess, against the same loop written with the oracle."""
    P = _P()
    from paper_1007_1609_amd import scf
    L, N, U = 8, 96, 2.2
    L2 = L * L
    db0 = np.zeros((2, L2), dtype=np.complex128)
    db0[0], db0[1] = 0.2, -0.2
    w = W.Workload("dw8", L, L, W.PERIODIC, W.PERIODIC, 1.0, -0.5, U, np.zeros(L2), np.zeros(L2, np.complex128),
                   db0, None, N, np.arange(L2, dtype=np.int32), L2, scalar="complex", pairing="bond")
    a = 6.0
    wts = oracle.gap_weights(N)
    cur = db0.copy()
    it_ref = 0
    for it_ref in range(1, 60):
        H = oracle.workload_csr(w.with_(delta_bond=cur), a, 0.0)
        _, he = oracle.neighbour_moments(H, L, L, 1, 1, np.arange(L2), N)
        new = oracle.bond_gap_map(he, U, L, L, 1, 1, wts)
        r = np.max(np.abs(new - cur))
        cur = new
        if r < 1e-9:
            break
    op = P.Operator.from_workload(w, DEV, fixed=(a, 0.0))
    res = scf.bond_plain_mixing(op, U, torch.zeros(L2, dtype=torch.complex128, device=DEV),
                                torch.as_tensor(db0.reshape(-1), device=DEV), N, 64, tol=1e-9, max_iter=60)
    op.close()
    got = res.delta.cpu().numpy().reshape(2, L2)
    print("bond SCF: oracle %d iterations, GPU %d, Delta_x %.6f, max |diff| %.2e" % (
        it_ref, res.iterations, cur[0].real.mean(), maxdiff(got, cur)))
    assert res.iterations == it_ref
    assert maxdiff(got, cur) < 1e-9
    assert np.max(np.abs(got[0] + got[1])) < 1e-9      # stays d-wave
