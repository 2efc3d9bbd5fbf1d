"""GPU parity at the launch geometry and sizes the benchmark runs.

The benchmark advances contiguous tiles of 1024 start sites (four lattice
rows of the 256x256 workload), so the light cone of a tile is active: early
passes cover a band of rows, later ones the whole lattice.  These tests run
those exact calls -- first, middle and last tile, FP64 by doubling and by the
direct recursion, the FP32-recursion form at N = 2048 -- and compare sampled
lanes element by element with the oracle's recursion of eq. (ref2), every
row against mu_0 = 1, |mu| <= 1 and particle-hole symmetry.  Further: the
complex workload at its real N = 2048 (complex128 and complex64), the
self-consistent Delta of the 256x256 workload and the Newton-Krylov Delta of
the differentiation workload put through the oracle's gap map of eq. (op1),
and the dLDOS(0)/dV gradient of the differentiation workload at full size.
"""
import os

import numpy as np
import pytest
import torch

import oracle
import workloads as W
from tests.gpu_common import DEV, TOL_MOMENT, maxdiff

pytestmark = pytest.mark.gpu

# lanes of a 1024-vector tile: the first and last lanes of the wavefronts
# and 256-lane chunks, the two sides of the first strip boundary (strips of
# 4 sites in x) and the tile's last lane
LANES = np.array([0, 1, 3, 4, 63, 64, 255, 256, 511, 512, 767, 768, 1022, 1023])
TILES = {"first": 0, "middle": 32768, "last": 64512}
TOL_FP32 = 2e-5


def _threads():
    return int(os.environ.get("OMP_NUM_THREADS", "0") or 0) or os.cpu_count() or 1


@pytest.fixture(scope="module")
def cfg1():
    """The 256x256 workload, its rescaling, and the oracle's moments of the
    sampled lanes of the three tiles at N = 2048 (the first 1024 of each row
    are the N = 1024 moments: the recursion does not depend on N)."""
    w = W.config1()
    _, _, a, b = oracle.workload_bounds(w)
    sites = np.concatenate([t0 + LANES for t0 in TILES.values()]).astype(np.int32)
    o_ee, o_he = oracle.workload_moments(w, a, b, sites=sites, N=2048, n_threads=_threads())
    return w, a, b, sites, o_ee, o_he


def _tile_moments(w, t0, N, prec, alg, fixed):
    import paper_1007_1609_amd as P
    op = P.Operator.from_workload(w, DEV, fixed=fixed)
    sites = torch.arange(t0, t0 + 1024, dtype=torch.int32, device=DEV)
    mu_ee, mu_he = P.chebyshev_moments(op, sites, N, 1024, prec, algorithm=alg)
    torch.cuda.synchronize()
    op.close()
    return mu_ee.cpu().numpy(), mu_he.cpu().numpy()


def _row_invariants(g_ee, g_he, tol):
    assert np.all(g_ee[:, 0] == 1.0) and np.all(g_he[:, 0] == 0.0)
    assert np.max(np.abs(g_ee)) <= 1.0 + tol and np.max(np.abs(g_he)) <= 1.0 + tol
    assert np.max(np.abs(g_he[:, 0::2])) < tol       # particle-hole symmetry, b = 0


@pytest.mark.parametrize("tile", list(TILES))
@pytest.mark.parametrize("alg", [0, 1], ids=["auto-doubling", "direct"])
def test_config1_benchmark_tiles_fp64(cfg1, tile, alg):
    w, a, b, sites, o_ee, o_he = cfg1
    k = list(TILES).index(tile)
    g_ee, g_he = _tile_moments(w, TILES[tile], 1024, 0, alg, (a, b))
    sel = slice(k * len(LANES), (k + 1) * len(LANES))
    e_ee = maxdiff(g_ee[LANES], o_ee[sel, :1024])
    e_he = maxdiff(g_he[LANES], o_he[sel, :1024])
    print("256x256 %s tile, alg %d: max |diff| ee %.2e he %.2e" % (tile, alg, e_ee, e_he))
    assert e_ee <= TOL_MOMENT and e_he <= TOL_MOMENT
    _row_invariants(g_ee, g_he, 1e-12)


@pytest.mark.parametrize("tile", list(TILES))
def test_config2_benchmark_tiles_fp32(cfg1, tile):
    w, a, b, sites, o_ee, o_he = cfg1
    k = list(TILES).index(tile)
    g_ee, g_he = _tile_moments(w, TILES[tile], 2048, 1, 0, (a, b))
    sel = slice(k * len(LANES), (k + 1) * len(LANES))
    e_ee = maxdiff(g_ee[LANES], o_ee[sel])
    e_he = maxdiff(g_he[LANES], o_he[sel])
    print("256x256 %s tile, FP32 recursion N=2048: max |diff| ee %.2e he %.2e" % (tile, e_ee, e_he))
    assert e_ee <= TOL_FP32 and e_he <= TOL_FP32
    _row_invariants(g_ee, g_he, TOL_FP32)


@pytest.mark.parametrize("prec,tol", [(0, TOL_MOMENT), (1, TOL_FP32)], ids=["complex128", "complex64"])
def test_config3_full_N_on_one_tile(prec, tol):
    """512x512 Peierls / d-wave lattice at N = 2048: the first 1024-site tile
    of the stride-8 grid, four lanes against the oracle."""
    import paper_1007_1609_amd as P
    w = W.config3()
    _, _, a, b = oracle.workload_bounds(w)
    op = P.Operator.from_workload(w, DEV, fixed=(a, b))
    sites = torch.as_tensor(w.start_sites[:1024], device=DEV)
    mu_ee, mu_he = P.chebyshev_moments(op, sites, w.N, 1024, prec)
    torch.cuda.synchronize()
    op.close()
    g_ee, g_he = mu_ee.cpu().numpy(), mu_he.cpu().numpy()
    lanes = [0, 511, 512, 1023]
    o_ee, o_he = oracle.workload_moments(w, a, b, sites=w.start_sites[lanes], n_threads=_threads())
    e_ee, e_he = maxdiff(g_ee[lanes], o_ee), maxdiff(g_he[lanes], o_he)
    print("512x512 complex N=2048 (%s): max |diff| ee %.2e he %.2e" % ("c64" if prec else "c128", e_ee, e_he))
    assert e_ee <= tol and e_he <= tol
    assert np.all(g_ee[:, 0] == 1.0)
    assert np.max(np.abs(g_ee)) <= 1.0 + tol and np.max(np.abs(g_he)) <= 1.0 + tol


def _sampled_sites(w, n, seed):
    """Impurity sites, the corners, and seeded random sites."""
    rng = np.random.default_rng(seed)
    imp = np.flatnonzero(w.eps)[: n // 4]
    corners = [0, w.Lx - 1, w.L2 - w.Lx, w.L2 - 1]
    rest = rng.choice(w.L2, n - len(imp) - len(corners), replace=False)
    return np.unique(np.concatenate([imp, corners, rest])).astype(np.int32)


def _oracle_map_residual(w, delta_star, sites, a, b):
    """max over sites of |F_oracle(Delta*)_i - Delta*_i| with the oracle's
    recursion and gap map of eq. (op1) on the operator built with Delta*."""
    _, o_he = oracle.workload_moments(w, a, b, sites=sites, delta=delta_star, n_threads=_threads())
    f = oracle.gap_map(o_he, w.U).real
    return float(np.max(np.abs(f - delta_star[sites])))


@pytest.mark.timeout(600)
def test_config1_self_consistent_delta_is_an_oracle_fixed_point():
    """The self-consistent Delta of the 256x256 workload (solved on the GPU to
    max|F(Delta) - Delta| < 1e-6 by the fastest schedule: Anderson mixing with
    FP32 recursion first and an N = 256 warm-up; only an FP64 evaluation
    below 1e-6 ends it) satisfies the oracle's gap map at 64 sampled sites."""
    import paper_1007_1609_amd as P
    from paper_1007_1609_amd import scf
    w = W.config1()
    _, _, a, b = oracle.workload_bounds(w)
    op = P.Operator.from_workload(w, DEV, fixed=(a, b))
    r = scf.anderson_mixing(op, w.U, torch.as_tensor(w.delta, device=DEV), w.N, w.tile, tol=1e-6,
                            max_iter=60, fast_precision=P.CBDG_FP32_ACC64, warmup_N=256,
                            callback=lambda it, res: print("iteration %d residual %.3e" % (it, res), flush=True))
    op.close()
    assert r.residual < 1e-6
    dstar = r.delta.cpu().numpy()
    sites = _sampled_sites(w, 64, 11)
    res = _oracle_map_residual(w, dstar, sites, a, b)
    print("256x256 Delta*: %d GPU evaluations, oracle-map residual %.2e at %d sites" % (
        r.iterations, res, len(sites)))
    assert res <= 2e-6


@pytest.mark.timeout(600)
@pytest.mark.parametrize("jv", ["vjp", "fd", "jacobian"])
def test_config4_newton_krylov_delta_is_an_oracle_fixed_point(jv):
    """Newton-Krylov on the full 128x128 differentiation workload (N = 512):
    its Delta satisfies the oracle's gap map at 64 sampled sites."""
    import paper_1007_1609_amd as P
    from paper_1007_1609_amd import scf
    w = W.config4()
    _, _, a, b = oracle.workload_bounds(w)
    op = P.Operator.from_workload(w, DEV, fixed=(a, b))
    r = scf.newton_krylov(op, w.U, torch.as_tensor(w.delta, device=DEV), w.N, w.tile, tol=1e-6, jv=jv)
    op.close()
    assert r.residual < 1e-6
    dstar = r.delta.cpu().numpy()
    sites = _sampled_sites(w, 64, 12)
    res = _oracle_map_residual(w, dstar, sites, a, b)
    print("128x128 Newton-Krylov (%s) Delta*: %s, oracle-map residual %.2e" % (jv, r.counts, res))
    assert res <= 2e-6


def test_config4_ldos_gradient_at_full_size():
    """dLDOS(E=0)/dV_i at the centre site of the 128x128 workload (N = 512)
    against the oracle's full-storage adjoint, relative 1e-10."""
    import paper_1007_1609_amd as P
    from paper_1007_1609_amd import autograd as AG
    w = W.config4()
    _, _, a, b = oracle.workload_bounds(w)
    s0 = w.notes["centre_site"]
    geom = AG.Geometry.of(w, a, b)
    eps = torch.as_tensor(w.eps, device=DEV).requires_grad_(True)
    delta = torch.as_tensor(w.delta, device=DEV)
    mu_ee, _ = AG.moments(eps, delta, geom, torch.tensor([s0], dtype=torch.int32, device=DEV), w.N, 64)
    AG.local_dos(mu_ee, torch.zeros(1, dtype=torch.float64, device=DEV), P.weights(a, b)).sum().backward()
    g = eps.grad.cpu().numpy()
    n = np.arange(w.N)
    wee = np.where(n == 0, 1.0, 2.0) * oracle.jackson(w.N) * np.cos(n * np.pi / 2) / (np.pi * a)
    oe, _ = oracle.moments_backward(oracle.workload_csr(w, a, b), [s0], w.N, wee[None, :],
                                    np.zeros((1, w.N)), n_threads=_threads())
    rel = float(np.max(np.abs(g - oe)) / np.max(np.abs(oe)))
    print("128x128 dLDOS(0)/dV rel err %.2e" % rel)
    assert rel < 1e-10


@pytest.mark.timeout(600)
def test_config4_jacobian_rows_at_full_size():
    """The whole Jacobian of the 128x128 workload's gap map (N = 512, all
    16384 start sites in tiles of 1024: the geometry of the differentiation
    benchmark's Newton solve), its cotangent the oracle's gap-map weights:
    rows at the centre, a corner, the last site and sampled sites against the
    oracle's full-storage adjoint of that one start site (1e-10 relative)."""
    import paper_1007_1609_amd as P
    w = W.config4()
    _, _, a, b = oracle.workload_bounds(w)
    cot = 0.5 * w.U * oracle.gap_weights(w.N)          # dF_k / dmu_he[k][n] of eq. (op1)
    op = P.Operator.from_workload(w, DEV, fixed=(a, b))
    d_mu = torch.as_tensor(np.ascontiguousarray(np.broadcast_to(cot, (w.L2, w.N))), device=DEV)
    s = torch.arange(w.L2, dtype=torch.int32, device=DEV)
    _, J = P.chebyshev_moments_jacobian(op, s, w.N, w.tile, None, d_mu)
    rows = np.unique(np.concatenate([[w.notes["centre_site"], 0, w.L2 - 1, 1023, 1024],
                                     _sampled_sites(w, 8, 21)])).astype(np.int64)
    Jr = J[torch.as_tensor(rows, device=DEV)].cpu().numpy()
    del J
    op.close()
    csr = oracle.workload_csr(w, a, b)
    for k, site in enumerate(rows):
        _, od = oracle.moments_backward(csr, [int(site)], w.N, np.zeros((1, w.N)), cot[None, :],
                                        n_threads=_threads())
        err = float(np.max(np.abs(Jr[k] - od)) / np.max(np.abs(od)))
        print("128x128 Jacobian row %d: rel err %.2e" % (site, err))
        assert err < 1e-10, site
