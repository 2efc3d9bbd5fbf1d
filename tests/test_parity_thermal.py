"""Finite-temperature gap weights and the electron density on the GPU
against the oracle's quadrature: coefficients, one gap update, the density
and its transpose, and a finite-temperature self-consistent solve."""
import numpy as np
import pytest
import torch

import oracle
import workloads as W
from tests.gpu_common import DEV, gpu_moments, maxdiff

pytestmark = pytest.mark.gpu


def _P():
    import paper_1007_1609_amd as P
    return P


@pytest.mark.parametrize("quantity,T,E_c,a,b", [
    ("gap", 0.1, 0.0, 6.0, 0.0),
    ("gap", 0.3, 2.0, 6.0, 0.0),      # cutoff inside the zone's reach
    ("gap", 0.02, 0.0, 5.3, 0.4),     # narrow zone, shifted spectrum
    ("gap", 0.0, 1.5, 6.0, -0.2),     # T = 0 through the same path
    ("gap", 2.0, 0.0, 6.0, 0.0),      # zone covers the whole interval
    ("density", 0.1, 0.0, 6.0, 0.0),
    ("density", 0.0, 0.0, 5.3, 0.4),
    ("density", 0.05, 0.0, 7.7, -0.3),
])
def test_coefficients_match_oracle_quadrature(quantity, T, E_c, a, b):
    P = _P()
    N = 256
    w = P.weights(a, b, T=T, E_c=E_c)
    q = P.CBDG_QTY_GAP if quantity == "gap" else P.CBDG_QTY_DENSITY
    got = P.sum_coefficients(w, N, q, DEV).cpu().numpy()
    ref = oracle.jackson(N) * oracle.thermal_coefficients(N, a, b, T, E_c, quantity)
    print("%s T=%g E_c=%g b=%g: max |diff| %.2e" % (quantity, T, E_c, b, maxdiff(got, ref)))
    assert maxdiff(got, ref) < 1e-12


def test_coefficients_at_the_workload_size():
    """N = 1024 with the 256x256 workload's rescaling, T = 0.01 (a narrow
    transition zone, thousands of panels)."""
    P = _P()
    N, a = 1024, 7.6876
    w = P.weights(a, 0.0, T=0.01)
    got = P.sum_coefficients(w, N, P.CBDG_QTY_GAP, DEV).cpu().numpy()
    ref = oracle.jackson(N) * oracle.thermal_coefficients(N, a, 0.0, 0.01)
    assert maxdiff(got, ref) < 1e-12


def test_zero_temperature_coefficients_equal_the_builtin_weights():
    """cbdg_gap_update with NULL coefficients (closed form) and with the
    quadrature path at T = 0 give the same Delta."""
    P = _P()
    rng = np.random.default_rng(3)
    mu = torch.as_tensor(rng.uniform(-1, 1, (50, 200)), device=DEV)
    d = torch.zeros(50, dtype=torch.float64, device=DEV)
    w = P.weights(5.0, 0.1, E_c=2.0)
    a_, _ = P.gap_update(mu, w, 2.0, d)
    c = P.sum_coefficients(w, 200, P.CBDG_QTY_GAP, DEV)
    b_, _ = P.gap_update(mu, w, 2.0, d, coeff=c)
    assert maxdiff(a_.cpu().numpy(), b_.cpu().numpy()) < 1e-13


@pytest.mark.parametrize("complex_", [False, True])
def test_finite_temperature_gap_update(complex_):
    P = _P()
    w = W.small_random(12, 10, N=200, seed=17, complex_=complex_, bond=False)
    op, g_ee, g_he = gpu_moments(w)
    a, b = op.bounds.a, op.bounds.b
    T = 0.15
    wt = op.weights(T=T)
    d0 = torch.as_tensor(w.delta, device=DEV)
    new, r = P.gap_update(torch.as_tensor(g_he, device=DEV), wt, w.U, d0)
    op.close()
    o_ee, o_he = oracle.workload_moments(w, a, b)
    ref = oracle.gap_map_thermal(o_he, w.U, a, b, T)
    if not complex_:
        ref = ref.real
    assert maxdiff(new.cpu().numpy(), ref) < 1e-10
    assert abs(float(r.item()) - np.max(np.abs(ref - w.delta))) < 1e-10


@pytest.mark.parametrize("T", [0.0, 0.1])
def test_density(T):
    P = _P()
    w = W.small_random(12, 10, N=200, seed=19)
    op, g_ee, _ = gpu_moments(w)
    a, b = op.bounds.a, op.bounds.b
    n = P.density(torch.as_tensor(g_ee, device=DEV), op.weights(T=T))
    op.close()
    o_ee, _ = oracle.workload_moments(w, a, b)
    ref = oracle.density(o_ee, a, b, T)
    print("density T=%g: max |diff| %.2e, mean n %.4f" % (T, maxdiff(n.cpu().numpy(), ref), ref.mean()))
    assert maxdiff(n.cpu().numpy(), ref) < 1e-10


def test_density_backward_and_gap_backward_at_finite_temperature():
    P = _P()
    N, T, a = 120, 0.2, 5.5
    w = P.weights(a, 0.0, T=T)
    cd = oracle.jackson(N) * oracle.thermal_coefficients(N, a, 0.0, T, quantity="density")
    cg = oracle.jackson(N) * oracle.thermal_coefficients(N, a, 0.0, T)
    dn = torch.as_tensor(np.random.default_rng(4).normal(size=30), device=DEV)
    dmu = P.density_backward(dn, N, w).cpu().numpy()
    assert maxdiff(dmu, 2.0 * np.outer(dn.cpu().numpy(), cd)) < 1e-12
    dmu_g, din = P.gap_update_backward(dn, N, w, 2.0, 0.7)
    assert maxdiff(dmu_g.cpu().numpy(), 0.7 * 1.0 * np.outer(dn.cpu().numpy(), cg)) < 1e-12


def test_finite_temperature_scf_matches_oracle():
    """Plain mixing at T = 0.1 on a 10x9 lattice with the same iteration count
    and fixed point as the oracle's loop."""
    P = _P()
    from paper_1007_1609_amd import scf
    w = W.small_random(10, 9, N=160, seed=23, U=2.4)
    _, _, a, b = oracle.workload_bounds(w)
    ref, it, r, _ = oracle.scf_plain(w, tol=1e-8, T=0.1, bounds=(a, b))
    op = P.Operator.from_workload(w, DEV, fixed=(a, b))
    res = scf.plain_mixing(op, w.U, torch.as_tensor(w.delta, device=DEV), w.N, 90, tol=1e-8, T=0.1)
    op.close()
    print("finite-T SCF: oracle %d iterations, GPU %d, max |diff| %.2e" % (it, res.iterations,
                                                                        maxdiff(res.delta.cpu().numpy(), ref)))
    assert res.iterations == it
    assert maxdiff(res.delta.cpu().numpy(), ref) < 1e-9
