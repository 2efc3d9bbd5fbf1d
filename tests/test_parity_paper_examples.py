"""The paper's two example geometries at full size: sampled start sites
against the oracle, and the Lorentz-kernel LDOS of the first example."""
import numpy as np
import pytest
import torch

import oracle
import workloads as W
from tests.gpu_common import DEV, TOL_MOMENT, gpu_moments, maxdiff

pytestmark = pytest.mark.gpu


def test_sn_surface_moments_and_lorentz_ldos():
    """400x500 (periodic in y), two surface start vectors, N = 600, against
    the oracle; LDOS with the Lorentz kernel at the paper's constant
    broadening eps = 0.001t (lambda = N eps / a)."""
    import paper_1007_1609_amd as P
    w = W.sn_surface(N=600)
    sites = w.start_sites[[0, 63]]
    op, g_ee, g_he = gpu_moments(w, sites=sites, tile=2)
    a, b = op.bounds.a, op.bounds.b
    lam = w.N * 0.001 / a
    E = torch.as_tensor(w.energies, device=DEV)
    ld = P.ldos(torch.as_tensor(g_ee, device=DEV), op.weights("lorentz", lam=lam), E).cpu().numpy()
    op.close()
    o_ee, o_he = oracle.workload_moments(w, a, b, sites=sites)
    assert maxdiff(g_ee, o_ee) <= TOL_MOMENT and maxdiff(g_he, o_he) <= TOL_MOMENT
    ref = oracle.ldos(o_ee, w.energies, a, b, kernel="lorentz", lam=lam)
    assert maxdiff(ld, ref) <= 1e-10 * np.max(np.abs(ref))
    # translation invariance along the periodic surface
    assert maxdiff(g_ee[0], g_ee[1]) < 1e-12


@pytest.mark.parametrize("sc,imp", [(True, True), (False, True), (True, False)])
def test_sns_impurity_sampled_sites(sc, imp):
    w = W.sns_impurity(N=512, superconducting=sc, impurity=imp)
    pick = w.start_sites[[0, 220, 440]]       # corner of the window, the impurity, far corner
    op, g_ee, g_he = gpu_moments(w, sites=pick, tile=3)
    a, b = op.bounds.a, op.bounds.b
    op.close()
    o_ee, o_he = oracle.workload_moments(w, a, b, sites=pick)
    assert maxdiff(g_ee, o_ee) <= TOL_MOMENT and maxdiff(g_he, o_he) <= TOL_MOMENT
    if not sc:
        assert np.max(np.abs(g_he)) == 0.0   # a normal metal has no anomalous moments


@pytest.mark.parametrize("kernel", ["jackson", "lorentz"])
def test_ldos_beyond_one_lds_chunk(kernel):
    """N = 5000 (three LDS chunks of the recurrence) and 300 energies (two
    thread blocks of energies) against the oracle's dense weights."""
    import paper_1007_1609_amd as P
    rng = np.random.default_rng(8)
    mu = rng.uniform(-1, 1, (3, 5000)) / np.arange(1, 5001) ** 0.5
    a, b, lam = 5.0, 0.2, 4.0
    E = np.linspace(-4.5, 4.9, 300)
    w = P.weights(a, b, kernel, lam=lam)
    got = P.ldos(torch.as_tensor(mu, device=DEV), w, torch.as_tensor(E, device=DEV)).cpu().numpy()
    ref = oracle.ldos(mu, E, a, b, kernel=kernel, lam=lam)
    assert maxdiff(got, ref) <= 1e-10 * np.max(np.abs(ref))
