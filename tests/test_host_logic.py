"""Host-side pieces of the product that need no GPU."""
import numpy as np


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
