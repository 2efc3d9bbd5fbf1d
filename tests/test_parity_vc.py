"""The vector-contiguous passes (lattices with Lx = 64 W, real operators with
uniform hopping, moment doubling): one wavefront per vector and row segment,
x-halo across lanes, every vector clipped to its own light cone.  Moments
against the oracle's eq. (ref2) recursion and against the GPU's direct
algorithm (vector-major kernels), across widths, boundary conditions,
ragged tiles, segment counts, start sites at the lattice's corners and
edges, odd and even N, and invalid or repeated start sites."""
import numpy as np
import pytest

import oracle
import workloads as W
from tests.gpu_common import TOL_MOMENT, gpu_moments, maxdiff

pytestmark = pytest.mark.gpu

DIRECT, DOUBLING = 1, 2
TOL_FP32 = 2e-5


def _run(w, N, tile, sites=None, precision=0, algorithm=DOUBLING):
    op, ee, he = gpu_moments(w, sites=sites, N=N, tile=tile, precision=precision, algorithm=algorithm)
    a, b = op.bounds.a, op.bounds.b
    op.close()
    return ee, he, a, b


@pytest.mark.parametrize("Lx,Ly,bcx,bcy,tile,N", [
    (64, 9, 0, 0, 37, 41),      # W = 1, ragged tiles
    (64, 70, 0, 0, 37, 64),     # four row segments per vector
    (64, 12, 1, 1, 100, 33),    # periodic both ways
    (64, 5, 1, 0, 64, 97),      # periodic x only; cones cover the lattice early
    (128, 7, 0, 1, 130, 40),    # W = 2, periodic y only, two tiles
    (128, 3, 1, 1, 200, 7),     # three rows, periodic: rows wrap within the cone
    (256, 5, 0, 0, 512, 64),    # W = 4, one tile
    (256, 4, 1, 0, 300, 3),     # N = 3: the first step and one more
    (256, 6, 0, 0, 1024, 8),    # N = 8: first step, one three-step pass
])
def test_vc_matches_oracle_and_direct(Lx, Ly, bcx, bcy, tile, N):
    w = W.small_random(Lx, Ly, N=N, seed=Lx + 3 * Ly + N, bc_x=bcx, bc_y=bcy)
    ee, he, a, b = _run(w, N, tile)
    d_ee, d_he, _, _ = _run(w, N, tile, algorithm=DIRECT)
    o_ee, o_he = oracle.workload_moments(w, a, b)
    print("%dx%d bc %d%d N=%d: |diff| vs oracle %.2e %.2e, vs direct %.2e" % (
        Lx, Ly, bcx, bcy, N, maxdiff(ee, o_ee), maxdiff(he, o_he), maxdiff(ee, d_ee)))
    assert maxdiff(ee, o_ee) <= TOL_MOMENT and maxdiff(he, o_he) <= TOL_MOMENT
    assert maxdiff(ee, d_ee) <= 1e-12 and maxdiff(he, d_he) <= 1e-12
    assert np.all(he[:, 0::2] == 0)


@pytest.mark.parametrize("Lx,Ly,bcx,bcy,N", [
    (64, 1, 0, 0, 30),      # one row: every halo row is outside the lattice
    (64, 2, 0, 0, 31),      # two rows
    (64, 3, 0, 1, 33),      # three rows, periodic in y (the fewest a periodic direction has)
    (128, 1, 1, 0, 24),     # one periodic row
    (256, 3, 0, 0, 16),
])
def test_vc_degenerate_lattices(Lx, Ly, bcx, bcy, N):
    w = W.small_random(Lx, Ly, N=N, seed=Lx + Ly + 7 * bcy, bc_x=bcx, bc_y=bcy)
    ee, he, a, b = _run(w, N, 100)
    d_ee, d_he, _, _ = _run(w, N, 100, algorithm=DIRECT)
    o_ee, o_he = oracle.workload_moments(w, a, b)
    assert maxdiff(ee, o_ee) <= TOL_MOMENT and maxdiff(he, o_he) <= TOL_MOMENT
    assert maxdiff(ee, d_ee) <= 1e-12 and maxdiff(he, d_he) <= 1e-12


@pytest.mark.parametrize("N", list(range(4, 22)) + [25, 26, 33, 34, 40])
def test_vc_every_split_of_the_steps(N):
    """N/2 steps taken as the first step, passes of several steps and the
    single steps left over, for every remainder of the pass length."""
    w = W.small_random(64, 11, N=N, seed=N)
    ee, he, a, b = _run(w, N, 128)
    o_ee, o_he = oracle.workload_moments(w, a, b)
    assert maxdiff(ee, o_ee) <= TOL_MOMENT and maxdiff(he, o_he) <= TOL_MOMENT


@pytest.mark.parametrize("bc", [0, 1])
def test_vc_corner_and_edge_start_sites(bc):
    """Light cones cut by the lattice edges (or wrapping around them)."""
    Lx, Ly = 128, 40
    w = W.small_random(Lx, Ly, N=120, seed=11 + bc, bc_x=bc, bc_y=bc)
    pts = [(0, 0), (Lx - 1, 0), (0, Ly - 1), (Lx - 1, Ly - 1), (1, 1), (63, 0), (64, 39), (2, 20), (127, 20),
           (60, 19), (65, 20)]
    sites = np.array([y * Lx + x for x, y in pts], np.int32)
    ee, he, a, b = _run(w, 120, 16, sites=sites)
    o_ee, o_he = oracle.workload_moments(w, a, b, sites=sites)
    assert maxdiff(ee, o_ee) <= TOL_MOMENT and maxdiff(he, o_he) <= TOL_MOMENT


def test_vc_invalid_and_repeated_sites():
    w = W.small_random(64, 10, N=50, seed=4)
    sites = np.array([5, -1, 640, 5, 639, 0, 64, 320], np.int32)
    ee, he, a, b = _run(w, 50, 8, sites=sites)
    assert np.all(np.isnan(ee[[1, 2]])) and np.all(np.isnan(he[[1, 2]]))
    ok = [0, 3, 4, 5, 6, 7]
    o_ee, o_he = oracle.workload_moments(w, a, b, sites=sites[ok])
    assert maxdiff(ee[ok], o_ee) <= TOL_MOMENT and maxdiff(he[ok], o_he) <= TOL_MOMENT
    assert np.array_equal(ee[0], ee[3]) and np.array_equal(he[0], he[3])


@pytest.mark.parametrize("Lx,Ly,bc,N", [(128, 6, 1, 64), (256, 5, 0, 64), (128, 40, 0, 64), (128, 9, 0, 23),
                                         (256, 7, 1, 35)])
def test_vc_fp32_recursion(Lx, Ly, bc, N):
    """FP32 vectors with FP64 sums (W = 2 and 4: two pairs per 16-byte access)."""
    w = W.small_random(Lx, Ly, N=N, seed=Lx + Ly, bc_x=bc, bc_y=bc)
    ee, he, a, b = _run(w, N, 256, precision=1)
    o_ee, o_he = oracle.workload_moments(w, a, b)
    assert maxdiff(ee, o_ee) <= TOL_FP32 and maxdiff(he, o_he) <= TOL_FP32


def test_native_runner_one_call():
    """The native runner (host code over the C ABI, no Python in the process)
    runs one moments call of a 128-wide lattice in both precisions and finds
    every moment bounded and mu_ee[0][0] = 1."""
    import os
    import subprocess
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    runner = os.path.join(root, "paper_1007_1609_amd", "cbdg_moments_run")
    for prec in ("fp64", "fp32"):
        r = subprocess.run([runner, "128", "40", "64", "256", "1000", prec, "16", "100"], capture_output=True,
                           text=True, timeout=120)
        print(r.stdout)
        assert r.returncode == 0, r.stderr
        assert "bounded yes" in r.stdout and "copy: 16 MiB" in r.stdout
