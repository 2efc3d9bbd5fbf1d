"""Light-cone clipping of the recursion steps (a_n vanishes farther than n
sites from the tile's start sites, so those strips and rows are skipped):
tiles whose bounding box is small, sits in a corner, follows a tile with a
larger box, mixes in invalid sites, or lies on a periodic direction, all
against the oracle with both moment algorithms."""
import numpy as np
import pytest

import oracle
import workloads as W
from tests.gpu_common import TOL_MOMENT, gpu_moments, maxdiff

pytestmark = pytest.mark.gpu

ALGS = [1, 2]  # direct, doubling


def _check(w, sites, tile, alg, N=None):
    op, g_ee, g_he = gpu_moments(w, sites=sites, N=N, tile=tile, algorithm=alg)
    a, b = op.bounds.a, op.bounds.b
    op.close()
    valid = (sites >= 0) & (sites < w.L2)
    o_ee, o_he = oracle.workload_moments(w, a, b, sites=sites[valid], N=N)
    assert maxdiff(g_ee[valid], o_ee) <= TOL_MOMENT
    assert maxdiff(g_he[valid], o_he) <= TOL_MOMENT
    assert np.all(np.isnan(g_ee[~valid]))


def _block(Lx, x0, x1, y0, y1):
    return np.array([y * Lx + x for y in range(y0, y1) for x in range(x0, x1)], dtype=np.int32)


@pytest.mark.parametrize("alg", ALGS)
def test_corner_tile_on_a_long_lattice(alg):
    # 48x80, sites in a 5x3 corner block: the cone covers the lattice only
    # after ~75 steps (direct) or ~40 steps (doubling) of N = 96
    w = W.small_random(48, 80, N=96, seed=21)
    _check(w, _block(48, 0, 5, 0, 3), 64, alg)


@pytest.mark.parametrize("alg", ALGS)
def test_small_tile_after_large_tiles(alg):
    # tile 1: spread over the lattice; tile 2: one site far from everything;
    # tile 3: a block at the other end -- stale values of earlier tiles must
    # not leak into the skipped rows
    w = W.small_random(40, 64, N=80, seed=22)
    spread = np.arange(0, w.L2, 97, dtype=np.int32)[:26]
    one = np.array([63 * 40 + 39], dtype=np.int32)
    blk = _block(40, 30, 36, 60, 64)[:26]
    sites = np.concatenate([spread, np.repeat(one, 26), blk])
    _check(w, sites, 26, alg)


@pytest.mark.parametrize("alg", ALGS)
def test_column_of_sites_clips_strips(alg):
    # every row, x in 0..2: the box is narrow in x, full in y
    w = W.small_random(64, 24, N=64, seed=23)
    _check(w, _block(64, 0, 3, 0, 24), 128, alg)


@pytest.mark.parametrize("alg", ALGS)
@pytest.mark.parametrize("bc", [dict(bc_x=W.PERIODIC), dict(bc_y=W.PERIODIC),
                                dict(bc_x=W.PERIODIC, bc_y=W.PERIODIC)])
def test_periodic_directions_are_not_clipped(alg, bc):
    w = W.small_random(32, 40, N=72, seed=24, **bc)
    _check(w, _block(32, 0, 4, 0, 4), 16, alg)


@pytest.mark.parametrize("alg", ALGS)
def test_invalid_sites_do_not_widen_or_empty_the_box(alg):
    w = W.small_random(32, 48, N=64, seed=25)
    sites = np.concatenate([_block(32, 10, 14, 20, 22), np.array([-5, w.L2, 10 ** 6], np.int32)])
    _check(w, sites, 64, alg)
    # a tile of invalid sites only, followed by a valid corner tile
    sites = np.concatenate([np.full(8, -1, np.int32), _block(32, 0, 2, 0, 4)])
    _check(w, sites, 8, alg)


@pytest.mark.parametrize("alg", ALGS)
def test_complex_bond_operator_corner(alg):
    w = W.small_random(36, 44, N=70, seed=26, complex_=True, bond=True, flux=0.2)
    _check(w, _block(36, 30, 36, 40, 44), 32, alg)


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("alg", ALGS)
@pytest.mark.parametrize("Lx,Ly,bc,block,tile,N", [
    # tiles of 128 vectors or fewer: two steps per launch
    (48, 80, {}, (0, 5, 0, 3), 64, 97),                          # corner tile, light cone
    (36, 40, dict(bc_x=W.PERIODIC, bc_y=W.PERIODIC), (0, 4, 0, 4), 16, 64),
    (64, 24, {}, (0, 3, 0, 24), 128, 66),                        # narrow column
    # larger tiles: three steps per launch, then a pair and/or a single step
    (48, 80, {}, (0, 16, 0, 10), 160, 97),                       # corner block, light cone
    (36, 40, dict(bc_x=W.PERIODIC, bc_y=W.PERIODIC), (0, 12, 0, 12), 144, 64),
    (64, 24, {}, (0, 8, 0, 24), 192, 66),                        # full height, narrow in x
    (13, 37, {}, (0, 13, 0, 37), 200, 65),                       # ragged: tiles 200, 200, 81
])
def test_multi_step_passes(prec, alg, Lx, Ly, bc, block, tile, N):
    """Real operators with uniform hopping take several recursion steps per
    launch (three for tiles of more than 128 vectors, else two, and a pair
    and/or a single step for the remainder): moments within 1e-10 (FP64) or
    2e-5 (FP32 recursion) of the FP64 oracle."""
    w = W.small_random(Lx, Ly, N=N, seed=Lx + Ly + N, **bc)
    sites = _block(Lx, *block)
    op, g_ee, g_he = gpu_moments(w, sites=sites, tile=tile, precision=prec, algorithm=alg)
    a, b = op.bounds.a, op.bounds.b
    op.close()
    o_ee, o_he = oracle.workload_moments(w, a, b, sites=sites)
    e = max(maxdiff(g_ee, o_ee), maxdiff(g_he, o_he))
    print("prec %d %dx%d N=%d alg=%d tile=%d: max error %.2e" % (prec, Lx, Ly, N, alg, tile, e))
    assert e < (TOL_MOMENT if prec == 0 else 2e-5)
