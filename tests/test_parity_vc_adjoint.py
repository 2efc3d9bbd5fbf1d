"""Reverse passes without checkpoints (ckpt_stride = -1): the forward vectors
regenerated backwards beside the transposed recursion, in the
vector-contiguous layout.  Against the CPU oracle's full-storage adjoint and
against the checkpointed reverse pass, across widths, boundary conditions,
ragged tiles, row segments, pass splits (M below, at and above the pass
length, every remainder), invalid and repeated start sites, and at the
differentiation workload's size."""
import numpy as np
import pytest
import torch

import oracle
import workloads as W
from tests.gpu_common import DEV

pytestmark = pytest.mark.gpu

DOUBLING = 2
REV = -1


def _P():
    import paper_1007_1609_amd as P
    return P


def _rel(x, ref):
    return float(np.max(np.abs(np.asarray(x) - np.asarray(ref))) / max(np.max(np.abs(ref)), 1e-300))


def _backward(w, N, dee, dhe, tile, ckpt, sites=None):
    P = _P()
    op = P.Operator.from_workload(w, DEV)
    s = torch.as_tensor(w.start_sites if sites is None else sites, dtype=torch.int32, device=DEV)
    ge, gd = P.chebyshev_moments_backward(
        op, s, N, tile, None if dee is None else torch.as_tensor(dee, device=DEV),
        None if dhe is None else torch.as_tensor(dhe, device=DEV), ckpt, algorithm=DOUBLING)
    torch.cuda.synchronize()
    a, b = op.bounds.a, op.bounds.b
    op.close()
    return ge.cpu().numpy(), gd.cpu().numpy(), a, b


@pytest.mark.parametrize("Lx,Ly,bcx,bcy,N,tile", [
    (64, 9, 0, 0, 24, 37),      # W = 1, ragged tiles, M = 12 (three full passes)
    (64, 6, 1, 1, 33, 100),     # periodic both ways, odd N, M = 16
    (64, 70, 0, 0, 20, 37),     # four row segments per vector
    (128, 7, 0, 1, 41, 300),    # W = 2, periodic y, M = 20, two tiles
    (128, 5, 1, 0, 18, 64),     # periodic x, M = 9 (two full passes and one level)
    (256, 4, 0, 0, 27, 512),    # W = 4 (two levels per pass), M = 13: six full passes and one level
    (256, 5, 1, 1, 20, 300),    # W = 4, periodic both ways, M = 10: full passes only, two tiles
    (256, 40, 0, 0, 22, 64),    # W = 4, several row segments per vector, M = 11
    (128, 3, 1, 1, 14, 200),    # three rows, periodic: rows wrap within a pass
])
def test_reverse_passes_match_oracle_and_checkpoints(Lx, Ly, bcx, bcy, N, tile):
    w = W.small_random(Lx, Ly, N=N, seed=Lx + 3 * Ly + N, bc_x=bcx, bc_y=bcy)
    rng = np.random.default_rng(N + Ly)
    n = len(w.start_sites)
    dee, dhe = rng.normal(size=(n, N)), rng.normal(size=(n, N))
    ge, gd, a, b = _backward(w, N, dee, dhe, tile, REV)
    ce, cd, _, _ = _backward(w, N, dee, dhe, tile, 0)
    oe, od = oracle.moments_backward(oracle.workload_csr(w, a, b), w.start_sites, N, dee, dhe)
    print("%dx%d bc %d%d N=%d: rel err vs oracle %.2e %.2e, vs checkpoints %.2e %.2e" % (
        Lx, Ly, bcx, bcy, N, _rel(ge, oe), _rel(gd, od), _rel(ge, ce), _rel(gd, cd)))
    assert _rel(ge, oe) < 1e-10 and _rel(gd, od) < 1e-10
    assert _rel(ge, ce) < 1e-11 and _rel(gd, cd) < 1e-11


@pytest.mark.parametrize("N", [3, 4, 5, 6, 7, 8, 9, 10, 11, 12, 13, 16, 17, 19])
def test_every_split_of_the_reverse_sweep(N):
    """M = N/2 levels as full passes of six (64-wide lattice) and one shorter
    last pass, for every remainder, including M below the pass length."""
    w = W.small_random(64, 8, N=N, seed=N)
    rng = np.random.default_rng(3 * N)
    n = len(w.start_sites)
    dee, dhe = rng.normal(size=(n, N)), rng.normal(size=(n, N))
    ge, gd, a, b = _backward(w, N, dee, dhe, 128, REV)
    oe, od = oracle.moments_backward(oracle.workload_csr(w, a, b), w.start_sites, N, dee, dhe)
    assert _rel(ge, oe) < 1e-10 and _rel(gd, od) < 1e-10


@pytest.mark.parametrize("which", ["ee", "he"])
def test_one_cotangent_only(which):
    N = 22
    w = W.small_random(128, 6, N=N, seed=5)
    rng = np.random.default_rng(7)
    n = len(w.start_sites)
    d = rng.normal(size=(n, N))
    dee, dhe = (d, None) if which == "ee" else (None, d)
    ge, gd, a, b = _backward(w, N, dee, dhe, 256, REV)
    z = np.zeros((n, N))
    oe, od = oracle.moments_backward(oracle.workload_csr(w, a, b), w.start_sites, N,
                                     d if which == "ee" else z, d if which == "he" else z)
    assert _rel(ge, oe) < 1e-10 and _rel(gd, od) < 1e-10


def test_invalid_and_repeated_sites():
    N = 20
    w = W.small_random(64, 10, N=N, seed=4)
    sites = np.array([5, -1, 640, 5, 639, 0, 64, 320], np.int32)
    rng = np.random.default_rng(2)
    dee, dhe = rng.normal(size=(len(sites), N)), rng.normal(size=(len(sites), N))
    ge, gd, a, b = _backward(w, N, dee, dhe, 8, REV, sites=sites)
    ok = [0, 3, 4, 5, 6, 7]
    oe, od = oracle.moments_backward(oracle.workload_csr(w, a, b), sites[ok], N, dee[ok], dhe[ok])
    assert _rel(ge, oe) < 1e-10 and _rel(gd, od) < 1e-10


def test_gradients_accumulate_into_the_outputs():
    P = _P()
    N = 16
    w = W.small_random(64, 6, N=N, seed=9)
    op = P.Operator.from_workload(w, DEV)
    s = torch.as_tensor(w.start_sites, dtype=torch.int32, device=DEV)
    rng = np.random.default_rng(4)
    dee = torch.as_tensor(rng.normal(size=(len(w.start_sites), N)), device=DEV)
    ge0 = torch.full((op.L2,), 0.5, dtype=torch.float64, device=DEV)
    gd0 = torch.full((op.L2,), -0.25, dtype=torch.float64, device=DEV)
    ge, gd = P.chebyshev_moments_backward(op, s, N, 64, dee, None, REV, grad_eps=ge0.clone(),
                                          grad_delta=gd0.clone(), algorithm=DOUBLING)
    g1, g2 = P.chebyshev_moments_backward(op, s, N, 64, dee, None, REV, algorithm=DOUBLING)
    torch.cuda.synchronize()
    op.close()
    assert torch.equal(ge - ge0, g1) or float((ge - ge0 - g1).abs().max()) < 1e-15
    assert float((gd - gd0 - g2).abs().max()) < 1e-15


def test_unsupported_operators_are_rejected():
    P = _P()
    w = W.small_random(12, 10, N=16, seed=1)   # Lx not a multiple of 64
    op = P.Operator.from_workload(w, DEV)
    s = torch.as_tensor(w.start_sites, dtype=torch.int32, device=DEV)
    dee = torch.zeros((len(w.start_sites), 16), dtype=torch.float64, device=DEV)
    with pytest.raises(Exception):
        P.chebyshev_moments_backward(op, s, 16, 64, dee, None, REV, algorithm=DOUBLING)
    assert not P.reversible_supported(op, 64, 16)
    op.close()


def test_two_moments_take_the_direct_algorithm_and_are_rejected():
    """N = 2 has no doubling step (the automatic choice is the direct
    algorithm), so the reverse passes without checkpoints refuse it with
    EUNSUPPORTED and the automatic choice of the autograd path falls back
    to checkpoints."""
    P = _P()
    w = W.small_random(64, 8, N=2, seed=2)
    op = P.Operator.from_workload(w, DEV)
    s = torch.as_tensor(w.start_sites, dtype=torch.int32, device=DEV)
    dee = torch.ones((len(w.start_sites), 2), dtype=torch.float64, device=DEV)
    assert P.reversible_supported(op, 64, 4)
    assert not P.reversible_supported(op, 64, 2)
    with pytest.raises(P.CbdgError) as e:
        P.chebyshev_moments_backward(op, s, 2, 64, dee, None, REV)
    assert "EUNSUPPORTED" in str(e.value)
    op.close()


def test_differentiation_workload_matches_checkpoints():
    """128x128, N = 512, one 1024-vector tile (the launch geometry of the
    differentiation benchmark) plus a ragged one: the regenerated vectors
    keep the gradient within 1e-9 of the checkpointed reverse pass."""
    P = _P()
    w = W.config4()
    N = w.N
    op = P.Operator.from_workload(w, DEV)
    sites = torch.arange(0, 1024 + 300, dtype=torch.int32, device=DEV) * 7 % w.L2
    rng = np.random.default_rng(11)
    dee = torch.as_tensor(rng.normal(size=(sites.numel(), N)) / N, device=DEV)
    dhe = torch.as_tensor(rng.normal(size=(sites.numel(), N)) / N, device=DEV)
    ge, gd = P.chebyshev_moments_backward(op, sites, N, 1024, dee, dhe, REV, algorithm=DOUBLING)
    ce, cd = P.chebyshev_moments_backward(op, sites, N, 1024, dee, dhe, 0, algorithm=DOUBLING)
    torch.cuda.synchronize()
    op.close()
    re = float((ge - ce).abs().max() / ce.abs().max())
    rd = float((gd - cd).abs().max() / cd.abs().max())
    print("128x128 N=%d: rel diff eps %.2e delta %.2e" % (N, re, rd))
    assert re < 1e-9 and rd < 1e-9


def test_benchmark_lattice_matches_checkpoints():
    """256x256, N = 1024 (three levels per reverse pass at W = 4): one
    contiguous 1024-site tile of the benchmark's geometry (its light cones
    grow from a four-row band) and a ragged tile of spread sites; the
    regenerated vectors keep the gradient within 1e-9 of the checkpointed
    reverse pass over 512 reverse levels."""
    P = _P()
    w = W.config1()
    N = w.N
    op = P.Operator.from_workload(w, DEV)
    sites = torch.cat([torch.arange(32768, 32768 + 1024, dtype=torch.int32),
                       torch.arange(0, 200, dtype=torch.int32) * 331 % w.L2]).to(DEV)
    rng = np.random.default_rng(12)
    dee = torch.as_tensor(rng.normal(size=(sites.numel(), N)) / N, device=DEV)
    dhe = torch.as_tensor(rng.normal(size=(sites.numel(), N)) / N, device=DEV)
    ge, gd = P.chebyshev_moments_backward(op, sites, N, 1024, dee, dhe, REV, algorithm=DOUBLING)
    ce, cd = P.chebyshev_moments_backward(op, sites, N, 1024, dee, dhe, 0, algorithm=DOUBLING)
    torch.cuda.synchronize()
    op.close()
    re = float((ge - ce).abs().max() / ce.abs().max())
    rd = float((gd - cd).abs().max() / cd.abs().max())
    print("256x256 N=%d: rel diff eps %.2e delta %.2e" % (N, re, rd))
    assert re < 1e-9 and rd < 1e-9
