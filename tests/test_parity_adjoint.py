"""GPU reverse mode vs the CPU oracle's full-storage adjoint, vs finite
differences of the GPU forward, across checkpoint strides and tile splits;
autograd wrappers; Newton-Krylov vs plain mixing."""
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


def _rel(x, ref):
    return float(np.max(np.abs(np.asarray(x) - np.asarray(ref))) / max(np.max(np.abs(ref)), 1e-300))


def _gpu_backward(w, N, dmu_ee, dmu_he, tile, ckpt=0, sites=None, algorithm=0, fixed=None):
    P = _P()
    op = P.Operator.from_workload(w, DEV, fixed=fixed)
    s = torch.as_tensor(w.start_sites if sites is None else sites, dtype=torch.int32, device=DEV)
    ge, gd = P.chebyshev_moments_backward(
        op, s, N, tile, None if dmu_ee is None else torch.as_tensor(dmu_ee, device=DEV),
        None if dmu_he is None else torch.as_tensor(dmu_he, device=DEV), ckpt, algorithm=algorithm)
    torch.cuda.synchronize()
    a, b = op.bounds.a, op.bounds.b
    op.close()
    return ge.cpu().numpy(), gd.cpu().numpy(), a, b


ALGS = [1, 2]  # direct adjoint, adjoint of the doubling formulas


@pytest.mark.parametrize("alg", ALGS)
@pytest.mark.parametrize("Lx,Ly,N,tile,ckpt,bc", [
    (12, 10, 40, 64, 0, 0),      # default stride, one tile
    (12, 10, 40, 37, 3, 0),      # ragged tiles, stride 3
    (10, 9, 33, 128, 1, 0),      # stride 1 (every vector a checkpoint), W = 2 strips
    (9, 13, 25, 50, 25, 0),      # one segment, odd width (W = 1)
    (8, 8, 31, 64, 4, 1),        # periodic
    (16, 20, 64, 300, 0, 0),     # several 256-lane chunks of one tile
    (12, 14, 41, 64, 2, 0),      # stride 2 (pairs only), odd N
    (12, 14, 44, 64, 5, 0),      # even N, ragged last segment
    (16, 20, 64, 200, 6, 0),     # three-step checkpointing forward (stride 6), ragged tiles
    (14, 12, 47, 168, 3, 1),     # three-step forward, stride 3, periodic
])
def test_backward_matches_oracle(Lx, Ly, N, tile, ckpt, bc, alg):
    w = W.small_random(Lx, Ly, N=N, seed=Lx + Ly + N, bc_x=bc, bc_y=bc)
    rng = np.random.default_rng(N)
    n = len(w.start_sites)
    dee, dhe = rng.normal(size=(n, N)), rng.normal(size=(n, N))
    ge, gd, a, b = _gpu_backward(w, N, dee, dhe, tile, ckpt, algorithm=alg)
    H = oracle.workload_csr(w, a, b)
    oe, od = oracle.moments_backward(H, w.start_sites, N, dee, dhe)
    print("backward %dx%d N=%d tile=%d k=%d alg=%d: rel err eps %.2e delta %.2e" % (
        Lx, Ly, N, tile, ckpt, alg, _rel(ge, oe), _rel(gd, od)))
    assert _rel(ge, oe) < 1e-10 and _rel(gd, od) < 1e-10


@pytest.mark.parametrize("alg", ALGS)
@pytest.mark.parametrize("N", [2, 3, 4, 5])
def test_backward_few_moments(N, alg):
    w = W.small_random(6, 5, N=N, seed=3)
    rng = np.random.default_rng(1)
    n = len(w.start_sites)
    dee, dhe = rng.normal(size=(n, N)), rng.normal(size=(n, N))
    ge, gd, a, b = _gpu_backward(w, N, dee, dhe, 64, algorithm=alg)
    oe, od = oracle.moments_backward(oracle.workload_csr(w, a, b), w.start_sites, N, dee, dhe)
    assert _rel(ge, oe) < 1e-12 and _rel(gd, od) < 1e-12


@pytest.mark.parametrize("alg", ALGS)
@pytest.mark.parametrize("which", ["ee", "he"])
def test_only_one_cotangent(which, alg):
    w = W.small_random(8, 7, N=30, seed=4)
    n = len(w.start_sites)
    g = np.random.default_rng(2).normal(size=(n, 30))
    z = np.zeros((n, 30))
    args = (g, None) if which == "ee" else (None, g)
    ge, gd, a, b = _gpu_backward(w, 30, *args, 64, algorithm=alg)
    oargs = (g, z) if which == "ee" else (z, g)
    oe, od = oracle.moments_backward(oracle.workload_csr(w, a, b), w.start_sites, 30, *oargs)
    assert _rel(ge, oe) < 1e-10 and _rel(gd, od) < 1e-10


@pytest.mark.parametrize("tile", [64, 144])
@pytest.mark.parametrize("alg", ALGS)
def test_checkpoint_strides_give_identical_bits(alg, tile):
    """Every kernel that applies Ht rounds alike, so the gradients do not
    depend on the checkpoint stride -- nor, with 144-vector tiles, on whether
    the checkpointing forward takes three steps per launch (strides that are
    multiples of 3) or two."""
    w = W.small_random(12, 12, N=50, seed=6)
    rng = np.random.default_rng(3)
    n = len(w.start_sites)
    dee, dhe = rng.normal(size=(n, 50)), rng.normal(size=(n, 50))
    ref = _gpu_backward(w, 50, dee, dhe, tile, 1, algorithm=alg)
    for k in (2, 3, 6, 7, 25, 26, 49, 50):
        got = _gpu_backward(w, 50, dee, dhe, tile, k, algorithm=alg)
        assert np.array_equal(got[0], ref[0]) and np.array_equal(got[1], ref[1]), k


def test_doubling_adjoint_needs_centred_rescaling():
    P = _P()
    w = W.small_random(8, 8, N=20, seed=7)
    rng = np.random.default_rng(5)
    n = len(w.start_sites)
    dee, dhe = rng.normal(size=(n, 20)), rng.normal(size=(n, 20))
    with pytest.raises(P.CbdgError) as e:
        _gpu_backward(w, 20, dee, dhe, 64, algorithm=2, fixed=(7.5, 0.2))
    assert e.value.code == -1
    # AUTO falls back to the direct adjoint and matches the oracle
    ge, gd, a, b = _gpu_backward(w, 20, dee, dhe, 64, algorithm=0, fixed=(7.5, 0.2))
    oe, od = oracle.moments_backward(oracle.workload_csr(w, 7.5, 0.2), w.start_sites, 20, dee, dhe)
    assert _rel(ge, oe) < 1e-10 and _rel(gd, od) < 1e-10


def test_backward_accumulates_into_outputs():
    P = _P()
    w = W.small_random(8, 8, N=20, seed=8)
    op = P.Operator.from_workload(w, DEV)
    s = torch.as_tensor(w.start_sites, device=DEV)
    dhe = torch.ones((w.L2, 20), dtype=torch.float64, device=DEV)
    g1 = P.chebyshev_moments_backward(op, s, 20, 64, None, dhe)
    ge = torch.full((w.L2,), 3.0, dtype=torch.float64, device=DEV)
    gd = torch.zeros(w.L2, dtype=torch.float64, device=DEV)
    P.chebyshev_moments_backward(op, s, 20, 64, None, dhe, grad_eps=ge, grad_delta=gd)
    op.close()
    assert maxdiff(ge.cpu().numpy() - 3.0, g1[0].cpu().numpy()) < 1e-13


def test_complex_operator_is_unsupported():
    P = _P()
    w = W.small_random(6, 6, N=10, seed=1, complex_=True)
    op = P.Operator.from_workload(w, DEV)
    with pytest.raises(P.CbdgError) as e:
        P.chebyshev_moments_backward(op, torch.as_tensor(w.start_sites, device=DEV), 10, 64, None,
                                     torch.ones((w.L2, 10), dtype=torch.float64, device=DEV))
    op.close()
    assert e.value.code == -5


# ----------------------------------------------------------------- autograd
def _small_cfg4(L=24, N=160, n_imp=9):
    w = W.config4(L=L, N=N, tile=256)
    rng = np.random.default_rng(4)
    eps = np.zeros(L * L)
    eps[rng.choice(L * L, n_imp, replace=False)] = rng.uniform(0, 4, n_imp)
    return w.with_(eps=eps)


def _sum_delta_and_grad(w, eps_np, a, b, grad=True):
    P = _P()
    from paper_1007_1609_amd import autograd as AG
    geom = AG.Geometry.of(w, a, b)
    eps = torch.as_tensor(eps_np, device=DEV).requires_grad_(grad)
    delta = torch.as_tensor(w.delta, device=DEV).requires_grad_(grad)
    sites = torch.as_tensor(w.start_sites, device=DEV)
    with torch.set_grad_enabled(grad):
        mu_ee, mu_he = AG.moments(eps, delta, geom, sites, w.N, w.tile)
        new = AG.gap_map(mu_he, delta, w.U, P.weights(a, b))
        loss = new.sum()
    if not grad:
        return float(loss.item())
    loss.backward()
    return float(loss.item()), eps.grad.cpu().numpy(), delta.grad.cpu().numpy()


def test_autograd_sum_delta_matches_oracle_and_fd():
    w = _small_cfg4()
    _, _, a, b = oracle.workload_bounds(w)
    L0, g_eps, g_delta = _sum_delta_and_grad(w, w.eps, a, b)
    # oracle: d/deps of sum_i (U/2) sum_n g_n c_n mu_he_n(i)
    N = w.N
    wg = 0.5 * w.U * oracle.gap_weights(N, a=a, b=b)
    H = oracle.workload_csr(w, a, b)
    oe, od = oracle.moments_backward(H, w.start_sites, N, np.zeros((w.L2, N)), np.tile(wg, (w.L2, 1)))
    print("dSum(Delta)/deps rel err vs oracle %.2e" % _rel(g_eps, oe))
    assert _rel(g_eps, oe) < 1e-10
    # delta.grad also carries the direct path through delta_in (alpha = 1 -> none)
    assert _rel(g_delta, od) < 1e-10
    # Richardson finite differences of the GPU forward at three sites
    imp = np.flatnonzero(w.eps)[:2].tolist() + [w.L2 // 2 + 3]
    for j in imp:
        def f(h):
            e = w.eps.copy()
            e[j] += h
            return _sum_delta_and_grad(w, e, a, b, grad=False)
        d1 = (f(1e-3) - f(-1e-3)) / 2e-3
        d2 = (f(5e-4) - f(-5e-4)) / 1e-3
        rich = (4 * d2 - d1) / 3
        assert abs(g_eps[j] - rich) <= 1e-6 * max(1.0, np.max(np.abs(g_eps))), j


def test_autograd_second_backward_through_a_retained_graph():
    # the moments' operator lives as long as the graph: a second backward
    # through a retained graph runs the reverse pass again and adds the same
    # gradient
    P = _P()
    from paper_1007_1609_amd import autograd as AG
    w = _small_cfg4(L=16, N=64)
    _, _, a, b = oracle.workload_bounds(w)
    geom = AG.Geometry.of(w, a, b)
    eps = torch.as_tensor(w.eps, device=DEV).requires_grad_(True)
    delta = torch.as_tensor(w.delta, device=DEV)
    sites = torch.as_tensor(w.start_sites, device=DEV)
    mu_ee, mu_he = AG.moments(eps, delta, geom, sites, w.N, w.tile)
    loss = AG.gap_map(mu_he, delta, w.U, P.weights(a, b)).sum()
    loss.backward(retain_graph=True)
    g1 = eps.grad.clone()
    loss.backward()
    torch.cuda.synchronize()
    assert torch.equal(eps.grad, 2.0 * g1)


def test_autograd_ldos_at_zero_matches_oracle():
    P = _P()
    from paper_1007_1609_amd import autograd as AG
    w = _small_cfg4()
    _, _, a, b = oracle.workload_bounds(w)
    s0 = W.site(w.Lx, w.Lx // 2, w.Ly // 2)
    geom = AG.Geometry.of(w, a, b)
    eps = torch.as_tensor(w.eps, device=DEV).requires_grad_(True)
    delta = torch.as_tensor(w.delta, device=DEV)
    sites = torch.tensor([s0], dtype=torch.int32, device=DEV)
    mu_ee, _ = AG.moments(eps, delta, geom, sites, w.N, 64)
    E0 = torch.zeros(1, dtype=torch.float64, device=DEV)
    ld = AG.local_dos(mu_ee, E0, P.weights(a, b))
    ld.sum().backward()
    # oracle: w_ee_n = (2 - delta_n0) g_n cos(n pi/2) / (pi a)
    n = np.arange(w.N)
    wee = np.where(n == 0, 1.0, 2.0) * oracle.jackson(w.N) * np.cos(n * np.pi / 2) / (np.pi * a)
    oe, _ = oracle.moments_backward(oracle.workload_csr(w, a, b), [s0], w.N, wee[None, :], np.zeros((1, w.N)))
    assert _rel(eps.grad.cpu().numpy(), oe) < 1e-10


def test_config4_full_size_gradient_vs_fd():
    """128x128, 64 impurities, N = 512, all 16384 start sites, sqrt(N)
    checkpoints: dSum(Delta)/dV at sampled impurity sites vs Richardson FD."""
    w = W.config4()
    _, _, a, b = oracle.workload_bounds(w)
    L0, g_eps, _ = _sum_delta_and_grad(w, w.eps, a, b)
    imp = np.flatnonzero(w.eps)
    pick = [int(imp[0]), int(imp[31])]
    for j in pick:
        def f(h):
            e = w.eps.copy()
            e[j] += h
            return _sum_delta_and_grad(w, e, a, b, grad=False)
        d1 = (f(1e-3) - f(-1e-3)) / 2e-3
        d2 = (f(5e-4) - f(-5e-4)) / 1e-3
        rich = (4 * d2 - d1) / 3
        print("config4 site %d: adjoint %.12e  FD %.12e" % (j, g_eps[j], rich))
        assert abs(g_eps[j] - rich) <= 1e-6 * np.max(np.abs(g_eps))


# ----------------------------------------------------------- Newton-Krylov
@pytest.mark.parametrize("jv", ["vjp", "fd"])
def test_newton_krylov_matches_plain_mixing(jv):
    P = _P()
    from paper_1007_1609_amd import scf
    w = _small_cfg4(L=20, N=192)
    d0 = torch.as_tensor(w.delta, device=DEV)
    op = P.Operator.from_workload(w, DEV)
    plain = scf.plain_mixing(op, w.U, d0, w.N, w.tile, tol=1e-9, max_iter=400)
    op.close()
    op = P.Operator.from_workload(w, DEV)
    nk = scf.newton_krylov(op, w.U, d0, w.N, w.tile, tol=1e-9, jv=jv)
    op.close()
    print("plain mixing %d passes, Newton-Krylov(%s) %d Newton steps / %s" % (
        plain.moment_passes, jv, nk.counts["newton"], nk.counts))
    assert plain.residual < 1e-9 and nk.residual < 1e-9
    assert maxdiff(plain.delta.cpu().numpy(), nk.delta.cpu().numpy()) < 2e-8


def test_anderson_mixing_reaches_the_plain_mixing_fixed_point():
    P = _P()
    from paper_1007_1609_amd import scf
    w = _small_cfg4(L=20, N=192)
    d0 = torch.as_tensor(w.delta, device=DEV)
    op = P.Operator.from_workload(w, DEV)
    plain = scf.plain_mixing(op, w.U, d0, w.N, w.tile, tol=1e-9, max_iter=400)
    op.close()
    op = P.Operator.from_workload(w, DEV)
    aa = scf.anderson_mixing(op, w.U, d0, w.N, w.tile, tol=1e-9, max_iter=200)
    op.close()
    print("plain mixing %d iterations, Anderson %d" % (plain.iterations, aa.iterations))
    assert aa.residual < 1e-9
    assert maxdiff(plain.delta.cpu().numpy(), aa.delta.cpu().numpy()) < 2e-8
    assert aa.iterations < plain.iterations


@pytest.mark.parametrize("method", ["plain", "anderson"])
def test_fp32_first_passes_reach_the_fp64_fixed_point(method):
    """FP32 recursion for the early gap-map evaluations, FP64 for the last:
    the loop ends on an FP64 evaluation below tol, at the FP64 fixed point."""
    P = _P()
    from paper_1007_1609_amd import scf
    w = _small_cfg4(L=20, N=192)
    d0 = torch.as_tensor(w.delta, device=DEV)
    op = P.Operator.from_workload(w, DEV)
    plain = scf.plain_mixing(op, w.U, d0, w.N, w.tile, tol=1e-9, max_iter=400)
    op.close()
    op = P.Operator.from_workload(w, DEV)
    fn = scf.plain_mixing if method == "plain" else scf.anderson_mixing
    kw = dict(max_iter=400) if method == "plain" else dict(max_iter=200)
    mixed = fn(op, w.U, d0, w.N, w.tile, tol=1e-9, fast_precision=P.CBDG_FP32_ACC64, **kw)
    op.close()
    print("%s: %d FP32 + %d FP64 evaluations (FP64 only: %d)" % (
        method, mixed.fast_passes, mixed.iterations - mixed.fast_passes, plain.iterations))
    assert mixed.fast_passes > 0 and mixed.iterations > mixed.fast_passes
    assert mixed.residual < 1e-9
    assert maxdiff(plain.delta.cpu().numpy(), mixed.delta.cpu().numpy()) < 2e-8


def test_reduced_moment_warm_up_reaches_the_same_fixed_point():
    """Anderson mixing whose plain warm-up steps use N/4 moments: the later
    evaluations use N, so the loop ends at the N-moment fixed point."""
    P = _P()
    from paper_1007_1609_amd import scf
    w = _small_cfg4(L=20, N=192)
    d0 = torch.as_tensor(w.delta, device=DEV)
    op = P.Operator.from_workload(w, DEV)
    plain = scf.plain_mixing(op, w.U, d0, w.N, w.tile, tol=1e-9, max_iter=400)
    op.close()
    op = P.Operator.from_workload(w, DEV)
    aa = scf.anderson_mixing(op, w.U, d0, w.N, w.tile, tol=1e-9, max_iter=200, warmup_N=w.N // 4,
                             fast_precision=P.CBDG_FP32_ACC64)
    op.close()
    print("Anderson: %d evaluations, %d with N/4, %d FP32" % (aa.iterations, aa.warmup_passes, aa.fast_passes))
    assert aa.warmup_passes > 0 and aa.iterations > aa.warmup_passes
    assert aa.residual < 1e-9
    assert maxdiff(plain.delta.cpu().numpy(), aa.delta.cpu().numpy()) < 2e-8
