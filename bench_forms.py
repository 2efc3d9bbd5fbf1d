"""Measurements of the forms beside the default benchmark step (imported by
bench.py).  Each returns one JSON-able dict.

fp32_accuracy  FP32 recursion vs the FP64 recursion on the same operator:
               moments, one-step Delta and LDOS errors (the FP64 path itself is
               held to the oracle by the parity tests)
complex_form   512x512 Peierls + d-wave lattice, 4096 start sites, N = 2048,
               complex128 and complex64 recursion, LDOS at 512 energies
adjoint_form   128x128 workload with 64 impurities, N = 512: forward pass,
               reverse pass for dSum(Delta)/dV, dLDOS(0)/dV at the centre, and
               the self-consistent solve by plain mixing and by Newton-Krylov
scf_form       256x256 workload solved self-consistently to max|dDelta| < 1e-6
paper_form     the paper's two example geometries (surface LDOS convergence with
               N at constant Lorentz broadening; impurity LDOS maps)
"""
from __future__ import annotations

import os
import sys
import math
import time

import numpy as np
import torch

import paper_1007_1609_amd as P
import workloads as W
from paper_1007_1609_amd import scf

METRIC = "Chebyshev moments/sec and HBM GB/s (FP64 vs FP32); self-consistent solve time"
HBM_PEAK_GBS = 8000.0


def log(msg):
    print("[bench] " + msg, file=sys.stderr, flush=True)


def _cone_sites(x, y, Lx, Ly, bc_x, bc_y, n):
    """Sites inside the box of the start sites widened by n (open directions;
    x at site granularity, exact for tiles of whole lattice rows)."""
    if x.size == 0:
        return 0
    rows = Ly if bc_y else min(Ly - 1, int(y.max()) + n) - max(0, int(y.min()) - n) + 1
    cols = Lx if bc_x else min(Lx - 1, int(x.max()) + n) - max(0, int(x.min()) - n) + 1
    return max(rows, 0) * max(cols, 0)


def diamond_sites(x, y, Lx, Ly, bc_x, bc_y, R):
    """Summed over the start sites (x, y): the lattice sites within lattice
    (Manhattan) distance R of each, where a_R of a start vector can be
    non-zero (Ht couples nearest neighbours).  On an open lattice: the
    diamond's 2R^2 + 2R + 1 sites less the m^2 past each edge it crosses by m
    rows or columns, plus the (m+1)(m+2)/2 past each pair of adjacent edges
    it crosses with m = R - (distance to both edges) - 2 >= 0.  Periodic
    directions are counted row by row."""
    x = np.asarray(x, dtype=np.int64)
    y = np.asarray(y, dtype=np.int64)
    if R < 0 or x.size == 0:
        return 0
    if not bc_x and not bc_y:
        lx, rx, ly, ry = x, Lx - 1 - x, y, Ly - 1 - y   # distances to the four edges
        c = np.full(x.shape, 2 * R * R + 2 * R + 1, dtype=np.int64)
        for e in (lx, rx, ly, ry):
            m = np.maximum(R - e, 0)
            c -= m * m
        for ex in (lx, rx):
            for ey in (ly, ry):
                m = R - ex - ey - 2
                c += np.where(m >= 0, (m + 1) * (m + 2) // 2, 0)
        return int(c.sum())

    def width(r):
        if bc_x:
            return np.full(x.shape, min(2 * r + 1, Lx), dtype=np.int64)
        return np.minimum(x + r, Lx - 1) - np.maximum(x - r, 0) + 1

    total = 0
    if bc_y:
        for d in range(0, min(R, Ly // 2) + 1):
            mult = 1 if d == 0 or 2 * d == Ly else 2
            total += mult * int(width(R - d).sum())
    else:
        for dy in range(-R, R + 1):
            ok = (y + dy >= 0) & (y + dy < Ly)
            total += int(np.where(ok, width(R - abs(dy)), 0).sum())
    return total


def vc_traffic(sites, Lx, Ly, bc_x, bc_y, n_steps, K):
    """Launches of one tile in the vector-contiguous passes (one wavefront per
    vector, each clipped to its own light cone) and the Nambu pairs they must
    move through HBM at minimum, summed over the tile's vectors:
      first step   read a_0, write a_1: D(0) + D(1)
      K-step pass  read a_{n-2}, a_{n-1}, write a_{n+K-2}, a_{n+K-1}:
                   D(n-2) + D(n-1) + D(n+K-2) + D(n+K-1)
      single step  read a_{n-2}, a_{n-1}, write a_n: D(n-2) + D(n-1) + D(n)
    with D(R) the sites within distance R of the vector's start site.  Steps
    2.. go K at a time, a remainder of two or more in one shorter pass, a
    remainder of one as a single step.  Returns (launches, pairs
    moved, pairs of the plain one-step streaming recursion, 3 x L2 per step
    and vector)."""
    sites = np.asarray(sites)
    sites = sites[(sites >= 0) & (sites < Lx * Ly)]
    x, y = sites % Lx, sites // Lx
    if n_steps < 1 or sites.size == 0:
        return 0, 0, 0
    cache = {}

    def D(R):
        if R not in cache:
            cache[R] = diamond_sites(x, y, Lx, Ly, bc_x, bc_y, R)
        return cache[R]
    launches, moved = 1, D(0) + D(1)
    n = 2
    while n + K - 1 <= n_steps:
        launches += 1
        moved += D(n - 2) + D(n - 1) + D(n + K - 2) + D(n + K - 1)
        n += K
    rest = n_steps - n + 1
    if rest >= 2:  # one shorter pass
        launches += 1
        moved += D(n - 2) + D(n - 1) + D(n + rest - 2) + D(n + rest - 1)
        n += rest
    while n <= n_steps:
        launches += 1
        moved += D(n - 2) + D(n - 1) + D(n)
        n += 1
    return launches, moved, 3 * Lx * Ly * n_steps * sites.size


def recursion_traffic(sites, Lx, Ly, bc_x, bc_y, n_steps, two_step, three_step=False):
    """Recursion launches of one tile as the library issues them, and the
    vector elements (site x vector, in units of one Nambu pair per vector)
    each must move through HBM at minimum:
      first step   read a_0, write a_1 over the lattice: 2 x L2
      three-step   read a_{n-2}, a_{n-1}, write a_{n+1}, a_{n+2} inside the light
                   cone of step n+2: 4 x cone(n+2)
      two-step     read a_{n-2}, a_{n-1}, write a_n, a_{n+1} inside the light
                   cone of step n+1: 4 x cone(n+1)
      single step  read a_{n-2}, a_{n-1}, write a_n inside cone(n): 3 x cone(n)
    On real operators with uniform hopping steps 2.. go in threes (tiles of
    more than 128 vectors) or pairs, the remainder in a pair and/or a single
    step, as the library issues them.  Returns (launches, pair-elements moved, pair-elements of the
    plain one-step streaming recursion over the whole lattice, 3 x L2 per
    step)."""
    sites = np.asarray(sites)
    sites = sites[(sites >= 0) & (sites < Lx * Ly)]
    x, y = sites % Lx, sites // Lx
    L2 = Lx * Ly
    if n_steps < 1:
        return 0, 0, 0
    launches, moved = 1, 2 * L2
    n = 2
    if two_step and three_step:
        while n + 2 <= n_steps:
            launches += 1
            moved += 4 * _cone_sites(x, y, Lx, Ly, bc_x, bc_y, n + 2)
            n += 3
    if two_step:
        while n + 1 <= n_steps:
            launches += 1
            moved += 4 * _cone_sites(x, y, Lx, Ly, bc_x, bc_y, n + 1)
            n += 2
    while n <= n_steps:
        launches += 1
        moved += 3 * _cone_sites(x, y, Lx, Ly, bc_x, bc_y, n)
        n += 1
    return launches, moved, 3 * L2 * n_steps


def adjoint_traffic(N, L2, ckpt=0, tile=1024):
    """Vector streams of the doubling-form reverse pass of one tile (real
    operator, uniform hopping), each a whole-lattice read or write of every
    vector, as the library issues them: the forward a_0 .. a_M keeping the
    checkpoint pairs (M = N // 2; seed 1 write, first step 2, three-step
    passes 4 when the checkpoint stride is a multiple of 3 and the tile has
    more than 128 vectors, two-step passes 4, single steps 3), the
    recomputation of each segment's inner vectors (two-step passes 4, a last
    single step 3), and the adjoint steps m = M .. 1 (read lam_{m+1} and
    lam_{m+2} where they exist, a_{m-1} and a_m; write lam_m).  The default
    stride is ceil(sqrt(M + 1)) rounded up to a multiple of 3.
    Returns (streams, launches)."""
    M = N // 2
    top = M
    k = ckpt if ckpt > 0 else 3 * -(-int(math.ceil(math.sqrt(M + 1))) // 3)
    J = -(-(top + 1) // k)
    three = k % 3 == 0 and tile >= 129
    streams, launches = 1, 0
    n = 1
    while n <= top:
        if three and n >= 2 and n + 2 <= top:
            streams += 4; n += 3
        elif n >= 2 and n + 1 <= top:
            streams += 4; n += 2
        else:
            streams += 2 if n == 1 else 3; n += 1
        launches += 1
    for j in range(J):
        s0, e0 = j * k, min(j * k + k - 1, top)
        m = s0 + 2
        while m <= e0:
            if m + 1 <= e0:
                streams += 4; m += 2
            else:
                streams += 3; m += 1
            launches += 1
    for m in range(M, 0, -1):
        streams += (m + 1 <= M) + (m + 2 <= M) + 3
        launches += 1
    return streams, launches


def _timed(fn):
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    out = fn()
    e1.record(stream)
    torch.cuda.synchronize()
    return out, e0.elapsed_time(e1) / 1e3


def fp32_accuracy(w, op, mu_ee32, mu_he32, energies, dev, n_rows=2048, algorithm=0):
    """FP32-recursion results vs the FP64 recursion for the first n_rows
    start sites at the initial Delta (both with the same moment algorithm)."""
    d0 = torch.as_tensor(w.delta, device=dev)
    op.update_delta(d0)
    sites = torch.arange(n_rows, dtype=torch.int32, device=dev)
    m32 = P.chebyshev_moments(op, sites, w.N, w.tile, P.CBDG_FP32_ACC64, algorithm=algorithm)
    m64 = P.chebyshev_moments(op, sites, w.N, w.tile, P.CBDG_FP64, algorithm=algorithm)
    wt = op.weights()
    d32, _ = P.gap_update(m32[1], wt, w.U, d0[:n_rows].contiguous())
    d64, _ = P.gap_update(m64[1], wt, w.U, d0[:n_rows].contiguous())
    l32 = P.ldos(m32[0], wt, energies)
    l64 = P.ldos(m64[0], wt, energies)
    torch.cuda.synchronize()
    mom = max(float((m32[0] - m64[0]).abs().max()), float((m32[1] - m64[1]).abs().max()))
    return {"reference": "FP64 recursion on the GPU (held to the oracle at 1e-10 by the parity tests)",
            "rows": n_rows, "N": w.N,
            "moments_max_abs_err": mom,
            "delta_one_step_max_abs_err": float((d32 - d64).abs().max()),
            "ldos_max_err_rel_to_max": float((l32 - l64).abs().max() / l64.abs().max()),
            "bars": {"delta": 1e-6, "ldos_rel": 1e-5}}


def _algorithm(args, op, N):
    """(ABI algorithm, recursion launches per tile) for --algorithm."""
    alg = {"auto": P.CBDG_ALG_AUTO, "direct": P.CBDG_ALG_DIRECT,
           "doubling": P.CBDG_ALG_DOUBLING}[getattr(args, "algorithm", "auto")]
    dbl = alg == P.CBDG_ALG_DOUBLING or (alg == P.CBDG_ALG_AUTO and op.bounds.b == 0.0 and N >= 3)
    return alg, (N // 2 if dbl else N - 1)


def _moments_pass(op, sites, N, tile, prec, ws, out, alg=0):
    """All tiles, one call per tile with HIP events; returns per-launch us."""
    stream = torch.cuda.current_stream()
    n = sites.numel()
    ev = []
    for t0 in range(0, n, tile):
        t1 = min(n, t0 + tile)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        P.chebyshev_moments(op, sites[t0:t1], N, tile, prec, ws=ws, out=(out[0][t0:t1], out[1][t0:t1]),
                            algorithm=alg)
        e1.record(stream)
        ev.append((e0, e1, t1 - t0))
    torch.cuda.synchronize()
    total = sum(a.elapsed_time(b) for a, b, _ in ev) / 1e3
    return total, ev


def complex_form(args, dev):
    w = W.config3()
    N, tile = w.N, w.tile
    op = P.Operator.from_workload(w, dev)
    sites = torch.as_tensor(w.start_sites, device=dev)
    n = sites.numel()
    E = torch.as_tensor(w.energies, device=dev)
    wt = op.weights()
    res = {}
    ldos = {}
    alg, steps = _algorithm(args, op, N)
    for name, prec, s_bytes in (("complex128", P.CBDG_FP64, 8), ("complex64", P.CBDG_FP32_ACC64, 4)):
        ws = P.workspace(P.moments_workspace_bytes(op, tile, prec, alg), dev)
        out = (torch.empty((n, N), dtype=torch.float64, device=dev),
               torch.empty((n, N), dtype=torch.complex128, device=dev))
        # warm-up on one tile, then the timed pass over all 4 tiles
        P.chebyshev_moments(op, sites[:64], N, 64, prec, ws=ws, algorithm=alg)
        torch.cuda.synchronize()
        t, ev = _moments_pass(op, sites, N, tile, prec, ws, out, alg)
        ld, t_ldos = _timed(lambda: P.ldos(out[0], wt, E))
        ldos[name] = ld
        launches = 0
        nbytes = nfull = 0.0
        sites_np = w.start_sites
        for k, (_, _, bt) in enumerate(ev):
            nl, moved, full = recursion_traffic(sites_np[k * tile:k * tile + bt], w.Lx, w.Ly, w.bc_x, w.bc_y,
                                                steps, two_step=False)
            unit = 2 * 2 * s_bytes * ((bt + 63) // 64 * 64)  # (e,h) x (re,im) per vector
            launches += nl
            nbytes += moved * unit
            nfull += full * unit
        gbs = nfull / t / 1e9       # streaming recursion: 3 vectors over the lattice per step
        min_gbs = nbytes / t / 1e9  # what the launches must move at least (light cone)
        res[name] = {"moments_per_s": n * N / (t + t_ldos), "seconds_moments": t, "seconds_ldos": t_ldos,
                     "avg_launch_us": t / launches * 1e6, "achieved_GBps": gbs, "frac": gbs / HBM_PEAK_GBS,
                     "min_bytes_GBps": min_gbs, "min_bytes_frac": min_gbs / HBM_PEAK_GBS,
                     "moments_bounded": bool(P.check_moments(out[0], out[1], 1e-9 if s_bytes == 8 else 1e-4))}
        log("%s: %.2f s moments, %.0f GB/s" % (name, t, gbs))
        del ws, out
        torch.cuda.empty_cache()
    err = float((ldos["complex64"] - ldos["complex128"]).abs().max() / ldos["complex128"].abs().max())
    op.close()
    line = {"metric": METRIC, "value": res["complex128"]["moments_per_s"], "unit": "moments/s",
            "n_gpus": 1, "higher_is_better": True, "dtype": "complex128 (and complex64)",
            "data": "synthetic",
            "config": {"workload": "%s: 512x512 open lattice, Peierls flux 1/256 per plaquette, d-wave bond "
                                   "pairing with four phase windings, N=%d, 4096 start sites (stride-8 grid) "
                                   "in tiles of %d, LDOS at 512 energies" % (w.name, N, tile),
                       "recursion_launches_per_tile": steps},
            "forms": res, "complex64_ldos_err_rel_to_max": err,
            "roofline": {"kernel": "k_cheb_step<complex double>", "bound": "hbm",
                         "achieved": res["complex128"]["achieved_GBps"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": res["complex128"]["frac"], "traffic": None,
                         "basis": "streaming recursion: 3 vectors over the lattice per recursion step",
                         "min_bytes_GBps": res["complex128"]["min_bytes_GBps"],
                         "min_bytes_frac": res["complex128"]["min_bytes_frac"]}}
    if not args.no_cpu_baseline:
        import oracle
        threads = int(os.environ.get("OMP_NUM_THREADS", "0") or 0) or os.cpu_count() or 1
        a, b = oracle.workload_bounds(w)[2:]
        H = oracle.workload_csr(w, a, b)
        Nc = 256
        sample = w.start_sites[np.linspace(0, n - 1, threads).astype(int)]
        t0 = time.perf_counter()
        oracle.moments(H, sample, Nc, n_threads=threads)
        dt = time.perf_counter() - t0
        line["cpu_baseline"] = {"value": len(sample) * Nc / dt, "unit": "moments/s", "cores": oracle.max_threads(),
                                "kind": "oracle",
                                "sample": "%d start sites of the same 512x512 complex lattice, N=%d, "
                                          "%.1f s" % (len(sample), Nc, dt)}
    return line


def reversible_streams(N, K=6):
    """Vector streams of one tile in the checkpoint-free reverse passes (units
    of one vector of L2 pairs): the forward moments' minimum is counted by
    the forward; here one more forward step (read 2, write 1), then per pass
    the regenerated pair and the cotangent pair read and written and G read
    and written (the first pass reads no cotangents and no G; the last,
    shorter pass writes only G), then the sum of G over the tile."""
    M = N // 2
    passes = -(-M // K)
    full = M // K
    streams = 3 + 1
    for p in range(passes):
        is_full = p < full
        reads = 2 + (0 if p == 0 else 3)
        writes = (4 if is_full else 0) + 1
        streams += reads + writes
    return streams


def adjoint_form(args, dev):
    from paper_1007_1609_amd import autograd as AG
    w = W.config4()
    N, tile = w.N, w.tile
    op = P.Operator.from_workload(w, dev)
    a, b = op.bounds.a, op.bounds.b
    op.close()
    geom = AG.Geometry.of(w, a, b)
    sites = torch.as_tensor(w.start_sites, device=dev)
    wt = P.weights(a, b)

    def forward_backward(ckpt=0):
        eps = torch.as_tensor(w.eps, device=dev).requires_grad_(True)
        delta = torch.as_tensor(w.delta, device=dev).requires_grad_(True)
        mu_ee, mu_he = AG.moments(eps, delta, geom, sites, N, tile, ckpt)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        loss = AG.gap_map(mu_he, delta, w.U, wt).sum()
        loss.backward()
        torch.cuda.synchronize()
        return eps.grad, time.perf_counter() - t0

    forward_backward()  # warm-up (allocates the checkpoint workspace)
    eps0 = torch.as_tensor(w.eps, device=dev)
    d0 = torch.as_tensor(w.delta, device=dev)
    (_, _), t_fwd = _timed(lambda: AG.moments(eps0, d0, geom, sites, N, tile))
    g_sum, t_bwd = forward_backward()
    # the checkpoint-free reverse passes (forward vectors regenerated backwards)
    forward_backward(P.REVERSIBLE)
    g_rev, t_rev = forward_backward(P.REVERSIBLE)
    torch.cuda.empty_cache()
    # every forward vector stored (checkpoint stride 1: no segment
    # recomputation, about 70 GB of workspace per 1024-vector tile)
    forward_backward(1)
    g1, t_bwd1 = forward_backward(1)
    torch.cuda.empty_cache()
    # dLDOS(0)/dV at the centre site: one start vector
    s0 = w.notes["centre_site"]
    eps = torch.as_tensor(w.eps, device=dev).requires_grad_(True)
    t0 = time.perf_counter()
    mu_ee, _ = AG.moments(eps, d0, geom, torch.tensor([s0], dtype=torch.int32, device=dev), N, 64)
    AG.local_dos(mu_ee, torch.zeros(1, dtype=torch.float64, device=dev), wt).sum().backward()
    torch.cuda.synchronize()
    t_ldos = time.perf_counter() - t0
    log("adjoint: forward %.2f s, reverse %.2f s (checkpoints), %.2f s (regenerated vectors)" % (t_fwd, t_bwd, t_rev))
    rev_streams = reversible_streams(N)
    rev_b = sum(rev_streams * w.L2 * 16.0 * min(tile, w.L2 - t * tile) for t in range(-(-w.L2 // tile)))
    reversible = {"seconds": t_rev, "over_forward": t_rev / t_fwd, "vector_streams_per_tile": rev_streams,
                  "algorithmic_bytes": rev_b, "algorithmic_GBps": rev_b / t_rev / 1e9, "frac": rev_b / t_rev / 8e12,
                  "max_abs_grad_diff_vs_checkpoints": float((g_rev - g_sum).abs().max()),
                  "note": "includes the forward moments of every tile (vector-contiguous passes) and one step more"}
    # the whole Jacobian of the gap map (one reverse sweep, rows kept) and its
    # product with a vector
    op = P.Operator.from_workload(w, dev)
    d_mu, _ = P.gap_update_backward(torch.ones(w.L2, dtype=torch.float64, device=dev), N, op.weights("jackson"),
                                    w.U, 1.0, want_delta_in=False)
    all_sites = torch.arange(w.L2, dtype=torch.int32, device=dev)
    _, Jm = P.chebyshev_moments_jacobian(op, all_sites, N, tile, None, d_mu)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    P.chebyshev_moments_jacobian(op, all_sites, N, tile, None, d_mu, jac_delta=Jm)
    torch.cuda.synchronize()
    t_jac = time.perf_counter() - t0
    op.close()
    xv = torch.ones(w.L2, dtype=torch.float64, device=dev)
    yv = torch.empty_like(xv)
    P.jacobian_matvec(Jm, xv, out=yv)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(20):
        P.jacobian_matvec(Jm, xv, out=yv)
    e1.record()
    torch.cuda.synchronize()
    mv_ms = e0.elapsed_time(e1) / 20
    jacobian = {"seconds_build": t_jac, "rows": w.L2, "bytes": Jm.numel() * 8,
                "matvec_ms": mv_ms, "matvec_GBps": Jm.numel() * 8 / (mv_ms * 1e-3) / 1e9,
                "matvec_frac": Jm.numel() * 8 / (mv_ms * 1e-3) / 8e12,
                "note": "rows of dF/dDelta from one checkpoint-free reverse sweep (its forward included); "
                        "the matvec reads the matrix once per product"}
    del Jm
    torch.cuda.empty_cache()
    log("jacobian: build %.2f s, matvec %.3f ms" % (t_jac, mv_ms))
    n_tiles = -(-w.L2 // tile)
    streams, launches = adjoint_traffic(N, w.L2)
    rev_bytes = 0.0  # a vector of a tile: L2 sites x 16 B
    for t in range(n_tiles):
        bt = min(tile, w.L2 - t * tile)
        rev_bytes += streams * w.L2 * 16.0 * bt
    reverse = {"vector_streams_per_tile": streams, "launches_per_tile": launches,
               "algorithmic_bytes": rev_bytes, "algorithmic_GBps": rev_bytes / t_bwd / 1e9,
               "frac": rev_bytes / t_bwd / 8e12}
    out = {}
    if getattr(args, "no_scf", False):
        n_moments = w.L2 * N
        return {"metric": METRIC, "value": n_moments / t_fwd, "unit": "moments/s", "n_gpus": 1,
                "higher_is_better": True, "dtype": "f64", "data": "synthetic",
                "config": {"workload": "%s: 128x128, N=%d, reverse pass only" % (w.name, N)},
                "seconds_forward": t_fwd, "seconds_reverse_dsumdelta_dV": t_bwd, "reverse": reverse,
                "reverse_over_forward": t_bwd / t_fwd, "seconds_reverse_stride1": t_bwd1,
                "reverse_stride1_over_forward": t_bwd1 / t_fwd, "reverse_regenerated": reversible,
                "jacobian": jacobian}
    # self-consistency: plain mixing vs Newton-Krylov (both to 1e-6)
    op = P.Operator.from_workload(w, dev)
    r = scf.plain_mixing(op, w.U, d0, N, tile, tol=1e-6, max_iter=300)
    out["plain_mixing"] = {"iterations": r.iterations, "gap_map_evaluations": r.iterations,
                           "seconds": r.seconds, "residual": r.residual}
    ref = r.delta
    op.close()
    log("plain mixing: %d iterations, %.1f s" % (r.iterations, r.seconds))
    for name, jv, rebuild in (("vjp", "vjp", True), ("fd", "fd", True), ("jacobian", "jacobian", True),
                              ("jacobian_chord", "jacobian", False)):
        op = P.Operator.from_workload(w, dev)
        r = scf.newton_krylov(op, w.U, d0, N, tile, tol=1e-6, jv=jv, rebuild_jacobian=rebuild)
        op.close()
        out["newton_krylov_" + name] = {"newton_steps": r.counts["newton"], "warmup_iterations": r.counts["warmup"],
                                        "gap_map_evaluations": r.counts["F"], "jacobian_products": r.counts["J"],
                                        "jacobians_built": r.counts["jacobian"],
                                        "seconds": r.seconds, "residual": r.residual,
                                        "max_abs_diff_vs_plain": float((r.delta - ref).abs().max())}
        log("newton-krylov %s: %s, %.1f s" % (name, r.counts, r.seconds))
    n_moments = w.L2 * N
    return {"metric": METRIC, "value": n_moments / t_fwd, "unit": "moments/s", "n_gpus": 1,
            "higher_is_better": True, "dtype": "f64", "data": "synthetic",
            "config": {"workload": "%s: 128x128 open lattice, 64 impurities V~U[0,4] (seed 4), t=1 mu=-0.5 "
                                   "U=2, N=%d, all 16384 start sites in tiles of %d, sqrt(N) checkpoints"
                                   % (w.name, N, tile)},
            "seconds_forward": t_fwd, "seconds_reverse_dsumdelta_dV": t_bwd, "reverse": reverse,
            "reverse_over_forward": t_bwd / t_fwd, "seconds_dldos0_dV_centre": t_ldos,
            "seconds_reverse_stride1": t_bwd1, "reverse_stride1_over_forward": t_bwd1 / t_fwd,
            "stride1_max_abs_grad_diff": float((g1 - g_sum).abs().max()), "reverse_regenerated": reversible,
            "jacobian": jacobian,
            "grad_norm_inf": float(g_sum.abs().max()), "scf": out}


def differentiation_summary(dev):
    """The differentiation form in brief, for the default bench line (128x128
    workload, N = 512): d(sum Delta)/dV by the checkpoint-free reverse passes
    against a Richardson finite difference at the centre site, the whole
    Jacobian of the gap map, and the self-consistent solve by Newton on that
    Jacobian (kept from the first Newton step) against plain mixing."""
    from paper_1007_1609_amd import autograd as AG
    from paper_1007_1609_amd import scf
    w = W.config4()
    N, tile = w.N, w.tile
    op = P.Operator.from_workload(w, dev)
    a, b = op.bounds.a, op.bounds.b
    op.close()
    geom = AG.Geometry.of(w, a, b)
    sites = torch.as_tensor(w.start_sites, device=dev)
    wt = P.weights(a, b)
    d0 = torch.as_tensor(w.delta, device=dev)

    def grad_sum_delta():
        eps = torch.as_tensor(w.eps, device=dev).requires_grad_(True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, mu_he = AG.moments(eps, d0, geom, sites, N, tile, P.REVERSIBLE)
        AG.gap_map(mu_he, d0, w.U, wt).sum().backward()
        torch.cuda.synchronize()
        return eps.grad.cpu().numpy(), time.perf_counter() - t0

    def sum_delta(eps_np):
        with torch.no_grad():
            _, mu_he = AG.moments(torch.as_tensor(eps_np, device=dev), d0, geom, sites, N, tile)
            return float(AG.gap_map(mu_he, d0, w.U, wt).sum())

    grad_sum_delta()
    g, t_grad = grad_sum_delta()
    j = int(w.notes["centre_site"])

    def f(h):
        e = np.array(w.eps, dtype=np.float64)
        e[j] += h
        return sum_delta(e)

    d1 = (f(1e-3) - f(-1e-3)) / 2e-3
    d2 = (f(5e-4) - f(-5e-4)) / 1e-3
    rich = (4 * d2 - d1) / 3
    op = P.Operator.from_workload(w, dev)
    plain = scf.plain_mixing(op, w.U, d0, N, tile, tol=1e-6, max_iter=300)
    op.close()
    op = P.Operator.from_workload(w, dev)
    nk = scf.newton_krylov(op, w.U, d0, N, tile, tol=1e-6, jv="jacobian", rebuild_jacobian=False)
    op.close()
    torch.cuda.empty_cache()
    log("differentiation: gradient %.2f s, FD rel err %.1e; plain %.2f s, Newton (Jacobian) %.2f s" % (
        t_grad, abs(g[j] - rich) / np.max(np.abs(g)), plain.seconds, nk.seconds))
    return {"workload": "%s: 128x128 open lattice, 64 impurities V~U[0,4] (seed 4), t=1 mu=-0.5 U=2, N=%d, "
                        "all 16384 start sites in tiles of %d" % (w.name, N, tile),
            "grad_sum_delta_dV_seconds": t_grad,
            "grad_note": "forward moments and checkpoint-free reverse passes, through torch.autograd",
            "fd_check": {"site": j, "adjoint": float(g[j]), "richardson_fd": float(rich),
                         "rel_err_vs_max_grad": float(abs(g[j] - rich) / np.max(np.abs(g))), "bar": 1e-6},
            "plain_mixing": {"seconds": plain.seconds, "gap_map_evaluations": plain.iterations,
                             "residual": plain.residual},
            "newton_whole_jacobian": {"seconds": nk.seconds, "gap_map_evaluations": nk.counts["F"],
                                      "jacobians_built": nk.counts["jacobian"], "newton_steps": nk.counts["newton"],
                                      "jacobian_products": nk.counts["J"], "residual": nk.residual,
                                      "max_abs_diff_vs_plain": float((nk.delta - plain.delta).abs().max())},
            "newton_over_plain_speedup": plain.seconds / nk.seconds}


def scf_form(args, dev):
    w = W.config1()
    op = P.Operator.from_workload(w, dev)
    d0 = torch.as_tensor(w.delta, device=dev)
    method = getattr(args, "scf_method", "plain")
    fast = P.CBDG_FP32_ACC64 if getattr(args, "scf_fp32", False) else None
    cb = lambda it, res: log("iteration %d residual %.3e" % (it, res))  # noqa: E731
    sched = (", FP32 recursion until the residual is below 5e-7, FP64 after (only an FP64 "
             "evaluation ends the loop)") if fast is not None else ""
    if method == "plain":
        r = scf.plain_mixing(op, w.U, d0, w.N, w.tile, tol=1e-6, max_iter=60, callback=cb,
                             fast_precision=fast)
        how = "plain mixing (alpha=1)" + sched
        passes = r.iterations
        extra = {"fp32_passes": r.fast_passes, "fp64_passes": passes - r.fast_passes}
    elif method == "anderson":
        wn = int(getattr(args, "scf_warmup_n", 0) or 0)
        r = scf.anderson_mixing(op, w.U, d0, w.N, w.tile, tol=1e-6, max_iter=60, callback=cb,
                                fast_precision=fast, warmup_N=wn)
        how = "Anderson mixing (depth 5, beta 1)" + sched
        if 0 < wn < w.N:
            how += ", plain-mixing warm-up with N=%d moments down to a residual of 1e-2" % wn
        passes = r.iterations
        extra = {"fp32_passes": r.fast_passes, "fp64_passes": passes - r.fast_passes,
                 "warmup_passes": r.warmup_passes, "warmup_N": wn}
    elif method == "nk-jacobian":
        r = scf.newton_krylov(op, w.U, d0, w.N, w.tile, tol=1e-6, jv="jacobian", rebuild_jacobian=False,
                              callback=cb)
        how = ("Newton on the whole Jacobian (one checkpoint-free reverse sweep, kept from the first Newton "
               "step) after plain-mixing warm-up to 1e-2")
        passes = r.counts["F"]
        extra = {"counts": r.counts}
    else:
        r = scf.newton_krylov(op, w.U, d0, w.N, w.tile, tol=1e-6, jv="fd", callback=cb)
        how = "Newton-Krylov with finite-difference Jacobian products after plain-mixing warm-up to 1e-2"
        passes = r.counts["F"] + r.counts["J"]
        extra = {"counts": r.counts}
    op.close()
    line = {"metric": METRIC, "value": r.seconds, "unit": "s (self-consistent solve)", "n_gpus": 1,
            "higher_is_better": False, "dtype": "f64", "data": "synthetic",
            "config": {"workload": "%s: 256x256 open lattice, 655 disordered sites, U=2.5, N=1024, "
                                   "all 65536 sites, %s to max|dDelta| < 1e-6" % (w.name, how)},
            "iterations": r.iterations, "moment_passes": passes, "residual": r.residual, "history": r.history,
            "seconds_per_pass": r.seconds / passes,
            "moments_per_s": w.L2 * (w.N * (passes - r.warmup_passes)
                                     + getattr(args, "scf_warmup_n", 0) * r.warmup_passes) / r.seconds}
    line.update(extra)
    return line


def resident_form(args, dev, tiles=(64, 128, 256)):
    """The 128x128 differentiation workload's forward moments (16384 start
    sites, N = 512, FP64 doubling) with every recursion step of a tile in one
    persistent launch (tiles whose two buffers stay in the Infinity Cache),
    beside the HBM-streaming path at the same tile sizes and at its default
    1024-vector tiles.  Bytes: 3 vectors over the whole lattice per step for
    the resident launch (it has no light cone), the minimum per launch for
    the streaming path (bench.launch_bytes)."""
    from bench import launch_bytes
    w = W.config4()
    N = w.N
    op = P.Operator.from_workload(w, dev)
    sites = torch.as_tensor(w.start_sites, device=dev)
    n = sites.numel()
    out = (torch.empty((n, N), dtype=torch.float64, device=dev), torch.empty((n, N), dtype=torch.float64, device=dev))
    res = {"workload": "%s: 128x128, 64 impurities, N=%d, all %d start sites, FP64, moment doubling" % (w.name, N, n)}
    stream = torch.cuda.current_stream()
    ref = None
    for tile in tiles:
        ws = P.workspace(P.resident_workspace_bytes(op, tile), dev)
        P.chebyshev_moments_resident(op, sites[:tile], N, tile, ws=ws, out=(out[0][:tile], out[1][:tile]))
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        P.chebyshev_moments_resident(op, sites, N, tile, ws=ws, out=out)
        e1.record(stream)
        torch.cuda.synchronize()
        t = e0.elapsed_time(e1) / 1e3
        steps = N // 2
        nbytes = 3.0 * steps * w.L2 * 16 * ((tile + 63) // 64 * 64) * (n // tile)
        res["resident_tile%d" % tile] = {"seconds": t, "moments_per_s": n * N / t,
                                         "vector_GBps": nbytes / t / 1e9,
                                         "buffers_MiB": 2 * w.L2 * ((tile + 63) // 64 * 64) * 16 / 2 ** 20}
        if ref is None:
            ref = out[0].clone()
        del ws
        log("resident tiles of %d: %.3f s" % (tile, t))
    res["resident_max_abs_diff_between_tilings"] = float((out[0] - ref).abs().max())
    for tile in tiles + (1024,):
        ws = P.workspace(P.moments_workspace_bytes(op, tile), dev)
        P.chebyshev_moments(op, sites[:tile], N, tile, ws=ws, out=(out[0][:tile], out[1][:tile]))
        torch.cuda.synchronize()
        ev = []
        for t0 in range(0, n, tile):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            P.chebyshev_moments(op, sites[t0:t0 + tile], N, tile, ws=ws, out=(out[0][t0:t0 + tile], out[1][t0:t0 + tile]))
            e1.record(stream)
            ev.append((e0, e1, min(tile, n - t0)))
        torch.cuda.synchronize()
        kern, nl, ms, moved, streamed = launch_bytes(ev, w.start_sites, tile, len(ev), w, N // 2, True, 8)
        res["streaming_tile%d" % tile] = {"seconds": ms / 1e3, "moments_per_s": n * N / (ms / 1e3),
                                          "kernel": kern, "min_bytes_GBps": moved / (ms / 1e3) / 1e9,
                                          "effective_GBps": streamed / (ms / 1e3) / 1e9}
        del ws
        log("streaming tiles of %d: %.3f s" % (tile, ms / 1e3))
    op.close()
    return res


def paper_form(args, dev):
    """The paper's two examples as synthetic workloads.

    First example (planar normal metal 380a / superconductor 20a x 500a,
    Delta = 0.1t): LDOS at 64 surface sites of the normal metal with the
    Lorentz kernel at constant broadening eps = 0.001t (lambda = N eps / a),
    for N = 2000 .. 16000, and how far each N is from the largest.
    Second example (SC/N/SC 50a/50a/50a x 100a, Gaussian impurity V = 2t at
    (60a, 50a)): LDOS maps at E = 0, 0.03t, 0.06t on the 21x21 square around
    the impurity, minus those of the clean system, for the sandwich and for a
    homogeneous normal metal."""
    res = {"sn_surface": {}, "sns_impurity": {}}
    eps = 0.001
    Ns = (2000, 4000, 8000, 16000)
    w0 = W.sn_surface(N=Ns[-1])
    op = P.Operator.from_workload(w0, dev)
    a = op.bounds.a
    sites = torch.as_tensor(w0.start_sites, device=dev)
    E = torch.as_tensor(w0.energies, device=dev)
    ld = {}
    for N in Ns:
        lam = N * eps / a
        wt = op.weights("lorentz", lam=lam)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        mu_ee, _ = P.chebyshev_moments(op, sites, N, len(w0.start_sites))
        l = P.ldos(mu_ee, wt, E)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        ld[N] = l
        res["sn_surface"][str(N)] = {"seconds": dt, "lambda": lam, "moments_per_s": sites.numel() * N / dt}
        log("S/N surface N=%d: %.2f s" % (N, dt))
    ref = ld[Ns[-1]]
    scale = float(ref.abs().max())
    for N in Ns[:-1]:
        res["sn_surface"][str(N)]["max_ldos_change_to_N16000_rel"] = float((ld[N] - ref).abs().max()) / scale
    res["sn_surface"]["workload"] = w0.name
    res["sn_surface"]["bounds_a"] = a
    op.close()

    for sc in (True, False):
        maps = {}
        for imp in (True, False):
            w = W.sns_impurity(superconducting=sc, impurity=imp)
            op = P.Operator.from_workload(w, dev)
            s = torch.as_tensor(w.start_sites, device=dev)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            mu_ee, _ = P.chebyshev_moments(op, s, w.N, w.tile)
            maps[imp] = P.ldos(mu_ee, op.weights(), torch.as_tensor(w.energies, device=dev))
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            op.close()
            res["sns_impurity"]["%s_%s_seconds" % ("sns" if sc else "normal", "imp" if imp else "clean")] = dt
        diff = (maps[True] - maps[False]).cpu().numpy()       # [441, 3]
        key = "sns" if sc else "normal"
        res["sns_impurity"][key + "_max_abs_dldos_per_energy"] = [float(v) for v in np.abs(diff).max(axis=0)]
        res["sns_impurity"][key + "_dldos_at_impurity_per_energy"] = [float(v) for v in diff[220]]
        log("%s impurity maps done" % key)
    return {"metric": METRIC, "value": res["sn_surface"]["16000"]["moments_per_s"], "unit": "moments/s",
            "n_gpus": 1, "higher_is_better": True, "dtype": "f64", "data": "synthetic",
            "config": {"workload": "the paper's two examples as synthetic lattices: planar N 380a / S 20a x "
                                   "500a surface LDOS (Lorentz kernel, eps = 0.001t, N = 2000..16000) and "
                                   "SC/N/SC 150a x 100a impurity LDOS maps (N = 2048)"},
            "examples": res}
