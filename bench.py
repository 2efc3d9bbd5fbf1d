"""Benchmark of the Chebyshev-BdG hot path on one MI355X.

One step = one iteration of the paper's self-consistency loop (plain mixing,
alpha = 1, FP64) over the whole 256x256 lattice of the disordered s-wave
workload (t = 1, mu = -0.4, U = 2.5, 1% of sites with V ~ U[-2, 2],
N = 1024 Jackson-damped moments, all 65536 sites in tiles of 1024 start
vectors):
  operator update with the current Delta -> batched Chebyshev moments of all
  65536 start vectors -> T = 0 gap equation with mixing and residual -> LDOS
  of every site at 64 energies.
Delta carries over from step to step, so the warm-up and timed steps are the
iterations of the self-consistent solve; their residuals stay on the device
until the timed region has ended.  `scf_solve` is that solve: the summed
iteration times up to the first residual below 1e-6 (iterations continue after
the timed steps if it has not converged by then).

Prints one JSON line.  `value` is moments/s (start vectors x N per second)
with every input resident in HBM.  The moments come from moment doubling
(N/2 recursion steps per tile) unless --algorithm direct asks for N - 1
steps; on this lattice (256 = 64 x 4 columns) the library advances a tile
seven steps per launch in the vector-contiguous passes, one wavefront per
start vector, each vector clipped to its own light cone, the pass writing the
doubling moments of its steps itself.  `roofline` reports the recursion
launches, timed with HIP events on the launch stream around each tile (the
tile's seed and coefficient kernels are charged to the recursion launches):
`achieved` counts the bytes each launch must move through HBM -- its input
and output vectors inside their light cones -- over the average launch
duration; `effective_GBps` counts instead the bytes of the plain one-step
recursion streamed over the whole lattice, which the multi-step passes and
the light cone avoid.  `traffic` is the HBM traffic per launch from the
rocprofv3 counters stored under profiles/ (null when they were taken on a
different kernel source).  `precision_form` runs the FP32-recursion form
(FP64 moment sums) and the FP64 path at N = 2048 on the same 16 tiles;
`differentiation_form` the 128x128 gradient (against a finite difference)
and the Newton solve on the whole Jacobian against plain mixing;
`cpu_baseline` times the CPU oracle on a bounded sample of start vectors.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Chebyshev moments/sec and HBM GB/s (FP64 vs FP32); self-consistent solve time"
HBM_PEAK_GBS = 8000.0


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for f in ("stencil.hpp", "step.hpp", "recursion.hip", "vcstep.hip", "common.hpp"):
        with open(os.path.join(ROOT, "paper_1007_1609_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def stored_traffic(kind: str):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if it
    was taken on the current kernel source."""
    path = os.path.join(ROOT, "profiles", "cheb_step_%s_traffic.txt" % kind)
    if not os.path.exists(path):
        return None
    rec = None
    with open(path) as f:
        for line in f:
            line = line.strip()
            if line.startswith("{"):
                rec = json.loads(line)
    if not rec or rec.get("kernel_source_hash") != kernel_source_hash():
        return None
    return rec.get("hbm_bytes_per_launch")


def cpu_baseline(w, a, b, n_sites: int, threads: int, target_s: float = 15.0):
    """Oracle moments/s on a bounded sample of start sites: a pilot of one
    site per thread sizes the timed sample to about target_s seconds."""
    import numpy as np

    import oracle
    H = oracle.workload_csr(w, a, b)
    if n_sites <= 0:
        pilot = np.linspace(0, w.L2 - 1, threads).astype(np.int32)
        t0 = time.perf_counter()
        oracle.moments(H, pilot, w.N, n_threads=threads)
        per_round = time.perf_counter() - t0
        n_sites = int(max(1, min(64, round(target_s / max(per_round, 1e-3))))) * threads
    sites = np.linspace(0, w.L2 - 1, n_sites).astype(np.int32)
    t0 = time.perf_counter()
    oracle.moments(H, sites, w.N, n_threads=threads)
    dt = time.perf_counter() - t0
    cores = oracle.max_threads()  # the threads that run used (set by the call above)
    # one thread on a few of the same sites (sets the oracle's thread count to 1)
    few = sites[:: max(1, n_sites // 3)][:3]
    t0 = time.perf_counter()
    oracle.moments(H, few, w.N, n_threads=1)
    dt1 = time.perf_counter() - t0
    model = ""
    try:
        with open("/proc/cpuinfo") as f:
            model = next((ln.split(":", 1)[1].strip() for ln in f if ln.startswith("model name")), "")
    except OSError:
        pass
    return {"value": n_sites * w.N / dt, "unit": "moments/s", "cores": cores,
            "kind": "oracle",
            "sample": "%d start sites spread over the same 256x256 lattice, N=%d, FP64 CSR "
                      "recursion, %.1f s" % (n_sites, w.N, dt),
            "value_1thread": len(few) * w.N / dt1, "sample_1thread": "%d of those sites, %.1f s" % (len(few), dt1),
            "cpu_model": model, "host_cpus": os.cpu_count()}


def log(msg):
    print("[bench] " + msg, file=sys.stderr, flush=True)


def copy_probe(dev, nbytes=2 << 30, reps=8):
    """Plain device-to-device copy of a known size: the reference for HBM
    counter scaling and the achievable copy bandwidth."""
    import torch
    src = torch.ones(nbytes // 8, dtype=torch.float64, device=dev)
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        dst.copy_(src)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    print(json.dumps({"probe": "device copy", "bytes_read_per_launch": nbytes,
                      "bytes_written_per_launch": nbytes, "launches": reps + 1,
                      "avg_ms": ms, "GBps_read_plus_write": 2 * nbytes / (ms / 1e3) / 1e9}), flush=True)


# Steps per launch of the vector-contiguous passes (FP64, FP32 recursion)
VC_STEPS = {8: 7, 4: 7}


def recursion_plan(real_uniform: bool, bt: int, s_bytes: int, Lx: int = 0, doubling: bool = True):
    """(kernel name, layout, steps per launch) of the passes the library
    issues for a tile of bt vectors.  Real operators with uniform hopping
    under moment doubling on lattices with Lx = 64 W (FP64: W = 1, 2, 4;
    FP32: W = 2, 4) take the vector-contiguous passes, seven steps per
    launch; other real uniform operators the vector-major
    passes, three steps per launch on tiles of more than 128 vectors and two
    on smaller ones; other operators one step per launch."""
    t = "double" if s_bytes == 8 else "float"
    W = Lx // 64 if Lx % 64 == 0 else 0
    if real_uniform and doubling and W in ((1, 2, 4) if s_bytes == 8 else (2, 4)):
        K = VC_STEPS[s_bytes]
        return "k_vc_pass<%s> (%d recursion steps per launch, one wavefront per vector)" % (t, K), "vc", K
    if not real_uniform:
        return "k_cheb_step<%s> (one recursion step per launch)" % t, "vm", 1
    if bt >= 129:
        return "k_cheb_step3<%s> (three recursion steps per launch)" % t, "vm", 3
    return "k_cheb_step2<%s> (two recursion steps per launch)" % t, "vm", 2


def launch_bytes(tile_events, sites_np, tile, n_tiles, w, steps_per_tile, real_uniform, s_bytes, doubling=True):
    """Launches, their summed duration (ms) and bytes over the timed tiles:
    the minimum each launch must move (vectors inside their light cones) and
    the bytes of the one-step streaming recursion over the whole lattice."""
    from bench_forms import recursion_traffic, vc_traffic
    launches = 0
    kern_ms = 0.0
    moved_b = streamed_b = 0.0
    kernel = None
    for k, (e0, e1, bt) in enumerate(tile_events):
        kern_ms += e0.elapsed_time(e1)
        bp = (bt + 63) // 64 * 64
        lo = (k % n_tiles) * tile
        name, layout, K = recursion_plan(real_uniform, bt, s_bytes, w.Lx, doubling)
        kernel = kernel or name
        ts = sites_np[lo:lo + bt]
        if layout == "vc":
            nl, moved, streamed = vc_traffic(ts, w.Lx, w.Ly, w.bc_x, w.bc_y, steps_per_tile, K)
            moved_b += moved * 2 * s_bytes
            streamed_b += streamed * 2 * s_bytes
        else:
            nl, moved, streamed = recursion_traffic(ts, w.Lx, w.Ly, w.bc_x, w.bc_y, steps_per_tile, K >= 2,
                                                    three_step=K == 3)
            moved_b += moved * 2 * bp * s_bytes
            streamed_b += streamed * 2 * bp * s_bytes
        launches += nl
    return kernel, launches, kern_ms, moved_b, streamed_b


def precision_form(w1, op, delta, dev, which, n_tiles=16, N=2048):
    """The FP32-recursion form (FP64 moment sums and everything downstream in
    FP64) against the FP64 path at the same N on the same tiles, with the
    operator at the given Delta: moments/s of both, the FP32 pass's HBM
    fraction on the bytes it must move, and the one-step Delta and LDOS
    errors of the FP32 form against the FP64 GPU path."""
    import numpy as np
    import torch
    import paper_1007_1609_amd as P
    tile = w1.tile
    n = n_tiles * tile
    sites = torch.arange(n, dtype=torch.int32, device=dev)
    sites_np = np.arange(n, dtype=np.int32)
    stream = torch.cuda.current_stream()
    op.update_delta(delta)
    wt = op.weights()
    energies = torch.linspace(-1.0, 1.0, 64, dtype=torch.float64, device=dev)
    res = {}
    out = {}
    for name, prec, s_bytes in (("fp64", P.CBDG_FP64, 8), ("fp32", P.CBDG_FP32_ACC64, 4)):
        ws = P.workspace(P.moments_workspace_bytes(op, tile, prec), dev)
        mu = (torch.empty((n, N), dtype=torch.float64, device=dev),
              torch.empty((n, N), dtype=torch.float64, device=dev))
        P.chebyshev_moments(op, sites[:tile], N, tile, prec, ws=ws, out=(mu[0][:tile], mu[1][:tile]))
        torch.cuda.synchronize()
        ev = []
        for k in range(n_tiles):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            P.chebyshev_moments(op, sites[k * tile:(k + 1) * tile], N, tile, prec, ws=ws,
                                out=(mu[0][k * tile:(k + 1) * tile], mu[1][k * tile:(k + 1) * tile]))
            e1.record(stream)
            ev.append((e0, e1, tile))
        torch.cuda.synchronize()
        kernel, launches, kern_ms, moved, streamed = launch_bytes(ev, sites_np, tile, n_tiles, w1, N // 2,
                                                                  True, s_bytes)
        gbs = moved / launches / (kern_ms / launches / 1e3) / 1e9
        res[name] = {"moments_per_s": n * N / (kern_ms / 1e3), "seconds": kern_ms / 1e3,
                     "kernel": kernel, "avg_launch_us": kern_ms / launches * 1e3,
                     "achieved_GBps": gbs, "frac": gbs / HBM_PEAK_GBS,
                     "effective_GBps": streamed / (kern_ms / 1e3) / 1e9}
        d_new, _ = P.gap_update(mu[1], wt, w1.U, delta[:n].contiguous())
        out[name] = (mu, d_new, P.ldos(mu[0], wt, energies))
        del ws
        torch.cuda.empty_cache()
        log("precision form %s: %.3g moments/s, %.0f GB/s moved" % (name, res[name]["moments_per_s"], gbs))
    torch.cuda.synchronize()
    m64, d64, l64 = out["fp64"]
    m32, d32, l32 = out["fp32"]
    res["fp32_over_fp64_same_N"] = res["fp32"]["moments_per_s"] / res["fp64"]["moments_per_s"]
    res["accuracy"] = {
        "reference": "FP64 recursion on the GPU at the same N (held to the oracle at 1e-10 by the parity tests)",
        "moments_max_abs_err": max(float((m32[0] - m64[0]).abs().max()), float((m32[1] - m64[1]).abs().max())),
        "delta_one_step_max_abs_err": float((d32 - d64).abs().max()),
        "ldos_max_err_rel_to_max": float((l32 - l64).abs().max() / l64.abs().max()),
        "bars": {"delta": 1e-6, "ldos_rel": 1e-5}}
    res["workload"] = ("%d tiles of %d start sites (sites 0..%d) of the 256x256 workload at N=%d, "
                       "operator at the %s Delta" % (n_tiles, tile, n - 1, N, which))
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--precision", choices=["fp64", "fp32"], default="fp64")
    ap.add_argument("--algorithm", choices=["auto", "direct", "doubling"], default="auto")
    ap.add_argument("--tiles", type=int, default=0, help="limit the number of tiles (0: whole lattice)")
    ap.add_argument("--cpu-sites", type=int, default=0, help="oracle sample size (0: sized to about 15 s)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-probe", action="store_true",
                    help="time a plain 2 GiB device copy instead (HBM calibration)")
    ap.add_argument("--form", choices=["scf-step", "complex", "adjoint", "scf", "paper", "resident"],
                    default="scf-step",
                    help="scf-step (default): iterations of the self-consistency loop of the 256x256 "
                         "workload; complex: 512x512 Peierls/d-wave LDOS workload; adjoint: 128x128 "
                         "gradients and Newton-Krylov; scf: a self-consistent solve of the 256x256 workload "
                         "by a chosen method; paper: the paper's two example geometries; resident: "
                         "cache-resident persistent tiles vs the streaming path (128x128)")
    ap.add_argument("--scf-method", choices=["plain", "nk-fd", "nk-jacobian", "anderson"], default="plain",
                    help="--form scf: plain mixing, Newton-Krylov with finite-difference products, "
                         "Newton on the whole Jacobian, or Anderson mixing")
    ap.add_argument("--scf-warmup-n", type=int, default=0,
                    help="--form scf --scf-method anderson: moments of the plain-mixing warm-up "
                         "evaluations (0: the workload's N)")
    ap.add_argument("--no-solve", action="store_true",
                    help="default form: do not continue the iterations past the timed steps to convergence")
    ap.add_argument("--no-precision-form", action="store_true",
                    help="default form: skip the FP32 / FP64 passes at N = 2048")
    ap.add_argument("--no-diff-form", action="store_true",
                    help="default form: skip the differentiation summary (128x128 gradient and Newton solve)")
    ap.add_argument("--no-scf", action="store_true",
                    help="--form adjoint: time the forward and reverse passes only (no solves)")
    ap.add_argument("--scf-fp32", action="store_true",
                    help="--form scf with plain or Anderson mixing: FP32 recursion until the residual "
                         "is below half the tolerance (5e-7), then FP64")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU: this build has no multi-GPU path "
              "(start vectors would shard across GPUs with one Delta all-gather per iteration)",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_1007_1609_amd as P
    import workloads as W

    dev = torch.device("cuda:0")
    if args.copy_probe:
        copy_probe(dev)
        return
    if args.form != "scf-step":
        import bench_forms
        line = {"complex": bench_forms.complex_form, "adjoint": bench_forms.adjoint_form,
                "scf": bench_forms.scf_form, "paper": bench_forms.paper_form,
                "resident": bench_forms.resident_form}[args.form](args, dev)
        print(json.dumps(line), flush=True)
        return
    N = 1024 if args.precision == "fp64" else 2048
    w = W.config1(N=N) if args.precision == "fp64" else W.config2()
    prec = P.CBDG_FP64 if args.precision == "fp64" else P.CBDG_FP32_ACC64
    s_bytes = 8 if args.precision == "fp64" else 4
    tile = w.tile
    n_tiles_all = (w.L2 + tile - 1) // tile
    n_tiles = n_tiles_all if args.tiles <= 0 else min(args.tiles, n_tiles_all)
    n_sites = min(w.L2, n_tiles * tile)

    op = P.Operator.from_workload(w, dev)
    a, b = op.bounds.a, op.bounds.b
    wts = op.weights()
    sites = torch.arange(n_sites, dtype=torch.int32, device=dev)
    alg = {"auto": P.CBDG_ALG_AUTO, "direct": P.CBDG_ALG_DIRECT, "doubling": P.CBDG_ALG_DOUBLING}[args.algorithm]
    doubling = alg == P.CBDG_ALG_DOUBLING or (alg == P.CBDG_ALG_AUTO and b == 0.0 and N >= 3)
    steps_per_tile = N // 2 if doubling else N - 1
    ws = P.workspace(P.moments_workspace_bytes(op, tile, prec, alg), dev)
    mu_ee = torch.empty((n_sites, N), dtype=torch.float64, device=dev)
    mu_he = torch.empty((n_sites, N), dtype=torch.float64, device=dev)
    full = n_sites == w.L2
    delta_full = torch.as_tensor(w.delta, device=dev).clone()
    delta = delta_full if full else torch.as_tensor(w.delta[:n_sites], device=dev).clone()
    nxt = torch.empty_like(delta)
    max_iter = max(60, args.warmup + args.steps)
    resid_hist = torch.full((max_iter,), float("nan"), dtype=torch.float64, device=dev)
    energies = torch.linspace(-1.0, 1.0, 64, dtype=torch.float64, device=dev)
    ldos = torch.empty((n_sites, 64), dtype=torch.float64, device=dev)
    stream = torch.cuda.current_stream()
    tile_events = []
    step_events = []

    def step(i, record):
        """Iteration i of the loop: Delta_{i+1} = F(Delta_i), residual into
        resid_hist[i] (stays on the device)."""
        nonlocal delta, nxt
        s0 = torch.cuda.Event(enable_timing=True)
        s1 = torch.cuda.Event(enable_timing=True)
        s0.record(stream)
        op.update_delta(delta if full else delta_full)
        for k in range(n_tiles):
            lo, hi = k * tile, min(n_sites, (k + 1) * tile)
            if record:
                e0 = torch.cuda.Event(enable_timing=True)
                e1 = torch.cuda.Event(enable_timing=True)
                e0.record(stream)
            P.chebyshev_moments(op, sites[lo:hi], N, tile, prec, ws=ws, out=(mu_ee[lo:hi], mu_he[lo:hi]),
                                algorithm=alg)
            if record:
                e1.record(stream)
                tile_events.append((e0, e1, hi - lo))
        P.gap_update(mu_he, wts, w.U, delta, 1.0, delta_out=nxt, resid=resid_hist[i:i + 1])
        P.ldos(mu_ee, wts, energies, out=ldos)
        delta, nxt = nxt, delta
        if not full:  # reduced runs only: the rest of the lattice keeps its Delta
            delta_full[:n_sites].copy_(delta)
        s1.record(stream)
        step_events.append((s0, s1))

    it = 0
    for i in range(args.warmup):
        step(it, False)
        it += 1
        torch.cuda.synchronize()
        log("warmup step %d done" % (i + 1))
    t_start = torch.cuda.Event(enable_timing=True)
    t_stop = torch.cuda.Event(enable_timing=True)
    t_start.record(stream)
    wall0 = time.perf_counter()
    for i in range(args.steps):
        step(it, True)
        it += 1
        if args.steps > 1:
            log("step %d enqueued" % (i + 1))
    t_stop.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - wall0
    ms_total = t_start.elapsed_time(t_stop)
    ms_per_step = ms_total / args.steps
    moments_per_step = n_sites * N
    value = moments_per_step * args.steps / (ms_total / 1e3)

    # Roofline of the dominant recursion kernel: the bytes each launch must
    # move (its input and output vectors inside their light cones, 2
    # components x s bytes per (site, vector)) over the average launch
    # duration; beside it the bytes the plain one-step recursion would stream
    # over the whole lattice (3 vectors per recursion step).
    sites_np = np.arange(n_sites, dtype=np.int32)
    kernel, launches, kern_ms, moved_b, streamed_b = launch_bytes(
        tile_events, sites_np, tile, n_tiles, w, steps_per_tile, True, s_bytes, doubling)
    avg_launch_ms = kern_ms / launches
    bytes_per_launch = moved_b / launches
    achieved = bytes_per_launch / (avg_launch_ms / 1e3) / 1e9
    effective = streamed_b / launches / (avg_launch_ms / 1e3) / 1e9
    traffic = stored_traffic(args.precision)
    ok = P.check_moments(mu_ee, mu_he, 1e-9 if args.precision == "fp64" else 1e-4)
    resid = resid_hist.cpu().numpy()
    log("timed steps done: %.1f ms/step, %.3g moments/s, %.0f GB/s moved" % (ms_per_step, value, achieved))

    line = {
        "metric": METRIC,
        "value": value,
        "unit": "moments/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.precision == "fp64" else "f32 recursion, f64 moments and sums",
        "data": "synthetic",
        "config": {
            "workload": "%s: 256x256 open lattice, 655 disordered sites V~U[-2,2] (seed 1), "
                        "t=1 mu=-0.4 U=2.5, N=%d Jackson, %d start sites in tiles of %d, "
                        "one iteration of the self-consistency loop (moments + gap update with plain "
                        "mixing + LDOS at 64 energies) per step"
                        % (w.name, N, n_sites, tile),
            "lattice": [w.Lx, w.Ly], "N": N, "start_sites": n_sites, "tile": tile,
            "precision": args.precision, "bounds_a": a,
            "algorithm": "doubling" if doubling else "direct", "recursion_steps_per_tile": steps_per_tile,
        },
        "roofline": {
            "kernel": kernel,
            "bound": "hbm",
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": traffic,
            "basis": "bytes each launch must move: its input and output vectors inside their light cones "
                     "(vector-contiguous passes: each vector's own diamond; vector-major passes: the box of "
                     "the tile's start sites; multi-step passes read 2 vectors and write 2)",
            "bytes_per_launch": bytes_per_launch,
            "effective_GBps": effective,
            "effective_frac": effective / HBM_PEAK_GBS,
            "effective_basis": "bytes of the one-step streaming recursion over the whole lattice, "
                               "3 vectors per recursion step",
            "avg_launch_us": avg_launch_ms * 1e3,
            "launches_timed": launches,
        },
        "moments_bounded": bool(ok),
        "wall_s_timed": wall,
    }
    if full and not args.no_solve:
        # continue the loop to convergence if the timed steps did not reach it
        while not (np.nanmin(resid[:it]) < 1e-6) and it < max_iter and np.isfinite(resid[it - 1]):
            step(it, False)
            it += 1
            torch.cuda.synchronize()
            resid = resid_hist.cpu().numpy()
            log("solve iteration %d residual %.3e" % (it, resid[it - 1]))
    if full:
        times = [a0.elapsed_time(a1) / 1e3 for a0, a1 in step_events[:it]]
        conv = np.flatnonzero(resid[:it] < 1e-6)
        k = int(conv[0]) + 1 if conv.size else it
        line["scf_solve"] = {
            "seconds": float(sum(times[:k])), "converged": bool(conv.size), "iterations": k,
            "residual": float(resid[k - 1]), "history": [float(r) for r in resid[:k]],
            "precision": args.precision,
            "method": "plain mixing alpha=1 (the paper's loop) from Delta=0.1, to max|F(Delta)-Delta| < 1e-6; "
                      "the warm-up and timed steps are its iterations, each timed with HIP events"}
        log("self-consistent solve: %s after %d iterations, %.1f s" % (
            "converged" if conv.size else "not converged", k, line["scf_solve"]["seconds"]))
    if args.precision == "fp64" and full and not args.no_precision_form:
        line["precision_form"] = precision_form(w, op, delta, dev,
                                                "self-consistent" if line["scf_solve"]["converged"] else "current")
    if args.precision == "fp64" and full and not args.no_diff_form:
        import bench_forms
        line["differentiation_form"] = bench_forms.differentiation_summary(dev)
    if not args.no_cpu_baseline:
        threads = int(os.environ.get("OMP_NUM_THREADS", "0") or 0) or os.cpu_count() or 1
        line["cpu_baseline"] = cpu_baseline(w, a, b, args.cpu_sites, threads)
    else:
        line["cpu_baseline"] = None
    op.close()
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
