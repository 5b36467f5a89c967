#!/usr/bin/env python3
"""Benchmark of the projection-step hot path on one MI355X.

Default workload (the one the fine-step metric is quoted on): the 128^3
lid-driven cavity, Re = 1000, dt = 5e-4, started from rest; a "step" is one
full fine projection step (predictor, Poisson right-hand side, Jacobi-PCG to
1e-10 relative residual, velocity correction) launched as one persistent
kernel.  W warm-up steps, then K timed steps; value = cells * K / wall time.

Other modes:
  --mode poisson   batched Poisson microbenchmark (32 x 128^3 right-hand
                   sides, a working set far above the 256 MB Infinity Cache)
  --mode parareal  Parareal on the 96^3 cavity (32 slices of 0.02, fine dt
                   5e-4, coarse dt --coarse-dt, mixed-precision F, FP64 G, jump < 1e-6)
                   against the serial FP64 fine solve on the GPU; with
                   --coarse-grid the coarse propagator runs on 48^3
  --mode obstacles uneven batch: 16 slices on each of 64^3, 96^3, 128^3 with
                   seeded cuboid obstacles, grouped launches, mixed precision
  --mode sim1      the paper's first test case: 32 x 32 x 5 quasi-2D cavity,
                   periodic in z, Re 1000, dt 1e-3 / 1e-2, FP64 Parareal;
                   defect against the serial fine solution per iteration
  --mode sim2      the paper's second test case: 32^3 cavity periodic in z
                   with 49 seeded cubes along the median plane, T = 24;
                   with --temporal-error also max |F_dt - F_dt/10| at T
  --mode copy      a plain device-to-device copy of 1 GiB (torch), the
                   reference for scaling rocprofv3 FETCH_SIZE / WRITE_SIZE

Prints ONE JSON line.  The CPU baseline (the plain FP64 oracle, N = 1 only)
times two fine steps of the same workload from the same state on the host.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0

# Algorithmic bytes per cell of the kernels' phases (FP64 state, 1-byte
# cell flags; face arrays counted as one entry per cell and component).
BYTES_CG_ITER = {"fp64": 66.0, "mixed": 34.0, "mixed_ru": 34.0}   # one CG iteration
BYTES_BICG_ITER = 139.0  # one BiCGStab iteration (FP64): phases of 49, 25 and 65 B
BYTES_SR_ITER = 81.0     # one single-reduction CG iteration (FP64): reads r, w, s, p, x, flags; writes r, w, s, p, x
BYTES_SR_START = 17.0    # the start of a single-reduction run: w = A M^-1 r (reads r, flags; writes w)
# The byte model of the method itself (not of this kernel's phase layout):
# per fine step 112 B per cell for momentum + right-hand side + correction,
# and 80 B per cell per FP64 CG iteration (read r, d, write d, q; read x, d,
# r, q, write x, r).
MODEL_STEP_FIXED, MODEL_CG_ITER = 112.0, 80.0
# a projection of the adjoint sweep: the step without its momentum predictor
# (read u, v, w, write F: 48 B per cell)
MODEL_PROJECT_FIXED = MODEL_STEP_FIXED - 48.0


def _prec(args):
    from paper_1705_06149_amd import nsp
    return {"fp64": nsp.FP64, "mixed": nsp.MIXED, "mixed_ru": nsp.MIXED_RU}[args.precision]


# reliable updates: replace the FP32 residual once it has fallen by this
# factor.  Measured (c3 batched sweep / 128^3 step): 1e-2 5.95 s / 123.2 M,
# 1e-3 5.65 s / 124.6 M with the same iteration counts; at 1e-4 the FP32
# recursion stagnates (790 iterations per 128^3 step instead of 635)
RU_DELTA = 1e-3


def _eta(args):
    """inner tolerance (restarted mixed solves) or update factor (reliable updates)"""
    if args.eta is not None:
        return args.eta
    return RU_DELTA if args.precision == "mixed_ru" else 1e-5


def _max_outer(args):
    return 64 if args.precision == "mixed_ru" else 8


def _parareal_fine_opts(args, nsp):
    """Poisson options of the batched fine sweeps of the Parareal modes"""
    prec = {"fp64": nsp.FP64, "mixed": nsp.MIXED, "mixed_ru": nsp.MIXED_RU}[args.parareal_fine]
    eta = args.eta if args.eta is not None else (RU_DELTA if args.parareal_fine == "mixed_ru" else 1e-5)
    return nsp.PoissonOpts(rtol=1e-10, prec=prec, inner_rtol=eta, max_outer=64 if args.parareal_fine == "mixed_ru"
                           else 8, extrapolate=args.parareal_extrapolate)


def _model_bytes(args, cells, iters_per_step, sweeps_per_launch):
    """The method's algorithmic bytes of one fine-step launch"""
    if args.precision == "fp64":
        return cells * (MODEL_STEP_FIXED + MODEL_CG_ITER * iters_per_step)
    return cells * (MODEL_STEP_FIXED + 0.5 * MODEL_CG_ITER * iters_per_step) + cells * 40.0 * sweeps_per_launch


def _solver(args):
    from paper_1705_06149_amd import nsp
    return {"pcg": nsp.PCG, "bicgstab": nsp.BICGSTAB, "pcg_sr": nsp.PCG_SR}[args.solver]


def _solver_name(args):
    return {"pcg": "Jacobi-PCG", "bicgstab": "Jacobi-BiCGStab",
            "pcg_sr": "Jacobi-PCG, single reduction"}[args.solver]


def _bytes_per_iter(args):
    if args.solver == "bicgstab":
        return BYTES_BICG_ITER
    if args.solver == "pcg_sr":
        return BYTES_SR_ITER
    return BYTES_CG_ITER[args.precision]
BYTES_STEP_FIXED = {"fp64": 212.0, "mixed": 212.0, "mixed_ru": 212.0}  # momentum, rhs, init/true, correction, gauge
BYTES_MIXED_SWEEP = 65.0  # mixed: one FP64 residual + cast + update sweep


def _kernel_source_hash():
    h = hashlib.sha256()
    for f in ("paper_1705_06149_amd/csrc/nsp_kernels.hip", "paper_1705_06149_amd/csrc/nsp_internal.h"):
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def _traffic_from_profile(name):
    """HBM bytes per launch measured with rocprofv3 counters, if the committed
    summary was taken on the current kernel source; else None."""
    path = os.path.join(ROOT, "profiles", name)
    if not os.path.exists(path):
        return None
    rec = {}
    with open(path) as fh:
        for line in fh:
            if "=" in line and not line.startswith("#"):
                k, v = line.split("=", 1)
                rec[k.strip()] = v.strip()
    if rec.get("kernel_source_sha256_16") != _kernel_source_hash():
        return None
    try:
        return float(rec["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def _log(*a):
    """Progress line on stderr (long modes print one per stage)."""
    print("[bench]", *a, file=sys.stderr, flush=True)


def _sync():
    import torch
    torch.cuda.synchronize()


def _fine_solid(args):
    """--obstacles: the 128^3 cavity of the obstacle batch (seed 3, cuboids
    of 4..12 cells, >= 5 % solid)."""
    if not args.obstacles:
        return None
    from paper_1705_06149_amd import inputs
    return inputs.obstacle_mask(128, seed=3)


def _fine_workload(args):
    if not args.obstacles:
        return "cavity128_re1000"
    return "cavity128_obstacles_%s_re1000" % ("slip" if args.slip else "noslip")


def bench_fine(args):
    import torch
    from paper_1705_06149_amd import nsp

    n, re_, dt = 128, 1000.0, 5e-4
    prec = _prec(args)
    opts = nsp.PoissonOpts(rtol=1e-10, maxit=100000, prec=prec, inner_rtol=_eta(args),
                           max_outer=_max_outer(args), solver=_solver(args), extrapolate=args.extrapolate)
    # equal launches of S steps: the largest divisor of the timed steps up to
    # --steps-per-launch (a graph replays one step)
    S = 1 if args.graph else math.gcd(args.steps, max(args.steps_per_launch, 1))
    h = nsp.Handle(n, n, n, re=re_, max_batch=1, solid=_fine_solid(args), slip_obstacles=args.slip)
    y = h.zeros_state(1)
    t = 0.0
    for _ in range(args.warmup):
        h.fine_step(y, t, t + dt, dt, opts)
        t += dt
    host_state = tuple(a[0].cpu().numpy().copy() for a in y)
    _sync()
    iters = 0
    launch_ms = []
    K = args.steps
    outer_per_launch = None
    if args.graph:
        # one step recorded as a HIP graph; K replays enqueued back to back,
        # read back once
        g = h.fine_step_graph(y, t, t + dt, dt, opts)
        _sync()
        t0 = time.perf_counter()
        for _ in range(K):
            g.launch()
        info = g.finish()
        _sync()
        wall = time.perf_counter() - t0
        t += K * dt
        iters = info[0]["iters"]
        launch_ms = [h.last_launch_ms() / K]
        outer_per_launch = info[0]["outer"] / K
        g.close()
    else:
        # K steps as K / S calls of S steps each (S = --steps-per-launch)
        t0 = time.perf_counter()
        for _ in range(K // S):
            info = h.fine_step(y, t, t + S * dt, dt, opts)
            t += S * dt
            iters += info[0]["iters"]
            launch_ms.append(h.last_launch_ms())
        _sync()
        wall = time.perf_counter() - t0
        outer_per_launch = info[0]["outer"]
    cells = n ** 3
    value = cells * K / wall
    err_vs_fp64 = None
    if args.precision != "fp64" and args.compare_fp64:
        # the same K steps in FP64 from the same warmed state
        import torch
        y64 = tuple(torch.from_numpy(a[None].copy()).cuda() for a in host_state)
        o64 = nsp.PoissonOpts(rtol=1e-10, maxit=100000, prec=nsp.FP64)
        h.fine_step(y64, t - K * dt, t, dt, o64)
        err_vs_fp64 = float(torch.sqrt(sum(((y[c] - y64[c]) ** 2).sum() for c in range(3)) /
                                       sum((y64[c] ** 2).sum() for c in range(3))))
    # bytes by the kernels' own phase layout
    per_iter = _bytes_per_iter(args)
    fixed = BYTES_STEP_FIXED[args.precision] + (BYTES_SR_START if args.solver == "pcg_sr" else 0.0)
    layout_bytes = S * cells * (fixed + per_iter * iters / K)
    if args.precision != "fp64":
        layout_bytes += cells * BYTES_MIXED_SWEEP * outer_per_launch
    avg_launch_s = float(np.mean(launch_ms)) * 1e-3
    # the roofline's algorithmic bytes: the method's byte model per cell and
    # step, 112 B plus 80 B per FP64 CG iteration (mixed: 40 B per FP32
    # iteration and 40 B per FP64 correction sweep), independent of how the
    # kernels lay the phases out or keep vectors on chip
    model_bytes = S * _model_bytes(args, cells, iters / K, outer_per_launch / S)
    achieved = model_bytes / avg_launch_s / 1e9
    sfx = "" if args.solver == "pcg" else "_" + args.solver
    traffic = (_traffic_from_profile("k_persistent_cavity128_%s%s_pmc.txt" % (args.precision, sfx))
               if not args.obstacles else None)
    out = {
        "metric": "fine-step cell-updates/s",
        "value": value,
        "unit": "cell-updates/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * wall / K,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.precision == "fp64" else "f32+f64",
        "data": "synthetic",
        "config": {"workload": _fine_workload(args), "grid": [n, n, n], "re": re_, "dt": dt,
                   "start": "rest, after %d warm-up steps" % args.warmup,
                   "poisson": _solver_name(args) + " rtol 1e-10" +
                   (", warm start 2 p^s - p^(s-1)" if args.extrapolate else ", warm start p^s"),
                   "precision": args.precision},
        "launch": ("one HIP graph replayed per step, read back once" if args.graph else
                   "one call per step" if S == 1 else "one call per %d steps" % S),
        "cg_iters_per_step": iters / K,
        "inner_rtol": _eta(args) if args.precision != "fp64" else None,
        "velocity_rel_l2_vs_fp64": err_vs_fp64,
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                     "frac": achieved / PEAK_HBM_GBS, "traffic": traffic,
                     "kernel": "k_persistent (%d fused fine step%s per launch)" % (S, "" if S == 1 else "s"),
                     "avg_launch_ms": 1e3 * avg_launch_s,
                     "algorithmic_bytes_per_launch": model_bytes,
                     "byte_model": "112 + 80 I B per cell and step (mixed: 112 + 40 I32 + 40 per sweep)",
                     "kernel_layout_bytes_per_launch": layout_bytes,
                     "kernel_layout_frac": layout_bytes / avg_launch_s / 1e9 / PEAK_HBM_GBS},
    }
    out["hbm_measured_GB_per_s"] = traffic / avg_launch_s / 1e9 if traffic else None
    h.close()
    return out, host_state, t


def cpu_baseline_fine(args, host_state, t):
    """The oracle as it stands, one fine step of the same workload from the
    same state, timed on the host cores."""
    from oracle import oracle as O

    O.build()
    n = 128
    g = O.Grid(n, n, n, re=1000.0, solid=_fine_solid(args), slip_obstacles=args.slip)
    prec = {"fp64": 0, "mixed": 1, "mixed_ru": 2}[args.precision]
    threads = O.num_threads()
    runs = {}
    for label, nthr, nsteps in (("all", threads, 2), ("one", 1, 1)):
        O.set_num_threads(nthr)
        t0 = time.perf_counter()
        _, iters, _, st = O.fine_steps(g, host_state, nsteps, 5e-4, prec=prec, rtol=1e-10, eta=_eta(args),
                                       max_outer=_max_outer(args), extrapolate=args.extrapolate)
        runs[label] = (nsteps, time.perf_counter() - t0, int(iters.sum()))
    O.set_num_threads(threads)
    (ns, wall, it), (n1, wall1, it1) = runs["all"], runs["one"]
    return {"value": ns * n ** 3 / wall, "unit": "cell-updates/s", "cores": threads, "kind": "oracle",
            "sample": "%d fine steps of the 128^3 cavity from the benchmark's warmed state "
                      "(%d CG iterations, %.1f s, %d threads)" % (ns, it, wall, threads),
            "one_core": {"value": n1 * n ** 3 / wall1, "cores": 1,
                         "sample": "%d fine step from the same state (%d CG iterations, %.1f s)" % (n1, it1, wall1)},
            "cpu_model": _cpu_model()}


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def bench_poisson(args):
    import torch
    from paper_1705_06149_amd import nsp

    n, B = 128, 32
    prec = nsp.MIXED if args.precision != "fp64" else nsp.FP64
    its = 100
    h = nsp.Handle(n, n, n, re=1000.0, max_batch=B)
    g = torch.Generator(device="cuda").manual_seed(0)
    b = torch.randn((B, n, n, n), dtype=torch.float64, device="cuda", generator=g)
    p = torch.zeros_like(b)
    opts = nsp.PoissonOpts(rtol=0.0, maxit=its, prec=prec, inner_rtol=1e-30, max_outer=1, solver=_solver(args))
    for _ in range(args.warmup):
        p.zero_()
        h.poisson_solve(b, p, opts, check=False)
    _sync()
    ms = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        p.zero_()
        info = h.poisson_solve(b, p, opts, check=False)
        ms.append(h.last_launch_ms())
    _sync()
    wall = time.perf_counter() - t0
    cells = B * n ** 3
    per_launch = cells * _bytes_per_iter(args) * its
    if args.precision != "fp64":
        per_launch += cells * BYTES_MIXED_SWEEP * info[0]["outer"]
    achieved = per_launch / (np.mean(ms) * 1e-3) / 1e9
    # the method's byte model: 80 B per cell and CG iteration (FP32: 40 B)
    model = cells * its * (MODEL_CG_ITER if args.precision == "fp64" else 0.5 * MODEL_CG_ITER)
    model_achieved = model / (np.mean(ms) * 1e-3) / 1e9
    out = {
        "metric": "Poisson HBM GB/s", "value": achieved, "unit": "GB/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": 1e3 * wall / args.steps, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64" if args.precision == "fp64" else "f32",
        "data": "synthetic",
        "config": {"workload": "poisson_32x128cube", "batch": B, "grid": [n, n, n], "iterations": its,
                   "solver": args.solver, "precision": args.precision},
        "roofline": {"bound": "hbm", "achieved": model_achieved, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                     "frac": model_achieved / PEAK_HBM_GBS,
                     "traffic": _traffic_from_profile("k_persistent_poisson32x128_%s%s_pmc.txt" % (
                         args.precision, "" if args.solver == "pcg" else "_" + args.solver)),
                     "kernel": "k_persistent (%d CG iterations on %d grids per launch)" % (its, B),
                     "avg_launch_ms": float(np.mean(ms)), "algorithmic_bytes_per_launch": model,
                     "byte_model": "80 B per cell and CG iteration (FP32 inner: 40 B)",
                     "kernel_layout_bytes_per_launch": per_launch,
                     "kernel_layout_frac": achieved / PEAK_HBM_GBS},
    }
    t = out["roofline"]["traffic"]
    out["hbm_measured_GB_per_s"] = t / (np.mean(ms) * 1e-3) / 1e9 if t else None
    h.close()
    return out


def bench_parareal(args):
    import torch
    from paper_1705_06149_amd import nsp

    n, re_, dt, N, T = 96, 1000.0, 5e-4, 32, 0.64
    cgrid = args.coarse_grid
    # on the 48^3 coarse grid the configuration's coarse step 1e-2 is stable
    # (Courant number 0.48, diffusion term 0.14)
    DT = args.coarse_dt if args.coarse_dt is not None else (1e-2 if cgrid else 5e-3)
    tol = 1e-6
    fine64 = nsp.PoissonOpts(rtol=1e-10, prec=nsp.FP64, extrapolate=args.parareal_extrapolate)
    mixed = _parareal_fine_opts(args, nsp)
    # the serial coarse sweep is a batch of one, latency-bound: FP32 saves no
    # time there and each defect-correction restart adds iterations, so G
    # solves in FP64 (measured at 96^3: 2.0 s per sweep vs 2.8 s mixed)
    coarse = nsp.PoissonOpts(rtol=args.coarse_rtol, prec=nsp.FP64)
    h = nsp.Handle(n, n, n, re=re_, max_batch=N)
    hc = nsp.Handle(n // 2, n // 2, n // 2, re=re_, max_batch=1) if cgrid else None
    if args.coarse_upwind:
        (hc if cgrid else h).set_coarse_convection(nsp.CONV_UPWIND)
    # serial FP64 fine solve, batch 1, over [0, T]
    y = h.zeros_state(1)
    _sync()
    t0 = time.perf_counter()
    for s in range(N):
        h.fine_step(y, s * T / N, (s + 1) * T / N, dt, fine64)
        if s % 8 == 7:
            _log("serial fp64 slice %d/%d  %.1f s" % (s + 1, N, time.perf_counter() - t0))
    _sync()
    serial = time.perf_counter() - t0
    ref = tuple(a[0].clone() for a in y)
    # batched mixed-precision Parareal, launch shape autotuned for the full batch
    tuned_wg, tuned_planes, tuned_items = h.autotune(N, mixed.prec)
    shapes = h.shapes()
    Y = tuple(torch.zeros((N + 1,) + s, dtype=torch.float64, device="cuda") for s in shapes)
    Fk = tuple(torch.zeros((N,) + s, dtype=torch.float64, device="cuda") for s in shapes)
    Gk = tuple(torch.zeros((N,) + s, dtype=torch.float64, device="cuda") for s in shapes)
    _sync()
    h.launch_stats(reset=True)
    if hc is not None:
        hc.launch_stats(reset=True)
    t0 = time.perf_counter()
    if cgrid:
        h.parareal_start_cgrid(hc, Y, Gk, N, 0.0, T, DT, coarse)
    else:
        h.parareal_start(Y, Gk, N, 0.0, T, DT, coarse)
    jumps = []
    k = 0
    iter_s = []
    while True:
        ti = time.perf_counter()
        if cgrid:
            jv, jp = h.parareal_iterate_cgrid(hc, Y, Fk, Gk, N, k, 0.0, T, dt, DT, mixed, coarse)
        else:
            jv, jp = h.parareal_iterate(Y, Fk, Gk, N, k, 0.0, T, dt, DT, mixed, coarse)
        iter_s.append(time.perf_counter() - ti)
        jumps.append(jv)
        _log("parareal iteration %d: %.1f s, jump %.3e" % (k, iter_s[-1], jv))
        k += 1
        if jv < tol or k >= N or k >= args.max_iters:
            break
    _sync()
    par = time.perf_counter() - t0
    err = float(torch.sqrt(sum(((Y[c][N] - ref[c]) ** 2).sum() for c in range(3)) /
                           sum((ref[c] ** 2).sum() for c in range(3))))
    cells = n ** 3
    nf = int(round(T / dt))
    kst = [h.launch_stats()["fine"]] + ([hc.launch_stats()["fine"]] if hc is not None else [])
    # one batched fine sweep (every slice over one slice length) from the
    # Parareal slice starts, in FP64 and in the run's fine precision
    sweep = {}
    for name, o in (("fp64", fine64), (args.parareal_fine, mixed)):
        ys = tuple(Y[c][:N].clone() for c in range(4))
        _sync()
        t1 = time.perf_counter()
        inf = h.fine_step(ys, 0.0, T / N, dt, o)
        _sync()
        sweep[name] = {"s": time.perf_counter() - t1,
                       "cg_iters_per_slice_step": sum(x["iters"] for x in inf) / float(nf)}
        _log("batched fine sweep %s: %.2f s" % (name, sweep[name]["s"]))
    klayout = sum(_stats_bytes(x, BYTES_STEP_FIXED["fp64"]) for x in kst)
    kbytes = sum(_stats_model_bytes(x) for x in kst)
    kms = sum(x["ms"] for x in kst)
    klaunch = sum(x["launches"] for x in kst)
    kach = kbytes / (kms * 1e-3) / 1e9
    out = {
        "metric": "Parareal speedup vs serial fine", "value": serial / par, "unit": "x", "n_gpus": 1,
        "steps": nf, "warmup": 0, "ms_per_step": 1e3 * par / nf, "higher_is_better": True, "scaling": "strong",
        "vs_baseline": None, "dtype": "f32+f64", "data": "synthetic",
        "roofline": {"bound": "hbm", "achieved": kach, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                     "frac": kach / PEAK_HBM_GBS,
                     "traffic": None if cgrid else _traffic_from_profile("k_persistent_parareal96_pmc.txt"),
                     "kernel": "k_persistent (batched fine sweeps and coarse steps of the Parareal run)",
                     "avg_launch_ms": kms / max(klaunch, 1), "launches": klaunch,
                     "algorithmic_bytes_per_launch": kbytes / max(klaunch, 1),
                     "kernel_layout_bytes_per_launch": klayout / max(klaunch, 1),
                     "kernel_layout_frac": klayout / (kms * 1e-3) / 1e9 / PEAK_HBM_GBS,
                     "k_persistent_share_of_wall": kms * 1e-3 / par},
        "config": {"workload": "parareal96_re1000", "grid": [n, n, n], "slices": N, "T": T, "dt": dt, "DT": DT,
                   "jump_tol": tol, "coarse_grid": [n // 2] * 3 if cgrid else [n, n, n],
                   "coarse_convection": "upwind" if args.coarse_upwind else "smart",
                   "fine_poisson": "%s, inner %g%s" % (args.parareal_fine, mixed.inner_rtol,
                                                       ", extrapolated start" if args.parareal_extrapolate else ""), "coarse_poisson": "fp64, rtol %g" % args.coarse_rtol},
        "parareal_iterations": k, "jumps": jumps, "iteration_s": iter_s, "serial_fp64_s": serial, "parareal_s": par,
        "batched_fine_sweep": sweep,
        "serial_equiv_cell_updates_per_s": cells * nf / par,
        "executed_cell_updates_per_s": sum(x["cell_steps"] for x in kst) / par,
        "end_state_rel_l2_vs_serial_fp64": err,
        "bound_paper_eq8": N / k,
        "autotuned_launch": {"workgroups": tuned_wg, "cg_tile_planes": tuned_planes,
                             "cg_rows_per_thread": tuned_items},
    }
    h.close()
    if hc is not None:
        hc.close()
    return out


def bench_obstacles(args):
    """Uneven batch: 16 Parareal slices on each of 64^3, 96^3 and 128^3 cavities
    with seeded cuboid obstacles, every fine sweep one grouped launch."""
    import torch
    from paper_1705_06149_amd import inputs, nsp

    grids = [(64, 1), (96, 2), (128, 3)]
    re_, dt, N, T = 1000.0, 5e-4, 16, 0.32
    DT = args.coarse_dt if args.coarse_dt is not None else 2.5e-3
    tol = 1e-6
    fine64 = nsp.PoissonOpts(rtol=1e-10, prec=nsp.FP64, extrapolate=args.parareal_extrapolate)
    mixed = _parareal_fine_opts(args, nsp)
    # the serial coarse sweep is a batch of one, latency-bound: FP32 saves no
    # time there and each defect-correction restart adds iterations, so G
    # solves in FP64 (measured at 96^3: 2.0 s per sweep vs 2.8 s mixed)
    coarse = nsp.PoissonOpts(rtol=args.coarse_rtol, prec=nsp.FP64)
    hs = [nsp.Handle(n, n, n, re=re_, solid=inputs.obstacle_mask(n, seed), max_batch=N) for n, seed in grids]
    if args.coarse_upwind:
        for h in hs:
            h.set_coarse_convection(nsp.CONV_UPWIND)
    # serial FP64 fine solve of each grid, batch 1
    refs, serial = [], 0.0
    for (n, _), h in zip(grids, hs):
        y = h.zeros_state(1)
        _sync()
        t0 = time.perf_counter()
        for s in range(N):
            h.fine_step(y, s * T / N, (s + 1) * T / N, dt, fine64)
            _log("serial fp64 %d^3 slice %d/%d  %.1f s" % (n, s + 1, N, time.perf_counter() - t0))
        _sync()
        serial += time.perf_counter() - t0
        refs.append(tuple(a[0].clone() for a in y))
    Ys = [tuple(torch.zeros((N + 1,) + s, dtype=torch.float64, device="cuda") for s in h.shapes()) for h in hs]
    Fks = [tuple(torch.zeros((N,) + s, dtype=torch.float64, device="cuda") for s in h.shapes()) for h in hs]
    Gks = [tuple(torch.zeros((N,) + s, dtype=torch.float64, device="cuda") for s in h.shapes()) for h in hs]
    _sync()
    for h in hs:
        h.launch_stats(reset=True)
    t0 = time.perf_counter()
    nsp.group_parareal_start(hs, Ys, Gks, N, 0.0, T, DT, coarse)
    k, jumps, iter_s = 0, [], []
    while True:
        ti = time.perf_counter()
        j = nsp.group_parareal_iterate(hs, Ys, Fks, Gks, N, k, 0.0, T, dt, DT, mixed, coarse)
        iter_s.append(time.perf_counter() - ti)
        jumps.append([jv for jv, _ in j])
        _log("parareal iteration %d: %.1f s, jumps %s" % (k, iter_s[-1], jumps[-1]))
        k += 1
        if max(jv for jv, _ in j) < tol or k >= N or k >= args.max_iters:
            break
    _sync()
    par = time.perf_counter() - t0
    errs = []
    for Y, ref in zip(Ys, refs):
        errs.append(float(torch.sqrt(sum(((Y[c][N] - ref[c]) ** 2).sum() for c in range(3)) /
                                     sum((ref[c] ** 2).sum() for c in range(3)))))
    cells = sum(n ** 3 for n, _ in grids)
    nf = int(round(T / dt))
    # grouped launches count on the first handle
    kst = [h.launch_stats()["fine"] for h in hs]
    klayout = sum(_stats_bytes(x, BYTES_STEP_FIXED["fp64"]) for x in kst)
    kbytes = sum(_stats_model_bytes(x) for x in kst)
    kms = sum(x["ms"] for x in kst)
    klaunch = sum(x["launches"] for x in kst)
    kach = kbytes / (kms * 1e-3) / 1e9
    out = {
        "metric": "Parareal speedup vs serial fine", "value": serial / par, "unit": "x", "n_gpus": 1,
        "steps": nf, "warmup": 0, "ms_per_step": 1e3 * par / nf, "higher_is_better": True, "scaling": "strong",
        "vs_baseline": None, "dtype": "f32+f64", "data": "synthetic",
        "roofline": {"bound": "hbm", "achieved": kach, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                     "frac": kach / PEAK_HBM_GBS, "traffic": None,
                     "kernel": "k_persistent (grouped fine sweeps and coarse steps of the Parareal run)",
                     "avg_launch_ms": kms / max(klaunch, 1), "launches": klaunch,
                     "algorithmic_bytes_per_launch": kbytes / max(klaunch, 1),
                     "kernel_layout_bytes_per_launch": klayout / max(klaunch, 1),
                     "kernel_layout_frac": klayout / (kms * 1e-3) / 1e9 / PEAK_HBM_GBS,
                     "k_persistent_share_of_wall": kms * 1e-3 / par},
        "config": {"workload": "obstacles_64_96_128", "grids": [n for n, _ in grids], "mask_seeds": [s for _, s in grids],
                   "slices_per_grid": N, "T": T, "dt": dt, "DT": DT, "jump_tol": tol,
                   "batch_cells": N * cells, "coarse_poisson": "fp64, rtol %g" % args.coarse_rtol},
        "parareal_iterations": k, "jumps_per_grid": jumps, "iteration_s": iter_s, "serial_fp64_s": serial,
        "parareal_s": par, "serial_equiv_cell_updates_per_s": cells * nf / par,
        "executed_cell_updates_per_s": sum(x["cell_steps"] for x in kst) / par,
        "end_state_rel_l2_vs_serial_fp64": errs,
    }
    for h in hs:
        h.close()
    return out


def paper_sim_config(sim):
    """Parameters of the paper's test cases (Sec. 3, Table 1)."""
    if sim == 1:
        return {"domain": [1.0, 1.0, 0.1], "cells": [32, 32, 5], "T": 80.0, "coarse_dt": 1e-2, "fine_dt": 1e-3,
                "re": 1000.0, "obstacles": 0}
    return {"domain": [1.0, 1.0, 1.0], "cells": [32, 32, 32], "T": 24.0, "coarse_dt": 1e-2, "fine_dt": 1e-3,
            "re": 1000.0, "obstacles": 49}


def bench_paper_sim(args, sim):
    """The paper's test cases (Sec. 3, Table 1), periodic in z, Re 1000, lid
    u = 1, fine dt 1e-3, coarse dt 1e-2, FP64:
      Sim 1: a quasi-2D cavity of 32 x 32 x 5 cells on [0,1]^2 x [0,0.1], T = 80;
      Sim 2: 32^3 cells on [0,1]^3 with 49 cubes along the median plane, T = 24
             (seeded cubes: the paper does not give their layout).
    Reports, per Parareal iteration, the defect of every slice end against
    the serial fine solution (max norm over u, v, w and over p), the quantity
    the paper plots against N_it; with --temporal-error also the temporal
    error of the fine propagator at T, max |F_dt - F_dt/10| over u, v, w (and
    p), the threshold the paper compares the defect with."""
    import torch
    from paper_1705_06149_amd import inputs, nsp

    c = paper_sim_config(sim)
    nx, ny, nz = c["cells"]
    lz, T_def, re_, dt, DT = c["domain"][2], c["T"], c["re"], c["fine_dt"], c["coarse_dt"]
    solid = inputs.median_plane_cubes(nx, seed=49, count=c["obstacles"]) if c["obstacles"] else None
    N = args.slices
    T = args.sim_t if args.sim_t is not None else T_def
    o64 = nsp.PoissonOpts(rtol=1e-10, prec=nsp.FP64)
    h = nsp.Handle(nx, ny, nz, lz=lz, re=re_, solid=solid, max_batch=N, periodic_z=True)
    shapes = h.shapes()
    ref = tuple(torch.zeros((N + 1,) + s, dtype=torch.float64, device="cuda") for s in shapes)
    y = h.zeros_state(1)
    _sync()
    t0 = time.perf_counter()
    for n in range(N):
        h.fine_step(y, n * T / N, (n + 1) * T / N, dt, o64)
        for c in range(4):
            ref[c][n + 1].copy_(y[c][0])
        _log("serial fine slice %d/%d  %.1f s" % (n + 1, N, time.perf_counter() - t0))
    _sync()
    serial = time.perf_counter() - t0
    Y = tuple(torch.zeros((N + 1,) + s, dtype=torch.float64, device="cuda") for s in shapes)
    Fk = tuple(torch.zeros((N,) + s, dtype=torch.float64, device="cuda") for s in shapes)
    Gk = tuple(torch.zeros((N,) + s, dtype=torch.float64, device="cuda") for s in shapes)

    def defect():
        dv = max(float((Y[c][1:] - ref[c][1:]).abs().max()) for c in range(3))
        return dv, float((Y[3][1:] - ref[3][1:]).abs().max())

    _sync()
    h.launch_stats(reset=True)
    t0 = time.perf_counter()
    h.parareal_start(Y, Gk, N, 0.0, T, DT, o64)
    defects = [defect()]
    jumps = []
    iter_wall = []
    k = 0
    while k < min(N, args.max_iters):
        jv, jp = h.parareal_iterate(Y, Fk, Gk, N, k, 0.0, T, dt, DT, o64, o64)
        jumps.append((jv, jp))
        k += 1
        defects.append(defect())
        _sync()
        iter_wall.append(time.perf_counter() - t0)
        _log("parareal iteration %d: jump %.3e, defect vs serial u,v,w %.3e p %.3e  %.1f s" %
             (k, jv, defects[-1][0], defects[-1][1], iter_wall[-1]))
    _sync()
    par = time.perf_counter() - t0
    nf = int(round(T / dt))
    kst = h.launch_stats()["fine"]
    klayout = _stats_bytes(kst, BYTES_STEP_FIXED["fp64"])
    kbytes = _stats_model_bytes(kst)
    kach = kbytes / max(kst["ms"] * 1e-3, 1e-12) / 1e9
    out = {
        "metric": "Parareal speedup vs serial fine", "value": serial / par, "unit": "x", "n_gpus": 1,
        "steps": nf, "warmup": 0, "ms_per_step": 1e3 * par / nf, "higher_is_better": True, "scaling": "strong",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "roofline": {"bound": "hbm", "achieved": kach, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                     "frac": kach / PEAK_HBM_GBS, "traffic": None,
                     "kernel": "k_persistent (Parareal sweeps; a small grid, so latency-bound)",
                     "avg_launch_ms": kst["ms"] / max(kst["launches"], 1), "launches": kst["launches"],
                     "algorithmic_bytes_per_launch": kbytes / max(kst["launches"], 1),
                     "kernel_layout_bytes_per_launch": klayout / max(kst["launches"], 1),
                     "k_persistent_share_of_wall": kst["ms"] * 1e-3 / par},
        "config": {"workload": "paper_sim%d" % sim, "grid": [nx, ny, nz], "domain": [1.0, 1.0, lz],
                   "periodic_z": True, "obstacles": "49 seeded cubes, median plane" if solid is not None else None,
                   "re": re_, "slices": N, "T": T, "dt": dt, "DT": DT},
        "parareal_iterations": k, "serial_fp64_s": serial, "parareal_s": par,
        "serial_equiv_cell_updates_per_s": nx * ny * nz * nf / par,
        "executed_cell_updates_per_s": kst["cell_steps"] / par,
        "wall_s_after_iteration": iter_wall,
        "defect_vs_serial_uvw_per_iteration": [d[0] for d in defects],
        "defect_vs_serial_p_per_iteration": [d[1] for d in defects],
        "jumps_uvw": [j[0] for j in jumps], "jumps_p": [j[1] for j in jumps],
    }
    if args.temporal_error:
        # serial F with dt/10 over [0, T], slice by slice (progress per slice)
        yr = h.zeros_state(1)
        t1 = time.perf_counter()
        for n in range(N):
            h.fine_step(yr, n * T / N, (n + 1) * T / N, dt / 10, o64)
            _log("reference F_dt/10 slice %d/%d  %.1f s" % (n + 1, N, time.perf_counter() - t1))
        _sync()
        out["temporal_error_uvw"] = max(float((yr[c][0] - ref[c][N]).abs().max()) for c in range(3))
        out["temporal_error_p"] = float((yr[3][0] - ref[3][N]).abs().max())
        out["reference_dt10_s"] = time.perf_counter() - t1
    h.close()
    return out


BYTES_PROJECT_FIXED = 163.0  # adjoint projection launch: a fine step's fixed bytes without the predictor


def _stats_model_bytes(st, fixed=MODEL_STEP_FIXED):
    """The method's algorithmic bytes of the launches in one entry of the
    launch statistics: `fixed` (112) B per cell and step, 80 B per FP64 CG
    iteration, 40 B per FP32 iteration and per mixed-precision sweep
    (BiCGStab, which the byte model does not list, at its kernel's 139 B)."""
    return (st["cell_steps"] * fixed + st["cg64_cell_iters"] * MODEL_CG_ITER +
            st["cg32_cell_iters"] * 0.5 * MODEL_CG_ITER + st["bicg_cell_iters"] * BYTES_BICG_ITER +
            st["mixed_cell_sweeps"] * 40.0)


def _stats_bytes(st, fixed):
    """Algorithmic bytes of the k_persistent launches summed in one entry of
    the library's launch statistics: `fixed` bytes per cell and step, plus
    per cell 66 B per FP64 PCG iteration, 34 B per FP32 inner iteration,
    139 B per BiCGStab iteration and 65 B per mixed-precision sweep."""
    return (st["cell_steps"] * fixed + st["cg64_cell_iters"] * BYTES_CG_ITER["fp64"] +
            st["cg32_cell_iters"] * BYTES_CG_ITER["mixed"] + st["bicg_cell_iters"] * BYTES_BICG_ITER +
            st["mixed_cell_sweeps"] * BYTES_MIXED_SWEEP)


def _time_momentum_adjoint(h, y, nsp, dt, reps=20):
    """Average duration of one nsp_momentum_adjoint launch (k_mom_adjoint) at
    the state y, with seeded adjoint weights, from HIP events on the stream it
    runs on (torch's current stream)."""
    import torch
    g = torch.Generator(device="cuda").manual_seed(17)
    mu = tuple(torch.randn(a.shape, dtype=torch.float64, device="cuda", generator=g) for a in y[:3])
    lam = tuple(torch.empty_like(a) for a in y[:3])
    glid = torch.zeros((h.nz, h.nx + 1), dtype=torch.float64, device="cuda")
    for _ in range(3):
        h.momentum_adjoint(y[:3], mu, lam, dt, glid)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        h.momentum_adjoint(y[:3], mu, lam, dt, glid)
    e1.record()
    e1.synchronize()
    return e0.elapsed_time(e1) / reps


def bench_adjoint(args):
    """The adjoint workload: 96^3 cavity, Re 400, 100 fine steps of 1e-3,
    J = kinetic energy at T, gradients with respect to the initial velocity
    (a seeded divergence-free N(0, 1e-2) perturbation) and the 16 x 16 lid
    sine coefficients, checkpoints every 10 steps, FP64.  A "step" is one
    whole gradient through the autograd path (J = kinetic_energy(...) then
    J.backward(): the forward sweep records its checkpoints, backward
    recomputes the segments from them and runs the reverse sweep); value =
    cells x fine steps / wall time per gradient.  The roofline is that of
    k_persistent over every launch inside the evaluations (forward segments,
    recomputation and the reverse projections), from the library's launch
    statistics (HIP events on the launch stream); k_mom_adjoint, the
    transposed momentum step, is timed on its own beside it."""
    import torch
    from paper_1705_06149_amd import inputs, nsp
    from paper_1705_06149_amd.autograd import LidFromModes, kinetic_energy

    n, re_, dt, nsteps, ck, M = 96, 400.0, 1e-3, 100, 10, 16
    K = args.steps if args.steps_given else 2
    W = args.warmup if args.warmup_given else 1
    h = nsp.Handle(n, n, n, re=re_, max_batch=1)
    u0 = [torch.from_numpy(np.ascontiguousarray(a)).cuda()
          for a in inputs.div_free_perturbation(n, n, n, seed=5, sigma=1e-2)]
    g = torch.Generator(device="cuda").manual_seed(16)
    coef = 1e-2 * torch.randn((M, M), dtype=torch.float64, device="cuda", generator=g)
    opts = nsp.PoissonOpts(rtol=1e-12)
    split = {"forward_s": 0.0, "backward_s": 0.0}

    def gradient():
        us = [a.clone().requires_grad_() for a in u0]
        c = coef.clone().requires_grad_()
        t0 = time.perf_counter()
        J = kinetic_energy(h, us[0], us[1], us[2], LidFromModes.apply(c, h), nsteps, dt, ckpt_every=ck, opts=opts)
        _sync()
        t1 = time.perf_counter()
        J.backward()
        _sync()
        split["forward_s"] += t1 - t0
        split["backward_s"] += time.perf_counter() - t1
        return float(J.detach()), [a.grad for a in us], c.grad

    for _ in range(W):
        gradient()
    _sync()
    split["forward_s"] = split["backward_s"] = 0.0
    h.launch_stats(reset=True)
    t0 = time.perf_counter()
    for i in range(K):
        J, gu, gc = gradient()
        _log("adjoint gradient %d/%d  %.1f s" % (i + 1, K, time.perf_counter() - t0))
    _sync()
    wall = time.perf_counter() - t0
    st = h.launch_stats()
    cells = n ** 3
    fine, proj = st["fine"], st["project"]
    byts = _stats_model_bytes(fine) + _stats_model_bytes(proj, MODEL_PROJECT_FIXED)
    klayout = _stats_bytes(fine, BYTES_STEP_FIXED["fp64"]) + _stats_bytes(proj, BYTES_PROJECT_FIXED)
    kms = fine["ms"] + proj["ms"]
    launches = fine["launches"] + proj["launches"]
    achieved = byts / (kms * 1e-3) / 1e9
    # k_mom_adjoint alone, at the 96^3 state after the forward sweep
    y = h.zeros_state(1)
    h.fine_step(y, 0.0, 0.01, dt, opts)
    ma_ms = _time_momentum_adjoint(h, y, nsp, dt)
    nfaces = (n + 1) * n * n * 3
    ma_bytes = 24.0 * nfaces + cells + 24.0 * n * (n + 1)
    ma_gbs = ma_bytes / (ma_ms * 1e-3) / 1e9
    out = {
        "metric": "adjoint cell-updates/s", "value": cells * nsteps * K / wall, "unit": "cell-updates/s",
        "n_gpus": 1, "steps": K, "warmup": W, "ms_per_step": 1e3 * wall / K, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": "adjoint96_re400", "grid": [n, n, n], "re": re_, "dt": dt, "fine_steps": nsteps,
                   "checkpoint_every": ck, "lid_modes": [M, M], "poisson": "Jacobi-PCG rtol 1e-12",
                   "step": "one gradient of J through autograd (forward sweep with checkpoints, then "
                           "recomputation and reverse sweep)"},
        "J": J, "grad_u0_l2": float(torch.sqrt(sum((a ** 2).sum() for a in gu))),
        "grad_lid_coef_l2": float(torch.linalg.norm(gc)),
        "forward_s_per_gradient": split["forward_s"] / K, "backward_s_per_gradient": split["backward_s"] / K,
        "k_persistent_share_of_wall": kms * 1e-3 / wall,
        "forward_cg_iters_per_step": fine["cg_cell_iters"] / max(fine["cell_steps"], 1.0),
        "reverse_cg_iters_per_projection": proj["cg_cell_iters"] / max(proj["cell_steps"], 1.0),
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                     "frac": achieved / PEAK_HBM_GBS,
                     "traffic": _traffic_from_profile("k_persistent_adjoint96_pmc.txt"),
                     "kernel": "k_persistent (forward segments, recomputation and reverse projections)",
                     "avg_launch_ms": kms / max(launches, 1), "launches": launches,
                     "algorithmic_bytes_per_launch": byts / max(launches, 1),
                     "kernel_layout_bytes_per_launch": klayout / max(launches, 1),
                     "kernel_layout_frac": klayout / (kms * 1e-3) / 1e9 / PEAK_HBM_GBS},
        "k_mom_adjoint": {"avg_launch_ms": ma_ms, "algorithmic_bytes_per_launch": ma_bytes,
                          "bytes_model": "read u, v, w and mu (3 face arrays each), write lam, flags, lid and "
                                         "g_lid: 24 B per face + 1 B per cell + 24 B per lid value",
                          "achieved": ma_gbs, "unit": "GB/s", "frac": ma_gbs / PEAK_HBM_GBS},
    }
    h.close()
    return out


def cpu_baseline_adjoint(args):
    """The oracle's adjoint gradient on the same 96^3 workload, over a bounded
    sample of 2 fine steps, timed on the host cores."""
    from oracle import oracle as O
    from paper_1705_06149_amd import inputs

    O.build()
    n, M, nsteps = 96, 16, 2
    rng = np.random.default_rng(16)
    basis = inputs.lid_profile_basis(n, n, M)
    lid = 1.0 + np.tensordot(1e-2 * rng.standard_normal((M, M)), basis, axes=([0, 1], [0, 1]))
    g = O.Grid(n, n, n, re=400.0, lid=lid)
    u0 = inputs.div_free_perturbation(n, n, n, seed=5, sigma=1e-2)
    st0 = (u0[0], u0[1], u0[2], np.zeros((n, n, n)))
    t0 = time.perf_counter()
    O.adjoint_gradient(g, st0, nsteps, 1e-3, rtol=1e-12, ckpt_every=1)
    wall = time.perf_counter() - t0
    return {"value": n ** 3 * nsteps / wall, "unit": "cell-updates/s", "cores": int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1)), "kind": "oracle",
            "sample": "gradient of J over %d fine steps of the 96^3 adjoint workload (%.1f s)" % (nsteps, wall)}


def bench_copy(args):
    import torch
    nbytes = 1 << 30
    a = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    for _ in range(args.warmup):
        b.copy_(a)
    _sync()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        b.copy_(a)
    _sync()
    wall = time.perf_counter() - t0
    gbs = 2 * nbytes * args.steps / wall / 1e9
    return {"metric": "copy GB/s", "value": gbs, "unit": "GB/s", "n_gpus": 1, "steps": args.steps,
            "warmup": args.warmup, "ms_per_step": 1e3 * wall / args.steps, "higher_is_better": True,
            "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
            "config": {"workload": "copy_1GiB", "bytes_read_per_launch": nbytes, "bytes_written_per_launch": nbytes}}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None, help="timed steps (default 30; adjoint mode: 2 gradients)")
    ap.add_argument("--warmup", type=int, default=None, help="warm-up steps (default 5; adjoint mode: 1)")
    ap.add_argument("--mode", choices=["fine", "poisson", "parareal", "obstacles", "sim1", "sim2", "adjoint", "copy"],
                    default="fine")
    ap.add_argument("--precision", choices=["fp64", "mixed", "mixed_ru"], default="fp64",
                    help="Poisson precision: FP64, FP32 inner solves restarted at each FP64 correction, or one "
                         "FP32 solve with reliable updates")
    ap.add_argument("--solver", choices=["pcg", "bicgstab", "pcg_sr"], default="pcg",
                    help="pressure solver: Jacobi-PCG, the paper's BiCGStab (FP64), or Jacobi-PCG with one "
                         "merged reduction per iteration (FP64)")
    ap.add_argument("--max-iters", type=int, default=32)
    ap.add_argument("--slices", type=int, default=16, help="sim1/sim2 modes: time slices")
    ap.add_argument("--sim-t", type=float, default=None,
                    help="sim1/sim2 modes: end time (default the paper's: 80 and 24)")
    ap.add_argument("--temporal-error", action="store_true",
                    help="sim1/sim2 modes: also run F with dt/10 and report max |F_dt - F_dt/10| at T")
    # Forward Euler is stable only while the advective Courant number plus
    # 2 nu dt sum_d 1/h_d^2 stays below 1.  At dt = 1e-2 that sum is about
    # 0.96 + 0.55 on the 96^3 grid and the coarse propagator blows up; the
    # defaults are 5e-3 for the 96^3 Parareal run (about 0.76) and 2.5e-3 for
    # the obstacle batch, whose 128^3 grid needs dt < ~4.4e-3.
    ap.add_argument("--graph", action="store_true",
                    help="fine mode: record the step as a HIP graph and replay it (nsp_fine_step_graph_create)")
    ap.add_argument("--steps-per-launch", type=int, default=15,
                    help="fine mode: the timed steps run as calls of this many steps each (default 15: the "
                         "30 timed steps in two launches)")
    ap.add_argument("--extrapolate", action=argparse.BooleanOptionalAction, default=True,
                    help="fine mode: Poisson warm start 2 p^s - p^(s-1) from the second step of a call on "
                         "(--no-extrapolate: p^s)")
    ap.add_argument("--coarse-dt", type=float, default=None)
    ap.add_argument("--parareal-extrapolate", action="store_true",
                    help="parareal and obstacles modes: the extrapolated warm start in the fine sweeps and in "
                         "the serial FP64 reference alike")
    ap.add_argument("--coarse-rtol", type=float, default=1e-6,
                    help="parareal and obstacles modes: relative residual of the coarse propagator's Poisson "
                         "solves (G only predicts; 1e-6 keeps the iterations of 1e-10, 1e-4 does not)")
    ap.add_argument("--coarse-upwind", action="store_true",
                    help="Parareal modes: donor-cell (first-order upwind) convection in the coarse propagator")
    ap.add_argument("--coarse-grid", action="store_true",
                    help="parareal mode: coarse propagator on a grid with half the cells per direction "
                         "(restriction, coarse steps, prolongation); coarse dt defaults to 1e-2")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--obstacles", action="store_true",
                    help="fine mode: the 128^3 cavity with the seeded cuboid obstacles of the obstacle batch")
    ap.add_argument("--slip", action="store_true", help="with --obstacles: free-slip obstacle walls")
    ap.add_argument("--parareal-fine", choices=["fp64", "mixed", "mixed_ru"], default="mixed_ru",
                    help="Parareal modes: Poisson precision of the batched fine sweeps")
    ap.add_argument("--eta", type=float, default=None,
                    help="mixed: inner FP32 tolerance (default 1e-5); mixed_ru: update factor (default 1e-3)")
    ap.add_argument("--compare-fp64", action="store_true",
                    help="mixed fine mode: also run the timed steps in FP64 and report the velocity difference")
    args = ap.parse_args()
    args.steps_given, args.warmup_given = args.steps is not None, args.warmup is not None
    if args.steps is None:
        args.steps = 30
    if args.warmup is None:
        args.warmup = 5
    if args.gpus != 1:
        print("bench.py runs on one GPU only: there is no multi-GPU path (time slices would shard "
              "across GPUs with point-to-point sends of slice-end states; not implemented)", file=sys.stderr)
        sys.exit(2)
    if args.mode == "fine":
        out, host_state, t = bench_fine(args)
        rank = int(os.environ.get("RANK", "0"))
        if rank == 0 and not args.no_cpu_baseline:
            out["cpu_baseline"] = cpu_baseline_fine(args, host_state, t)
    elif args.mode == "poisson":
        out = bench_poisson(args)
    elif args.mode == "copy":
        out = bench_copy(args)
    elif args.mode == "obstacles":
        out = bench_obstacles(args)
    elif args.mode == "adjoint":
        out = bench_adjoint(args)
        if int(os.environ.get("RANK", "0")) == 0 and not args.no_cpu_baseline:
            out["cpu_baseline"] = cpu_baseline_adjoint(args)
    elif args.mode in ("sim1", "sim2"):
        out = bench_paper_sim(args, int(args.mode[3]))
    else:
        out = bench_parareal(args)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
