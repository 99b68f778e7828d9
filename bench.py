"""Benchmark: preconditioned-CG surface-source solves per second on one GPU.

Default workload (the production single-subproblem configuration): 801 x 1601
grid at 5 m, seeded layered model, 2-8 staggered scheme, 20-cell PML, dt
0.5 ms, 4000 steps, source line at 20 m, 1601 receivers at 10 m, 30
preconditioned CG iterations, FP32 wavefields and vectors, FP64 Krylov
scalars.  One step = one complete solve (r_0 = F^T d, 30 x (N p, M^-1 r),
with all dots and recurrences) for the given data.  Data: d = F h_true with
h_true a Ricker point source at x_s on the source line, computed on the
device before timing (synthetic input preparation).

Prints one JSON line.  Also reports the dominant kernel's throughput
against the HBM roofline and the FP64 oracle's CPU rate on a bounded
sample of the same workload.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# sources of the full-grid step kernel (their hash keys the counter profile)
KERNEL_SOURCES = ("ssx_step.hip", "ssx_cell.h", "ssx_device.h", "ssx_internal.h")


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--config", default="c2",
                    choices=["c1", "c2", "c3", "c4", "c4bf", "c5", "xw", "vp", "3d"],
                    help="c1..c5: the benchmark configurations; xw: the paper's crosswell "
                         "example, CG against weighted PCG; vp: a variable-projection "
                         "outer loop on the crosswell example")
    ap.add_argument("--gradient", action="store_true",
                    help="c1..c4: time the misfit gradient in kappa (forward sweep storing "
                         "the step history, transposed sweep accumulating it) instead of "
                         "the solve")
    ap.add_argument("--outer", type=int, default=4, help="vp: outer iterations")
    ap.add_argument("--compare-cg", action="store_true",
                    help="c1..c4: after timing, also solve with M = I (plain CG) and report "
                         "both residual histories, misfits and source errors")
    ap.add_argument("--solver", default="plain", choices=["plain", "weighted"],
                    help="c1..c4: Algorithm 1 on the Euclidean normal equations (plain) or "
                         "on the weighted ones N_w h = F^T W_d d (weighted)")
    ap.add_argument("--density", action="store_true",
                    help="c1..c4: a density array from the velocity (Gardner's rule, "
                         "about 1.9-2.6 g/cm^3 on these models) instead of the constant "
                         "density, velocities unchanged")
    ap.add_argument("--alpha", type=float, default=1e-3,
                    help="weighted solver: penalty weight per metre")
    ap.add_argument("--iters", type=int, default=0,
                    help="override the PCG iteration count (xw: default 60)")
    ap.add_argument("--rtol", type=float, default=0.0,
                    help="c1..c4: stop a solve once ||r_k|| <= rtol ||r_0|| (at most the "
                         "configuration's iteration count; 0: always that count)")
    ap.add_argument("--autotune", type=int, default=1)
    ap.add_argument("--requests", type=int, default=24, help="c5: requests served")
    ap.add_argument("--max-shots", type=int, default=64,
                    help="c5: shots per request cap (64: the stream's own range)")
    ap.add_argument("--max-nt", type=int, default=4000,
                    help="c5: record length cap (4000: the stream's own range)")
    ap.add_argument("--c5-ref", type=int, default=1,
                    help="c5: after timing, solve shot 0 of every request again with FP64 "
                         "fields and vectors and report the served solution's error "
                         "against it")
    ap.add_argument("--slots", type=int, default=4, help="c5: concurrent requests")
    ap.add_argument("--batch", type=int, default=1,
                    help="c5: up to this many queued requests solved as one heterogeneous "
                         "batch per slot, their propagations merged (1: one request per slot)")
    ap.add_argument("--rate-sweep", action="store_true",
                    help="c5: also serve open-loop streams at 0.5, 1.0 and 1.2x the measured "
                         "capacity (0.8x is always run)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=12.0,
                    help="target length of the oracle's bounded CPU sample")
    ap.add_argument("--cpu-procs", type=int, default=16,
                    help="batched configurations: also time the oracle in this many "
                         "concurrent processes, one shot each (capped by the shots and the "
                         "host's cores)")
    ap.add_argument("--shots", type=int, default=0,
                    help="override the number of shots (spread across the surface as in "
                         "the batched configuration)")
    ap.add_argument("--dtype", default="", choices=["", "f64", "f32", "f16", "bf16"],
                    help="override the wavefield storage type")
    ap.add_argument("--tile-z", type=int, default=-1,
                    help="force the full-grid tile height after tuning (profiling runs)")
    ap.add_argument("--ref-f64", type=int, default=0,
                    help="after timing, solve the same problem with FP64 fields and vectors "
                         "(the FP64 path matches the FP64 oracle to 1e-9) and report the "
                         "timed solution's error against it")
    ap.add_argument("--shot-group", type=int, default=-1,
                    help="force the full-grid shots per launch after tuning (profiling runs)")
    ap.add_argument("--tile-loop", type=int, default=-1,
                    help="force the full-grid tile-loop setting after tuning (0 off, 1 on; "
                         "profiling runs)")
    ap.add_argument("--graphs", type=int, default=1)
    ap.add_argument("--prop-only", type=int, default=0,
                    help="run this many forward+adjoint propagation pairs and exit "
                         "(a short workload for kernel profiling)")
    ap.add_argument("--nt", type=int, default=0,
                    help="override the record length (for short profiling runs; the "
                         "result line then describes that shortened workload)")
    ap.add_argument("--slab-steps", type=int, default=-1,
                    help="time steps per launch on the thin slab (after the tuner; -1: "
                         "as tuned)")
    ap.add_argument("--slab-strip", type=int, default=-1,
                    help="strip width of the multi-step kernel on the thin slab (after the "
                         "tuner; -1: as tuned)")
    ap.add_argument("--prop-slab", action="store_true",
                    help="with --prop-only: the pairs are thin-slab propagations (X, then "
                         "X^T of its datum traces) instead of F^T, F")
    ap.add_argument("--calib-copy", type=float, default=0.0,
                    help="with --prop-only: also run 10 plain device copies of this many "
                         "MB (reference for hardware byte counters)")
    return ap.parse_args()


def oracle_parallel(cnum, steps, nproc):
    """Seconds that each of nproc concurrent child processes (fresh
    interpreters, one thread each, started together) takes for a steps-long
    oracle forward run of configuration cnum; None if any of them fails."""
    import subprocess
    start = time.time() + 8.0
    code = (
        "import sys, time, json\n"
        f"sys.path.insert(0, {ROOT!r})\n"
        "import numpy as np, inputs, oracle\n"
        f"wl = inputs.workload({cnum})\n"
        f"prob = wl.prob.replace(nt={steps}, xs=wl.prob.xs[:1])\n"
        "m = oracle.Model(prob, wl.kappa, wl.rho)\n"
        f"hs = np.random.default_rng(0).standard_normal(({steps}, prob.ns))\n"
        f"time.sleep(max(0.0, {start} - time.time()))\n"
        "t = time.perf_counter()\n"
        "m.fwd(hs)\n"
        "print(json.dumps(time.perf_counter() - t))\n")
    env = dict(os.environ, OMP_NUM_THREADS="1", OPENBLAS_NUM_THREADS="1", MKL_NUM_THREADS="1")
    procs = [subprocess.Popen([sys.executable, "-c", code], stdout=subprocess.PIPE,
                              stderr=subprocess.DEVNULL, env=env, text=True)
             for _ in range(nproc)]
    out = []
    for pr in procs:
        o, _ = pr.communicate()
        if pr.returncode != 0:
            return None
        out.append(float(o.strip().splitlines()[-1]))
    return out


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor()


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "bench.py runs on one GPU only; --gpus must be 1"}))
        sys.exit(2)
    import numpy as np
    import torch

    import inputs
    import paper_2203_16573_amd as ssx

    if not torch.cuda.is_available():
        print(json.dumps({"error": "no GPU visible"}))
        sys.exit(1)
    torch.cuda.set_device(0)

    if args.config == "c5":
        return serve_bench(args)
    if args.config == "xw":
        return crosswell_bench(args)
    if args.config == "vp":
        return varpro_bench(args)
    if args.config == "3d":
        return bench3d(args)
    cnum = {"c1": 1, "c2": 2, "c3": 3, "c4": 4, "c4bf": 4}[args.config]
    wl = inputs.workload(cnum)
    if args.density:
        wl = inputs.with_gardner_density(wl)
    if args.nt:
        wl.prob = wl.prob.replace(nt=args.nt)
    if args.shots:
        width = (wl.prob.nx - 1) * wl.prob.h
        wl.prob = wl.prob.replace(xs=inputs.shot_positions(args.shots, width))
    if args.iters:
        wl.K = args.iters
    weighted = args.solver == "weighted"
    if weighted:
        # receiver-side datum 5 cells beyond the receivers, away from the sources
        wl.prob = wl.prob.replace(rslab_dz=-5 if wl.prob.z_rec < wl.prob.z_src else 5)
    prob = wl.prob
    fd = {"c1": "f64", "c2": "f32", "c3": "f32", "c4": "f16", "c4bf": "bf16"}[args.config]
    if args.dtype:
        fd = args.dtype
    vdt = torch.float64 if fd == "f64" else torch.float32

    ctx = ssx.Context(prob, wl.kappa, wl.rho, field_dtype=fd)
    tuned = None
    if args.autotune:
        from paper_2203_16573_amd import autotune
        tuned = autotune.choose(prob, wl.kappa, wl.rho, field_dtype=fd)
        autotune.apply(ctx, tuned)
    if args.tile_z >= 0:
        ctx.set_option(ssx.OPT_TILE_Z, args.tile_z)
    if args.shot_group >= 0:
        ctx.set_option(ssx.OPT_SHOT_GROUP, args.shot_group)
    if args.tile_loop >= 0:
        ctx.set_option(ssx.OPT_TILE_LOOP, args.tile_loop)
    if args.slab_steps >= 0 or args.slab_strip >= 0:
        ctx.set_option(ssx.OPT_SLAB_STRIP, 0)
        if args.slab_steps >= 0:
            ctx.set_option(ssx.OPT_STEPS_PER_LAUNCH_SLAB, args.slab_steps)
        if args.slab_strip >= 0:
            ctx.set_option(ssx.OPT_SLAB_STRIP, args.slab_strip)
    ctx.set_graphs(bool(args.graphs))
    wav = inputs.source_wavelet(prob, wl.freq)
    htrue = np.stack([inputs.spike_gather(prob, wav, s) for s in range(prob.nshots)])
    # the data: F h_true with FP64 fields (input preparation, before any
    # timing), rounded to the vector type -- the data of the oracle's
    # full-length solves in tests/golden
    gen = ssx.Context(prob, wl.kappa, wl.rho, field_dtype="f64")
    d64 = gen.fwd(torch.tensor(htrue, dtype=torch.float64, device="cuda"), gen.empty_r())
    torch.cuda.synchronize()
    gen.close()
    d = d64.to(vdt).contiguous()
    del d64
    h = ctx.empty_s()
    torch.cuda.synchronize()
    if args.prop_only:
        if args.calib_copy:
            n = int(args.calib_copy * 1e6 / 4)
            src = torch.ones(n, device="cuda")
            dst = torch.empty_like(src)
            for _ in range(10):
                dst.copy_(src)
            torch.cuda.synchronize()
        g = ctx.empty_s()
        P, V = ctx.empty_s(), ctx.empty_s()
        if args.prop_slab:
            g.normal_()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.prop_only):
            if args.prop_slab:
                ctx.slab_fwd(g, P, V)
                ctx.slab_adj(V, P, g)
            else:
                ctx.adj(d, g)
                ctx.fwd(g, d)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        print(json.dumps({"mode": "prop-only" + (" slab" if args.prop_slab else ""),
                          "config": wl.name, "pairs": args.prop_only,
                          "ms_per_propagation": 1e3 * el / (2 * args.prop_only)}), flush=True)
        ctx.close()
        return

    if args.gradient:
        return gradient_bench(args, wl, ctx, d, fd)

    def solve():
        if weighted:
            return ctx.pcg_solve_w(d, args.alpha, wl.K, rtol=args.rtol, h=h,
                                   raise_on_breakdown=False)
        return ctx.pcg_solve(d, wl.alpha_rel, wl.K, rtol=args.rtol, h=h, raise_on_breakdown=False)

    for _ in range(args.warmup):
        solve()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    marks = []
    for _ in range(args.steps):
        _, hist, iters, st = solve()   # returns after synchronising the stream
        marks.append(time.perf_counter())
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    per_step = np.diff([t0] + marks) * 1e3
    solves = args.steps * prob.nshots
    value = solves / elapsed

    # dominant kernel: the full-grid time step.  One forward propagation is
    # nt launches of it (plus one sampling launch); time it with events on
    # the context's stream.
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    dtmp = ctx.empty_r()
    nrep = 3
    # one untimed propagation first: a new output buffer means a new captured
    # graph, whose capture and instantiation must not fall in the timed region
    ctx.fwd(h, dtmp)
    torch.cuda.synchronize()
    e0.record(stream)
    for _ in range(nrep):
        ctx.fwd(h, dtmp)
    e1.record(stream)
    torch.cuda.synchronize()
    step_ms = e0.elapsed_time(e1) / (nrep * prob.nt)
    NZ, NX = prob.nz + 2 * prob.npml, prob.nx + 2 * prob.npml
    cells = ctx.cells_per_launch()          # one launch: the shots of one group
    group = cells // (NZ * NX)
    launches = -(-prob.nshots // group)      # launches per time step
    fsz = {"f64": 8, "f32": 4, "f16": 2, "bf16": 2}[fd]
    csz = 8 if fd == "f64" else 4
    # algorithmic bytes per cell-update: read p, v_x, v_z and kappa once,
    # write p, v_x, v_z once; a density array adds the two velocity
    # coefficients
    b_alg = 6 * fsz + csz * (3 if args.density else 1)
    achieved = b_alg * NZ * NX * prob.nshots / (step_ms * 1e-3) / 1e9
    tz_used, spl_used, _, loop_used = ctx.launch_shape()
    traffic = None if args.density else measured_traffic(
        args.config, fd, prob.nshots, tz_used, group, loop_used, ctx.step_kernel_name())
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": None if traffic is None else traffic["bytes_per_launch"],
                "traffic_detail": traffic,
                "kernel": ctx.step_kernel_name(), "tile_z": tz_used, "tile_loop": loop_used,
                "us_per_launch": round(step_ms * 1e3 * spl_used / launches, 3),
                "steps_per_launch": spl_used,
                "launches_per_step": launches if spl_used == 1 else round(launches / spl_used, 4),
                "bytes_per_cell": b_alg,
                "cells_per_launch": cells}

    # cell-updates in one solve: (2K + 1) full propagations, 2 (K + 1) slab;
    # weighted: also 2 (K + 1) on the receiver-side slab and, with a nonzero
    # alpha, 2K more on the source-side one
    k = prob.order // 2
    nzs = abs(prob.slab_dz) + 1 + 2 * k + 2 * prob.npml
    Kr = iters if args.rtol > 0 else wl.K  # iterations the timed solves ran
    cu_solve = prob.nt * ((2 * Kr + 1) * NZ * NX + 2 * (Kr + 1) * nzs * NX)
    if weighted:
        nzr = abs(prob.rslab_dz) + 1 + 2 * k + 2 * prob.npml
        cu_solve += prob.nt * NX * (2 * (Kr + 1) * nzr + (2 * Kr * nzs if args.alpha else 0))
    gcell = cu_solve * prob.nshots / (elapsed / args.steps) / 1e9

    cpu = None
    if not args.no_cpu_baseline:
        import oracle

        def oracle_fwd_seconds(steps):
            m = oracle.Model(prob.replace(nt=steps, xs=prob.xs[:1]), wl.kappa, wl.rho)
            hs = np.random.default_rng(0).standard_normal((steps, prob.ns))
            t = time.perf_counter()
            m.fwd(hs)
            return time.perf_counter() - t

        # size the sample from a 4-step probe so that it takes about
        # --cpu-seconds of one core
        probe = oracle_fwd_seconds(4)
        ns_cpu = int(max(4, min(prob.nt, round(4 * args.cpu_seconds / max(probe, 1e-6)))))
        tc = oracle_fwd_seconds(ns_cpu)
        cpu_gcell = ns_cpu * NZ * NX / tc / 1e9
        cpu = {"value": cpu_gcell * 1e9 / cu_solve, "unit": "solves/s", "cores": 1,
               "kind": "oracle",
               "sample": f"FP64 NumPy oracle forward, {ns_cpu} steps of the {NZ}x{NX} "
                         f"padded grid ({tc:.1f} s, {cpu_gcell:.4f} Gcell/s, 1 thread), "
                         f"extrapolated linearly to {cu_solve:.3e} cell-updates per solve",
               "cpu": cpu_model()}
        nproc = min(prob.nshots, args.cpu_procs, os.cpu_count() or 1)
        if nproc > 1 and not (args.nt or args.shots or args.density):
            par = oracle_parallel(cnum, ns_cpu, nproc)
            if par:
                pg = sum(ns_cpu * NZ * NX / t for t in par) / 1e9
                cpu = {"value": pg * 1e9 / cu_solve, "unit": "solves/s", "cores": nproc,
                       "kind": "oracle",
                       "sample": f"FP64 NumPy oracle forward, {ns_cpu} steps of the {NZ}x{NX} "
                                 f"padded grid in {nproc} concurrent single-threaded "
                                 f"processes, one shot each ({min(par):.1f}-{max(par):.1f} s, "
                                 f"{pg:.4f} Gcell/s together), extrapolated linearly to "
                                 f"{cu_solve:.3e} cell-updates per solve",
                       "single_core_value": cpu["value"], "cpu": cpu_model()}

    cgcmp = None
    if args.compare_cg and not weighted:
        def summary(hh, hs_):
            r = hs_[:, :, 0] / hs_[:, :1, 0]
            hn = hh.double().cpu().numpy()
            dn_ = np.linalg.norm(d.double().cpu().numpy().reshape(prob.nshots, -1), axis=1)
            return {"rel_residual_every_5": [round(float(v), 4) for v in np.median(r, axis=0)[::5]],
                    "rel_residual_final": round(float(np.median(r[:, -1])), 4),
                    "misfit_final": round(float(np.median(hs_[:, -1, 3] / dn_)), 4),
                    "source_error": round(float(np.median(
                        [np.linalg.norm(hn[s] - htrue[s]) / np.linalg.norm(htrue[s])
                         for s in range(prob.nshots)])), 4)}
        pcg_sum = summary(h, hist)
        hc, histc, _, _ = ctx.pcg_solve(d, wl.alpha_rel, wl.K, use_precond=False,
                                         raise_on_breakdown=False)
        cgcmp = {"pcg": pcg_sum, "cg": summary(hc, histc),
                 "note": "medians over shots; residual = ||r_k|| / ||r_0|| of the Euclidean "
                         "normal equations, misfit = ||F h_K - d|| / ||d||, source error "
                         "against the point source that made d"}

    ref = None
    if args.ref_f64:
        rctx = ssx.Context(prob, wl.kappa, wl.rho, field_dtype="f64")
        h64, hist64, _, _ = rctx.pcg_solve(d.double(), wl.alpha_rel, wl.K, h=rctx.empty_s(),
                                           raise_on_breakdown=False)
        torch.cuda.synchronize()
        rctx.close()
        hh, hr = h.double().cpu().numpy(), h64.cpu().numpy()
        errs = [float(np.linalg.norm(hh[s] - hr[s]) / np.linalg.norm(hr[s]))
                for s in range(prob.nshots)]
        rr = hist[:, :, 0] / hist64[:, :, 0]
        ref = {"reference": "same solve with FP64 fields and vectors on the GPU",
               "h_rel_l2_median": float(np.median(errs)), "h_rel_l2_max": float(np.max(errs)),
               "residual_history_max_rel_diff": float(np.max(np.abs(rr - 1.0)))}

    out = {
        "metric": "weighted PCG surface-source solves/s" if weighted
        else "PCG surface-source solves/s",
        "value": round(value, 4),
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(1e3 * elapsed / args.steps, 2),
        "ms_per_step_median": round(float(np.median(per_step)), 2),
        "ms_per_step_range": [round(float(per_step.min()), 2), round(float(per_step.max()), 2)],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"f64": "f64", "f32": "f32", "f16": "f16-storage/f32", "bf16": "bf16-storage/f32"}[fd],
        "data": "synthetic (seeded layered model; d = F of a Ricker point source)",
        "config": {"workload": f"{wl.name}: {prob.nz}x{prob.nx} @ {prob.h} m, order "
                               f"{prob.order}, nt {prob.nt}, K {wl.K}, shots {prob.nshots}"
                               + (f", weighted, alpha {args.alpha}/m" if weighted else "")
                               + (", density array (Gardner)" if args.density else "")
                               + (f", stop at ||r_k|| <= {args.rtol:g} ||r_0||"
                                  if args.rtol > 0 else ""),
                   "nz": prob.nz, "nx": prob.nx, "nt": prob.nt, "K": wl.K,
                   "shots": prob.nshots, "field_dtype": fd},
        "gcell_updates_per_s": round(gcell, 2),
        "iters": iters,
        "pcg_status": int(st),
        "shots_with_gr_sign_change": int(np.sum(np.any(np.sign(hist[:, :, 2]) !=
                                                        np.sign(hist[:, :1, 2]), axis=1))),
        "kernel_choice": None if tuned is None else {k: v for k, v in tuned.items() if k != "us"},
        "final_rel_residual": float(np.median(hist[:, -1, 0] / hist[:, 0, 0])),
        # ||M^-1 r_k|| / ||M^-1 r_0|| (the preconditioned normal residual)
        "final_rel_precond_residual": float(np.median(hist[:, -1, 1] / hist[:, 0, 1])),
        "iters_to_drop": {
            name: {tag: (lambda idx: int(idx[0]) if idx.size else None)(
                np.nonzero(np.median(hist[:, :, col] / hist[:, :1, col], axis=0) <= lev)[0])
                   for tag, lev in (("10x", 0.1), ("100x", 0.01))}
            for name, col in (("residual", 0), ("precond_residual", 1))},
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    if ref is not None:
        out["error_vs_f64_solve"] = ref
    orc = oracle_golden_errors(cnum, wl, prob, h, hist, args, weighted)
    if orc is not None:
        out["error_vs_oracle"] = orc
    if cgcmp is not None:
        out["cg_comparison"] = cgcmp
    print(json.dumps(out), flush=True)
    ctx.close()


def crosswell_bench(args):
    """The paper's comparison of CG and preconditioned CG (Numerical
    Examples, the last subsection) in its crosswell geometry: data from a
    point source at (3500, 3500) m in the lens model, recorded at 1000 m
    over x = 2000..6000 m and inverted for an extended source on 3000 m in
    the homogeneous model.  CG runs Algorithm 1 with M = I on the Euclidean
    normal equations (the same penalty relative to the operator scale,
    alpha_rel = alpha); PCG runs it on the weighted normal equations with
    M^-1 = D W^-1 D.  For each alpha in {0, --alpha} the line reports the
    relative normal-residual curves (CG: ||r_k||; PCG: ||M^-1 r_k||, the
    left side of the norm1 form), the iterations each needs to reduce it by
    10x, 100x and 1000x, and the data misfit, and beside them the thin-slab
    preconditioner on the Euclidean normal equations.  It also reports the paper's
    operator checks as relative misfits: the pressure source -2 P_s v_z and
    the normal load -2 P_s p reproducing the point source's data, Lambda~
    with the 5-cell datum against the whole path to the receiver surface,
    the symmetrised Lambda~ of the gather used as a source (lens model),
    re-simulation of the time-reversal
    inverse 4 V^T d and of the unitary-norm inverse W^-1 F^T W_d d, the
    asymmetry of Lambda~ and the sv relation 1/4 Lambda_r F Lambda_s = V on
    the pressure gather that the point source leaves on z = 3000 m (all in
    the homogeneous model).  Then it times repeated weighted solves
    (--steps, after --warmup)."""
    import numpy as np
    import torch

    import inputs
    import paper_2203_16573_amd as ssx

    rho = inputs.RHO_WATERLIKE
    prob = inputs.crosswell_problem()
    if args.nt:
        prob = prob.replace(nt=args.nt)
    K = args.iters or 60
    fd = args.dtype or "f32"
    vdt = torch.float64 if fd == "f64" else torch.float32
    # data: the point source in the lens model
    pprob = inputs.crosswell_point_problem(prob)
    pctx = ssx.Context(pprob, inputs.crosswell_kappa(lens=True), rho, field_dtype=fd)
    w = inputs.bandpass_wavelet((np.arange(prob.nt) + 0.5) * prob.dt)
    hpt = torch.tensor((w / prob.h)[None, :, None], dtype=vdt, device="cuda").contiguous()
    d = pctx.fwd(hpt, pctx.empty_r())
    torch.cuda.synchronize()
    pctx.close()
    ctx = ssx.Context(prob, inputs.crosswell_kappa(lens=False), rho, field_dtype=fd)
    tuned = None
    if args.autotune:
        from paper_2203_16573_amd import autotune
        tuned = autotune.choose(prob, inputs.crosswell_kappa(lens=False), rho, field_dtype=fd)
        autotune.apply(ctx, tuned)
    ctx.set_graphs(bool(args.graphs))
    dn = float(torch.linalg.norm(d.double()))

    def reached(curve, level):
        idx = np.nonzero(curve <= level)[0]
        return int(idx[0]) if idx.size else None

    comparison = {}
    for alpha in sorted({0.0, args.alpha}):
        _, hc, _, stc = ctx.pcg_solve(d, alpha, K, use_precond=False, raise_on_breakdown=False)
        _, hp, _, stp = ctx.pcg_solve_w(d, alpha, K, raise_on_breakdown=False)
        _, he, _, ste = ctx.pcg_solve(d, alpha, K, raise_on_breakdown=False)
        cg = hc[0, :, 0] / hc[0, 0, 0]
        pcg = hp[0, :, 1] / hp[0, 0, 1]
        entry = {"cg_status": int(stc), "pcg_status": int(stp),
                 "pcg_gr_sign_changes": int(np.sum(np.sign(hp[0, :, 2]) != np.sign(hp[0, 0, 2]))),
                 "cg_curve": [round(float(v), 6) for v in cg],
                 "pcg_curve": [round(float(v), 6) for v in pcg],
                 "cg_misfit": round(float(hc[0, -1, 3] / dn), 5),
                 "pcg_misfit": round(float(hp[0, -1, 3] / dn), 5),
                 # the thin-slab preconditioner on the Euclidean normal
                 # equations (ssx_pcg_solve): both of its residual norms
                 "euclid_pcg": {"status": int(ste),
                                "r_curve": [round(float(v), 6) for v in he[0, :, 0] / he[0, 0, 0]],
                                "g_curve": [round(float(v), 6) for v in he[0, :, 1] / he[0, 0, 1]],
                                "misfit": round(float(he[0, -1, 3] / dn), 5)}}
        for tag, lev in (("10x", 1e-1), ("100x", 1e-2), ("1000x", 1e-3)):
            a, b = reached(cg, lev), reached(pcg, lev)
            entry[f"iters_to_{tag}"] = {"cg": a, "pcg": b,
                                       "ratio": round(a / b, 2) if a and b else None}
        # where <g_k, r_k> first changes sign (PCG): from then on beta_k < 0
        sg = np.sign(hp[0, :, 2])
        flips = np.nonzero(sg != sg[0])[0]
        entry["pcg_gr_first_sign_change_at"] = int(flips[0]) if flips.size else None
        entry["cg_misfit_curve"] = [round(float(v / dn), 5) for v in hc[0, :, 3]]
        entry["pcg_misfit_curve"] = [round(float(v / dn), 5) for v in hp[0, :, 3]]
        comparison[f"alpha={alpha:g}"] = entry

    # Like for like: both solvers' iterates h_k at checkpoints k, measured in
    # the same three norms: the Euclidean normal residual ||F^T d - N h|| /
    # ||F^T d|| (CG's own; N with CG's alpha), the preconditioned weighted
    # normal residual ||M^-1 (F^T W_d d - N_w h)|| / ||M^-1 F^T W_d d|| (the
    # norm1 form, PCG's own) and the data misfit ||F h - d|| / ||d||.  Also
    # the cost of an iteration of each and the time each takes to bring the
    # data misfit to given levels.
    Ftd = ctx.adj(d, ctx.empty_s()).clone()
    FtWd = ctx.adj(ctx.weight_d(d, ctx.empty_r()), ctx.empty_s()).clone()
    ftd_n = float(torch.linalg.norm(Ftd.double()))
    checkpoints = [k for k in (0, 2, 5, 10, 20, 30, 45, 60) if k <= K]
    q, Fh = ctx.empty_s(), ctx.empty_r()
    like = {}
    for alpha in sorted({0.0, args.alpha}):
        a_e = alpha * ftd_n / dn  # the absolute alpha ssx_pcg_solve derives
        MFtWd_n = float(torch.linalg.norm(ctx.precond(alpha, FtWd, ctx.empty_s()).double()))
        rows = {"cg": [], "pcg": []}
        for name in ("cg", "pcg"):
            for k in checkpoints:
                if k == 0:
                    hk = torch.zeros_like(Ftd)
                elif name == "cg":
                    hk, _, _, _ = ctx.pcg_solve(d, alpha, k, use_precond=False,
                                                raise_on_breakdown=False)
                else:
                    hk, _, _, _ = ctx.pcg_solve_w(d, alpha, k, raise_on_breakdown=False)
                hk = hk.clone()
                e_n = float(torch.linalg.norm((Ftd - ctx.normal(a_e, hk, q)).double())) / ftd_n
                rw = FtWd - ctx.normal_w(alpha, hk, q)
                e_w = float(torch.linalg.norm(ctx.precond(alpha, rw.contiguous(),
                                                          ctx.empty_s()).double())) / MFtWd_n
                mis = float(torch.linalg.norm((ctx.fwd(hk, Fh) - d).double())) / dn
                rows[name].append({"k": k, "euclid_normal_res": round(e_n, 6),
                                   "weighted_normal_res": round(e_w, 6),
                                   "misfit": round(mis, 5)})
        # seconds per iteration of each solver (K iterations, after one run)
        per_it = {}
        for name in ("cg", "pcg"):
            run = ((lambda: ctx.pcg_solve(d, alpha, K, use_precond=False,
                                          raise_on_breakdown=False)) if name == "cg" else
                   (lambda: ctx.pcg_solve_w(d, alpha, K, raise_on_breakdown=False)))
            run()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            run()
            torch.cuda.synchronize()
            per_it[name] = (time.perf_counter() - t0) / K
        curves = {"cg": np.array(comparison[f"alpha={alpha:g}"]["cg_misfit_curve"]),
                  "pcg": np.array(comparison[f"alpha={alpha:g}"]["pcg_misfit_curve"])}
        to_level = {}
        for lev in (0.5, 0.3, 0.2, 0.15, 0.1):
            ent = {}
            for name in ("cg", "pcg"):
                it = reached(curves[name], lev)
                ent[name] = None if it is None else {"iters": it,
                                                     "s": round(it * per_it[name], 4)}
            to_level[f"misfit<={lev:g}"] = ent
        like[f"alpha={alpha:g}"] = {"checkpoints": rows,
                                    "ms_per_iteration": {k: round(1e3 * v, 3)
                                                         for k, v in per_it.items()},
                                    "time_to_misfit": to_level}

    def nrm(t):
        return float(torch.linalg.norm(t.double()))

    # the point source's pressure gather on the source line, homogeneous model
    gprob = pprob.replace(z_rec=prob.z_src, x_rec0=prob.x_src0, nr=prob.ns)
    gctx = ssx.Context(gprob, inputs.crosswell_kappa(lens=False), rho, field_dtype=fd)
    ps = gctx.fwd(hpt, gctx.empty_r()).clone()
    torch.cuda.synchronize()
    gctx.close()
    Fh = ctx.empty_r()
    h_tr = ctx.tr_inverse(d, ctx.empty_s())
    mis_tr = nrm(ctx.fwd(h_tr, Fh) - d) / dn
    h_u = ctx.precond(0.0, ctx.adj(ctx.weight_d(d, ctx.empty_r()), ctx.empty_s()), ctx.empty_s())
    mis_u = nrm(ctx.fwd(h_u, Fh) - d) / dn
    lam = ctx.lam(0, False, ps, ctx.empty_s()).clone()
    lamt = ctx.lam(0, True, ps, ctx.empty_s())
    asym = nrm(lam - lamt) / nrm(lam)
    sv = 0.25 * ctx.lam(1, False, ctx.fwd(lam, ctx.empty_r()), ctx.empty_r())
    vx = ctx.fwd_v(ps, ctx.empty_r())
    sv_mis = nrm(sv - vx) / nrm(vx)
    # equivalence of pressure and normal-load sources (snull, tracejump
    # relations): h = -2 P_s v_z and f = -2 P_s p of the point source's field
    # on the source line reproduce its data on the receiver line
    gctx = ssx.Context(gprob, inputs.crosswell_kappa(lens=False), rho, field_dtype=fd)
    vs = gctx.block(0, 1, False, hpt, gctx.empty_r()).clone()
    torch.cuda.synchronize()
    gctx.close()
    hctx = ssx.Context(pprob, inputs.crosswell_kappa(lens=False), rho, field_dtype=fd)
    d_h = hctx.fwd(hpt, hctx.empty_r()).clone()
    torch.cuda.synchronize()
    hctx.close()
    dhn = nrm(d_h)
    mis_hs = nrm(ctx.fwd(-2.0 * vs, ctx.empty_r()) - d_h) / dhn
    # the model-space form of approxinv, 4 V^T F h ~ h, on that equivalent
    # pressure source
    h_eq = -2.0 * vs
    tr_model = nrm(ctx.tr_inverse(ctx.fwd(h_eq, ctx.empty_r()), ctx.empty_s()) - h_eq) / nrm(h_eq)
    mis_fs = nrm(ctx.block(1, 0, False, -2.0 * ps, ctx.empty_r()) - d_h) / dhn
    # the near datum against the whole path to the receiver surface: Lambda~
    # with the datum 100 cells from the source line (a slab of the full
    # source-to-receiver depth) against the 5-cell datum
    fctx = ssx.Context(prob.replace(slab_dz=-int(round((prob.z_src - prob.z_rec) / prob.h))),
                       inputs.crosswell_kappa(lens=False), rho, field_dtype=fd)
    lam_far = fctx.lam(0, False, ps, fctx.empty_s())
    near_far = nrm(lam - lam_far) / nrm(lam_far)
    torch.cuda.synchronize()
    fctx.close()
    # the symmetrised Lambda~ applied to the point source's pressure gather,
    # used as a pressure source, against the point source's data, all in the
    # lens model
    lctx = ssx.Context(prob, inputs.crosswell_kappa(lens=True), rho, field_dtype=fd)
    lg = ssx.Context(gprob, inputs.crosswell_kappa(lens=True), rho, field_dtype=fd)
    ps_l = lg.fwd(hpt, lg.empty_r()).clone()
    torch.cuda.synchronize()
    lg.close()
    hsym = lctx.precond(0.0, ps_l, lctx.empty_s())
    sym_src = nrm(lctx.fwd(hsym, lctx.empty_r()) - d) / dn
    torch.cuda.synchronize()
    lctx.close()
    checks = {"pressure_source_equivalence_misfit": round(mis_hs, 4),
              "lambda_near_vs_full_path": round(near_far, 4),
              "time_reversal_model_space_misfit": round(tr_model, 4),
              "symmetrised_lambda_source_misfit": round(sym_src, 4),
              "normal_load_equivalence_misfit": round(mis_fs, 4),
              "time_reversal_resimulation_misfit": round(mis_tr, 4),
              "unitary_inverse_resimulation_misfit": round(mis_u, 4),
              "lambda_asymmetry": round(asym, 4),
              "sv_relation_misfit": round(sv_mis, 4),
              "input": "pressure gather of the point source on z = 3000 m (homogeneous model)"}

    h = ctx.empty_s()
    for _ in range(args.warmup):
        ctx.pcg_solve_w(d, args.alpha, K, h=h, raise_on_breakdown=False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        ctx.pcg_solve_w(d, args.alpha, K, h=h, raise_on_breakdown=False)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    out = {
        "metric": "weighted PCG surface-source solves/s (crosswell example)",
        "value": round(args.steps / el, 4), "unit": "solves/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(1e3 * el / args.steps, 2), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": fd,
        "data": "synthetic (lens model of the paper's shape; bandpass point source)",
        "config": {"workload": f"crosswell: {prob.nz}x{prob.nx} @ {prob.h} m, order "
                               f"{prob.order}, nt {prob.nt}, K {K}, alpha {args.alpha}/m",
                   "nz": prob.nz, "nx": prob.nx, "nt": prob.nt, "K": K, "field_dtype": fd},
        "ms_per_iteration": round(1e3 * el / (args.steps * K), 3),
        "kernel_choice": None if tuned is None else {k: v for k, v in tuned.items() if k != "us"},
        "cg_vs_pcg": comparison,
        "cg_vs_pcg_same_norms": like,
        "operator_checks": checks,
    }
    print(json.dumps(out), flush=True)
    ctx.close()


def gradient_bench(args, wl, ctx, d, fd):
    """Timed misfit gradients in kappa (ssx_misfit_gradient) at h = a
    shifted copy of the true source: two full-grid sweeps of one step per
    launch, plus per step a store (forward) or an accumulation (transposed)
    pass over the physical cells.  Bytes per cell-update beyond the step's
    own: the stored residual (written, then read) and the transposed
    pressure and FP64 accumulator (read, read and written)."""
    import numpy as np
    import torch

    import inputs
    prob = wl.prob
    vdt = torch.float64 if fd == "f64" else torch.float32
    w = inputs.source_wavelet(prob, wl.freq)
    h = np.roll(np.stack([inputs.spike_gather(prob, w, s) for s in range(prob.nshots)]), 40,
                axis=2)
    h = torch.tensor(h, dtype=vdt, device="cuda")
    g = ctx.empty_model()
    for _ in range(args.warmup):
        ctx.misfit_gradient(h, d, g)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        _, J = ctx.misfit_gradient(h, d, g)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    NZ, NX = prob.nz + 2 * prob.npml, prob.nx + 2 * prob.npml
    cu = 2 * prob.nt * NZ * NX * prob.nshots
    fsz = 8 if fd == "f64" else 4
    # algorithmic bytes the gradient adds to the two sweeps, per physical
    # cell and step: the history written by the forward step (fsz), read
    # back with the transposed pressure (2 fsz), and the FP64 accumulator
    # read and written once per step pair (8)
    extra = prob.nt * prob.nz * prob.nx * prob.nshots * (3 * fsz + 8)
    out = {
        "metric": "misfit gradients in kappa/s", "value": round(args.steps / el, 4),
        "unit": "gradients/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(1e3 * el / args.steps, 2), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": fd,
        "data": "synthetic (seeded layered model; d = F of a Ricker point source)",
        "config": {"workload": f"{wl.name}: {prob.nz}x{prob.nx} @ {prob.h} m, order "
                               f"{prob.order}, nt {prob.nt}, shots {prob.nshots}, gradient",
                   "nz": prob.nz, "nx": prob.nx, "nt": prob.nt, "shots": prob.nshots,
                   "field_dtype": fd},
        "gcell_updates_per_s": round(cu * args.steps / el / 1e9, 2),
        # rows held in the grid's aligned groups of four columns
        "history_bytes": prob.nt * prob.nz * prob.nshots * fsz
        * 4 * ((prob.npml + prob.nx - 1) // 4 - prob.npml // 4 + 1),
        "extra_bytes_per_gradient": extra,
        "misfit": [float(v) for v in J],
    }
    print(json.dumps(out), flush=True)
    ctx.close()


def varpro_bench(args):
    """A variable-projection outer loop on the crosswell example: data of the
    point source in the lens model, starting from the homogeneous model.
    Each outer iteration solves the subproblem (Algorithm 1, --iters or 20
    iterations, M^-1 = D W^-1 D, alpha_rel = --alpha) for h*(kappa),
    evaluates the reduced objective 1/2 ||F h* - d||^2 + alpha^2/2 ||A h*||^2
    and its gradient (the misfit gradient at h*), and takes a steepest-
    descent step scaled to change kappa by at most 5 % (halved until the
    reduced objective falls, at most four times).  Reports the objective,
    the relative model error and the time per outer iteration."""
    import numpy as np
    import torch

    import inputs
    import paper_2203_16573_amd as ssx

    rho = inputs.RHO_WATERLIKE
    prob = inputs.crosswell_problem()
    if args.nt:
        prob = prob.replace(nt=args.nt)
    K = args.iters or 20
    fd = args.dtype or "f32"
    vdt = torch.float64 if fd == "f64" else torch.float32
    k_true = inputs.crosswell_kappa(lens=True)
    pctx = ssx.Context(inputs.crosswell_point_problem(prob), k_true, rho, field_dtype=fd)
    w = inputs.bandpass_wavelet((np.arange(prob.nt) + 0.5) * prob.dt)
    hpt = torch.tensor((w / prob.h)[None, :, None], dtype=vdt, device="cuda").contiguous()
    d = pctx.fwd(hpt, pctx.empty_r()).clone()
    torch.cuda.synchronize()
    pctx.close()
    dist = torch.tensor(np.abs(prob.x_src0 + prob.h * np.arange(prob.ns) - prob.xs[0]),
                        dtype=vdt, device="cuda")

    def reduced(k):
        ctx = ssx.Context(prob, k, rho, field_dtype=fd)
        h, _, _, _ = ctx.pcg_solve(d, args.alpha, K, raise_on_breakdown=False)
        b = ctx.adj(d, ctx.empty_s())
        alpha = args.alpha * float(torch.linalg.norm(b.double())) / float(
            torch.linalg.norm(d.double()))
        e = ctx.fwd(h, ctx.empty_r()) - d
        J = 0.5 * float(torch.sum(e.double() ** 2)) + 0.5 * alpha ** 2 * float(
            torch.sum((dist * h).double() ** 2))
        return ctx, h, J

    k = inputs.crosswell_kappa(lens=False)
    e0 = float(np.linalg.norm(k - k_true))
    hist = []
    t0 = time.perf_counter()
    ctx, h, J = reduced(k)
    for it in range(args.outer):
        g, _ = ctx.misfit_gradient(h, d)
        gk = g[0].double().cpu().numpy()
        ctx.close()
        step = 0.05 * k.max() / max(np.abs(gk).max(), 1e-300)
        entry = {"outer": it, "reduced_objective": J,
                 "model_error": float(np.linalg.norm(k - k_true)) / e0}
        for _ in range(5):
            kn = k - step * gk
            cn, hn, Jn = reduced(kn)
            if Jn < J:
                break
            cn.close()
            step *= 0.5
        entry["step_halvings"] = _
        hist.append(entry)
        if Jn >= J:
            ctx = None
            break
        k, ctx, h, J = kn, cn, hn, Jn
    el = time.perf_counter() - t0
    if ctx is not None:
        hist.append({"outer": len(hist), "reduced_objective": J,
                     "model_error": float(np.linalg.norm(k - k_true)) / e0})
        ctx.close()
    out = {
        "metric": "variable-projection outer iterations/s (crosswell example)",
        "value": round(len(hist) / el, 4), "unit": "outer iterations/s", "n_gpus": 1,
        "steps": args.outer, "warmup": 0, "ms_per_step": round(1e3 * el / max(len(hist), 1), 1),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": fd,
        "data": "synthetic (lens model of the paper's shape; bandpass point source)",
        "config": {"workload": f"crosswell: {prob.nz}x{prob.nx} @ {prob.h} m, order "
                               f"{prob.order}, nt {prob.nt}, K {K}, alpha_rel {args.alpha}",
                   "nz": prob.nz, "nx": prob.nx, "nt": prob.nt, "K": K, "field_dtype": fd},
        "history": hist,
    }
    print(json.dumps(out), flush=True)


def bench3d(args):
    """The 3D form (ssx3_*): one step is F then F^T (the propagations of one
    normal-operator application) on a 201 x 201 x 401 grid (z, y, x) at 10 m
    with 20 absorbing cells per side (241 x 241 x 441 = 25.6 M cells), order
    8, nt 1000 (--nt), a seeded 3D layered model (1.5-4 km/s, constant
    density), the source plane at 1000 m and the receiver plane at 200 m
    over the whole lateral grid, FP32 fields (--dtype f64 for FP64).  The
    roofline is that of one time step (k3_vel + k3_pres) timed with events
    on the context's stream over a forward propagation, against 9 field
    values per cell-update (read p, v_x, v_y, v_z and ck; write p, v_x, v_y,
    v_z).  Also one timed subproblem solve (Algorithm 1 with the thin-slab
    M^-1, --iters iterations, default 5) on the data of the pairs."""
    import numpy as np
    import torch

    import inputs
    import paper_2203_16573_amd as ssx

    fd = args.dtype or "f32"
    rho = 1000.0
    nz, ny, nx, hh = 201, 201, 401, 10.0
    prob = inputs.Problem3(nz=nz, ny=ny, nx=nx, h=hh, dt=1e-3, nt=args.nt or 1000, order=8,
                           npml=20, z_src=1000.0, nsx=nx, nsy=ny, z_rec=200.0, nrx=nx,
                           nry=ny, slab_dz=5, x_s=(nx // 2) * hh, y_s=(ny // 2) * hh)
    vel = inputs.layered_velocity3(nz, ny, nx, hh, np.random.default_rng(inputs.BASE_SEED + 30))
    kap = rho * vel * vel
    ctx = ssx.Context3(prob, kap, rho, field_dtype=fd)
    h = ctx.empty_src()
    w = inputs.ricker((np.arange(prob.nt) + 0.5) * prob.dt, 15.0)
    h[:, ny // 2, nx // 2] = torch.tensor(w / hh ** 2, dtype=ctx.dtype, device="cuda")
    d = ctx.empty_rec()
    g = ctx.empty_src()

    def step():
        ctx.fwd(h, d)
        ctx.adj(d, g)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    el = (time.perf_counter() - t0) / args.steps
    # per-step kernel time of the forward sweep, events on the context's stream
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(ctx.stream)
    ctx.fwd(h, d)
    e1.record(ctx.stream)
    torch.cuda.synchronize()
    us_step = 1e3 * e0.elapsed_time(e1) / prob.nt
    NZ, NY, NX = nz + 40, ny + 40, nx + 40
    cells = NZ * NY * NX
    esz = 8 if fd == "f64" else 4
    achieved = 9 * esz * cells / (us_step * 1e-6) / 1e9
    out = {
        "metric": "3D F + F^T pairs/s", "value": round(1.0 / el, 4), "unit": "pairs/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(1e3 * el, 2), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": fd,
        "data": "synthetic (seeded 3D layered model; Ricker point source on the source plane)",
        "config": {"workload": f"3d: {nz}x{ny}x{nx} @ {hh} m, order 8, nt {prob.nt}, "
                               f"planes {ny}x{nx}", "nz": nz, "ny": ny, "nx": nx,
                   "nt": prob.nt, "field_dtype": fd},
        "gcell_updates_per_s": round(2 * prob.nt * cells / el / 1e9, 2),
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": 8000.0,
                     "unit": "GB/s", "frac": round(achieved / 8000.0, 4), "traffic": None,
                     "kernel": "k3_vel + k3_pres", "us_per_step": round(us_step, 3),
                     "bytes_per_cell": 9 * esz, "cells_per_step": cells},
        "cpu_baseline": None,
    }
    # one subproblem solve: Algorithm 1 with M^-1 = D W^-1 D on the thin slab
    # (K = --iters, default 5, alpha_rel 1e-3) on the data of the point source
    K = args.iters or 5
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    hs, hist, it = ctx.pcg_solve(d, 1e-3, K)
    torch.cuda.synchronize()
    ts = time.perf_counter() - t0
    out["pcg_solve"] = {"K": K, "iters": it, "seconds": round(ts, 3),
                        "solves_per_s": round(1.0 / ts, 4),
                        "rel_residual": [round(float(x), 5) for x in hist[:, 0] / hist[0, 0]],
                        "rel_misfit": [round(float(x), 5) for x in hist[:, 3] / hist[0, 3]]}
    if not args.no_cpu_baseline:
        # the oracle's 3D forward on the same grid for a few steps,
        # extrapolated linearly to the step's 2 nt cell-updates
        from oracle.prop3 import Grid3, forward3
        gph = Grid3(kap, rho, hh, prob.dt, 20, prob.pml_R, 8)
        src = gph.p_plane(prob.z_src, 0.0, nx, 0.0, ny)
        ns_ = 2
        tc = time.perf_counter()
        forward3(gph, ns_, h_src=(src, h[:ns_].double().cpu().numpy().reshape(ns_, -1)))
        tc = time.perf_counter() - tc
        rate = ns_ * cells / tc
        out["cpu_baseline"] = {
            "value": round(rate / (2 * prob.nt * cells), 8), "unit": "pairs/s", "cores": 1,
            "kind": "oracle",
            "sample": f"FP64 NumPy 3D oracle forward, {ns_} steps of the {NZ}x{NY}x{NX} grid "
                      f"({tc:.1f} s, {rate / 1e9:.4f} Gcell/s, 1 thread), extrapolated "
                      f"linearly to {2 * prob.nt * cells:.3e} cell-updates per pair"}
    ctx.close()
    print(json.dumps(out), flush=True)


def oracle_golden_errors(cnum, wl, prob, h, hist, args, weighted):
    """Errors of the last timed solve against the FP64 oracle's solve of the
    same problem, read from the expected values in tests/golden (written by
    the oracle alone; see tests/golden/make_full_length.py), when the
    workload is the one they were written for: the kept traces' relative L2
    error of h_K, the relative error of its norm, and of the residual
    history (||r_k|| per iteration, and each column as a vector)."""
    import numpy as np
    import inputs
    if weighted or args.rtol > 0 or args.nt or args.shots or args.iters or args.density:
        return None
    name = {2: "c2_full_length.npz", 4: "c2_full_length.npz", 3: "c3_full_length.npz"}.get(cnum)
    if name is None:
        return None
    path = os.path.join(ROOT, "tests", "golden", name)
    if not os.path.exists(path):
        return None
    z = np.load(path)
    hh = h.double().cpu().numpy()
    shots = [0] if cnum in (2, 4) else [int(s) for s in z["shots"]]
    out = {"reference": f"FP64 oracle, tests/golden/{name}", "shots": {}}
    for s in shots:
        key = "h" if cnum in (2, 4) else f"h{s}"
        hk = "hist" if cnum in (2, 4) else f"hist{s}"
        cols = z[f"{key}_cols"]
        ref = z[f"{key}_sample"].astype(np.float64)
        a = hh[s][:, cols]
        hr, hg = z[hk], hist[s]
        rk = np.abs(hg[:, 0] - hr[:, 0]) / hr[:, 0]
        out["shots"][str(s)] = {
            "h_rel_l2_kept_traces": float(np.linalg.norm(a - ref) / np.linalg.norm(ref)),
            "h_norm_rel_err": float(abs(np.linalg.norm(hh[s]) / float(z[f"{key}_norm"]) - 1)),
            "residual_per_iteration_max_rel_err": float(rk.max()),
            "residual_per_iteration_rel_err": [round(float(v), 6) for v in rk],
            "history_columns_rel_l2": [float(np.linalg.norm(hg[:, j] - hr[:, j]) /
                                             np.linalg.norm(hr[:, j])) for j in range(4)]}
    return out


def measured_traffic(config, fd, nshots, tile_z, group, loop, kernel):
    """HBM bytes per launch of the full-grid step kernel from the committed
    counter profile, when it was taken on the current kernel source with the
    same workload and launch shape; None otherwise."""
    import hashlib
    import re
    path = os.path.join(ROOT, "profiles", "k_step_hbm_traffic.md")
    csrc = os.path.join(ROOT, "paper_2203_16573_amd", "csrc")
    h = hashlib.sha256()
    try:
        text = open(path).read()
        for name in KERNEL_SOURCES:
            h.update(open(os.path.join(csrc, name), "rb").read())
    except OSError:
        return None
    digest = h.hexdigest()
    m = re.search(r"```json\n(.*?)\n```", text, re.S)
    if not m:
        return None
    table = json.loads(m.group(1))
    if table.get("kernel_source_sha256") != digest or kernel != "k_step":
        return None
    e = table["launches"].get(f"{config}|{fd}|shots{nshots}|tz{tile_z}|group{group}|loop{loop}")
    if e is None:
        return None
    fetch = e["fetch_kib"] * 1024 * table["fetch_scale"]
    write = e["write_kib"] * 1024 * table["write_scale"]
    return {"bytes_per_launch": round(fetch + write), "fetch_bytes": round(fetch),
            "write_bytes": round(write), "source": "profiles/k_step_hbm_traffic.md"}


def serve_bench(args):
    """Serving workload: the first --requests requests of the seeded stream
    (grids 201x401 / 401x801 / 801x1601, layered models, 1..--max-shots
    shots, 500..--max-nt steps, K = 20, FP16 storage), data generated on the
    device before timing.  A closed-loop pass (all queued at t = 0) measures
    capacity; an open-loop pass with Poisson arrivals at 0.8x that rate
    measures latency (with --rate-sweep also 0.5x, 1.0x and 1.2x).  Each
    request runs on its own stream with its propagations replayed as
    captured graphs (--graphs 0: plain launches)."""
    import numpy as np
    import torch

    import inputs
    import paper_2203_16573_amd as ssx
    from paper_2203_16573_amd import autotune, serve

    torch.cuda.set_device(0)
    stream = inputs.serving_requests(args.requests, max_shots=args.max_shots,
                                     nt_range=(500, args.max_nt))
    reqs = []
    for i, (t, wl) in enumerate(stream):
        prob = wl.prob
        gen = ssx.Context(prob, wl.kappa, wl.rho, field_dtype="f32")
        wav = inputs.source_wavelet(prob, wl.freq)
        htrue = np.stack([inputs.spike_gather(prob, wav, s) for s in range(prob.nshots)])
        d = gen.fwd(torch.tensor(htrue, dtype=torch.float32, device="cuda"), gen.empty_r())
        torch.cuda.synchronize()
        gen.close()
        reqs.append(serve.Request(i, prob, wl.kappa, wl.rho, d, alpha_rel=wl.alpha_rel, K=wl.K,
                                  field_dtype="f16", arrival=t))
    tuner = None
    t_tune = time.perf_counter()
    if args.autotune:
        def tuner(ctx, req):
            autotune.apply(ctx, autotune.choose(req.prob, req.kappa, req.rho, field_dtype="f16"))
        for r in reqs:  # tune every shape before timing
            autotune.choose(r.prob, r.kappa, r.rho, field_dtype="f16")
            print(f"# tuned request {r.rid}: {r.prob.nz}x{r.prob.nx}, {r.nshots} shots, "
                  f"nt {r.prob.nt}", flush=True)
    t_tune = time.perf_counter() - t_tune
    budget = int(0.8 * torch.cuda.mem_get_info()[0])
    def progress(res):
        print(f"# request {res.rid} done: latency {res.t_done - res.t_arrival:.2f} s", flush=True)

    srv = serve.Server(budget, slots=args.slots, graphs=bool(args.graphs), tuner=tuner,
                       on_done=progress, batch=args.batch)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    closed = srv.run(reqs, realtime=False)
    wall_closed = time.perf_counter() - t0
    cap = serve.summarize(closed, wall_closed)
    unit_gaps = np.random.default_rng(inputs.BASE_SEED + 5).exponential(1.0, size=len(reqs))

    def open_loop(factor):
        rate = factor * cap["requests_per_s"]
        for r, t in zip(reqs, np.cumsum(unit_gaps / rate)):
            r.arrival = float(t)
        t0 = time.perf_counter()
        res = srv.run(reqs, realtime=True)
        return res, serve.summarize(res, time.perf_counter() - t0)

    print(f"# closed loop: {cap}", flush=True)
    opened, lat = open_loop(0.8)
    print(f"# open loop 0.8x: {lat}", flush=True)
    same = all(torch.equal(a.h, b.h) for a, b in zip(closed, opened))
    sweep = {}
    if args.rate_sweep:
        for factor in (0.5, 1.0, 1.2):
            res, summ = open_loop(factor)
            same = same and all(torch.equal(a.h, b.h) for a, b in zip(closed, res))
            sweep[f"open_loop_{factor:g}x"] = summ
    # accuracy: shot 0 of every request solved again with FP64 fields and
    # vectors (that path matches the FP64 oracle to 1e-12 per full-length
    # propagation); the served FP16-storage solution's relative L2 error
    per_req = []
    for r, res in zip(reqs, closed):
        row = {"rid": r.rid, "grid": f"{r.prob.nz}x{r.prob.nx}", "shots": r.nshots,
               "nt": r.prob.nt, "latency_s": round(res.latency, 3),
               "admit_wait_s": round(res.t_admit - res.t_arrival, 3)}
        if args.c5_ref:
            p1 = r.prob.replace(xs=(r.prob.xs[0],))
            ref = ssx.Context(p1, r.kappa, r.rho, field_dtype="f64")
            h64, _, _, _ = ref.pcg_solve(r.d[:1].double().contiguous(), r.alpha_rel, r.K,
                                         raise_on_breakdown=False)
            torch.cuda.synchronize()
            ref.close()
            h16 = res.h[:1].double()
            row["h_err_vs_f64"] = float(torch.linalg.norm(h16 - h64) / torch.linalg.norm(h64))
        per_req.append(row)
    errs = [q["h_err_vs_f64"] for q in per_req if "h_err_vs_f64" in q]
    caps = ("none" if args.max_shots >= 64 and args.max_nt >= 4000
            else f"shots <= {args.max_shots}, nt <= {args.max_nt}")
    out = {
        "metric": "served PCG surface-source solves/s (p50/p99 latency)",
        "value": round(cap["solves_per_s"], 4), "unit": "solves/s", "n_gpus": 1,
        "steps": len(reqs), "warmup": 0,
        "ms_per_step": round(1e3 * wall_closed / len(reqs), 2),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f16-storage/f32", "data": "synthetic (seeded serving stream)",
        "config": {"workload": f"c5: first {len(reqs)} requests of the seeded stream "
                               f"(grids 201x401 / 401x801 / 801x1601, 1-64 shots, "
                               f"nt 500-4000), caps: {caps}, K 20, FP16 storage, "
                               f"{args.slots} slots, graphs {int(bool(args.graphs))}"
                               + (f", batches of up to {args.batch}" if args.batch > 1 else ""),
                   "requests": len(reqs), "caps": caps, "batch": args.batch,
                   "admission_budget_bytes": budget},
        "closed_loop": cap, "open_loop_0p8": lat, **sweep,
        "p50_latency_s": round(lat["latency_p50_s"], 3),
        "p99_latency_s": round(lat["latency_p99_s"], 3),
        "results_identical_closed_vs_open": same,
        "autotune_s": round(t_tune, 1),
        "accuracy": {"h_err_vs_f64_solve": {"median": float(np.median(errs)) if errs else None,
                                            "max": float(np.max(errs)) if errs else None,
                                            "ref": "shot 0 of each request, FP64 fields"}},
        "per_request": per_req,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
