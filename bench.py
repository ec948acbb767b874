"""Benchmark of the MLPG transport hot path on one MI355X.

Workload (the 2D manufactured-solution problem): 128 x 128 jittered lattice
on the unit square, linear RK with support radius 2h, 64 ordinates, sigma_t
= 1, sigma_s = 0.5, psi = sin(pi x) sin(pi y)(1 + mu/2) e^{-t}, 20
backward-Euler steps of dt = 0.01 with c = 1, FP64.  One timed step is the
whole path: neighbour lists, cells, integration, assembly and the 20
time steps (each: first-flight solve, outer GMRES on Phi with inner
batched GMRES, recovery solve).  Inputs (points, sources for every time
level, initial state) are resident in HBM before timing starts.

Metric: DOF x ordinate x Krylov-iteration per second = N * (Arnoldi steps
summed over ordinates and solves) / time.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import workloads as W  # noqa: E402

PEAK_HBM_GBS = 8000.0
# HBM traffic of the operator sweep from the counter passes, valid for the
# kernel source it was taken on
COUNTERS = os.path.join(ROOT, "profiles", "counters_spmv_2d_mms_128x128_m64.md")
SPMV_SOURCE = os.path.join(ROOT, "paper_2008_02205_amd", "csrc", "ops.hip")


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--scale", type=int, default=None, help="lattice points per axis (default 128)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-ordinates", type=int, default=0, help="ordinates in the CPU sample (0: all)")
    ap.add_argument("--precision", choices=["fp64", "mixed", "both"], default="both",
                    help="fp64: plain FP64 path; mixed: FP32 SpMV/basis inside FP64 refinement")
    ap.add_argument("--tol-lo", type=float, default=None, help="FP32 correction tolerance of the mixed path")
    ap.add_argument("--serving", type=int, default=0,
                    help="instead of the benchmark: serve this many requests of the seeded request stream "
                         "(Poisson arrivals at 50/s, mixed precision) and print latency and throughput")
    ap.add_argument("--slots", type=int, default=4, help="concurrent problems in the serving mode")
    ap.add_argument("--serving-sample", type=int, default=40,
                    help="after the benchmark, serve the first K requests of the seeded request stream and add "
                         "their latency p50/p99 and offered/achieved load to the record (0: skip)")
    ap.add_argument("--workload", type=int, default=2, choices=[1, 2, 3, 4, 6, 7, 8, 9],
                    help="2: the benchmark above; 1, 3, 4: time that workload's whole path instead (phase times, "
                         "p50/p99 over --steps repetitions) and print its own record; 6, 7: the paper's sinusoidal "
                         "and outgoing-wave manufactured problems (steady, [-1,1]^2, --scale points per axis), "
                         "with the relative error against the exact scalar flux; 8: workload 2 with points "
                         "that move every step (geometry, integration and assembly inside the time loop); 9: the asteroid of "
                         "Sec. 5.4 at one tenth of its lengths (shell materials, Alg. 2 refined quadrature, the "
                         "paper's graded point spacing coarsened --scale times, default 1, one large time step)")
    ap.add_argument("--be-steps", type=int, default=None, help="backward-Euler steps per repetition (workloads 3/4)")
    ap.add_argument("--max-outer", type=int, default=None,
                    help="outer-iteration cap per solve in the --workload mode (the record states convergence)")
    ap.add_argument("--max-inner", type=int, default=None, help="inner-iteration cap per solve (--workload mode)")
    ap.add_argument("--restart", type=int, default=None,
                    help="inner GMRES restart length, 1-60 (--workload mode; default 30, 60 for workload 9)")
    ap.add_argument("--graphs", action="store_true",
                    help="replay the inner solves' restart cycles from captured HIP graphs (default: one by one)")
    ap.add_argument("--precond", choices=["jacobi", "patch"], default=None,
                    help="right preconditioner of the inner solves: point Jacobi (the default) or patch block "
                         "Jacobi (the default of workload 9 and of the served requests)")
    ap.add_argument("--accel", action="store_true",
                    help="workload modes: diffusion-synthetic acceleration of the outer iteration (the served "
                         "requests use it by default)")
    ap.add_argument("--no-accel", action="store_true", help="serving: without the diffusion-synthetic acceleration")
    ap.add_argument("--probe", action="store_true",
                    help="hardware-counter probe: setup, one short solve of the workload and a 256 MiB "
                         "device copy (the reference for counter scaling); prints nothing")
    return ap.parse_args()


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on exactly one GPU: only the single-GPU path is "
                                   "implemented (sharding the ordinates across GPUs is a design, not code)"}))
        sys.exit(2)
    import torch
    from paper_2008_02205_amd import mlpg
    from paper_2008_02205_amd.problem import GpuProblem

    torch.cuda.set_device(0)
    mlpg.lib()
    if args.serving:
        serve(args)
        return
    if args.workload == 9:
        asteroid_workload(args)
        return
    if args.workload != 2:
        other_workload(args)
        return
    w = W.config(2, args.scale)
    x, dx = W.points_for(w)
    R = W.radii_for(w, x, dx)
    n = x.shape[0]
    om, wq = mlpg.mlpg_angular_quadrature(2, w.n_ord)
    M = om.shape[0]
    # resident inputs
    qs = [torch.from_numpy(np.ascontiguousarray(W.source_values(w, x, om, (s + 1) * w.dt))).cuda()
          for s in range(w.steps)]
    psi0 = torch.from_numpy(np.ascontiguousarray(W.initial_psi(w, x, om))).cuda()
    tau = torch.full((n,), dx, dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()

    def one_step(prec=mlpg.MLPG_FP64):
        P = GpuProblem(x, R, w.lo, w.hi)
        P.integrate(w.rk_order)
        P.assemble(om, wq, list(w.sigma_t), list(w.sigma_s), w.inv_c_dt, tau, precision=prec)
        P.set_state(psi0)
        its = 0
        sweeps = 0
        outer = 0
        solves = 0
        phi = pv = None
        opts = mlpg.mlpg_default_opts()
        opts.precond = mlpg.MLPG_PRECOND_PATCH if args.precond == "patch" else mlpg.MLPG_PRECOND_JACOBI
        opts.graphs = 1 if args.graphs else 0
        if args.tol_lo:
            opts.tol_inner_lo = args.tol_lo
        ref = f64c = 0
        for s in range(w.steps):
            phi, pv, _, info = P.step(qs[s], None, opts, want_psi=False)
            its += info["inner_iters"]
            sweeps += info["inner_sweeps"]
            outer += info["outer_iters"]
            solves += info["inner_solves"]
            ref += info["refinements"]
            f64c += info["fp64_completions"]
        P.close()
        extra["refinements"] = ref
        extra["fp64_completions"] = f64c
        return its, sweeps, outer, solves, pv

    extra = {}

    def timed(prec):
        for _ in range(args.warmup):
            one_step(prec)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        tot = {"its": 0, "sw": 0, "out": 0, "solves": 0, "refinements": 0, "fp64_completions": 0, "step_s": []}
        pv = None
        for _ in range(args.steps):
            ts = time.perf_counter()
            its, sw, out, solves, pv = one_step(prec)
            torch.cuda.synchronize()
            tot["step_s"].append(time.perf_counter() - ts)
            tot["its"] += its
            tot["sw"] += sw
            tot["out"] += out
            tot["solves"] += solves
            tot["refinements"] += extra["refinements"]
            tot["fp64_completions"] += extra["fp64_completions"]
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        # one more step, identical to the timed ones, with HIP events around every
        # launch of the profiled kernel classes (on the stream they run on)
        mlpg.mlpg_profile_begin()
        one_step(prec)
        prof = mlpg.mlpg_profile_end()
        return el, tot, pv, prof

    if args.probe:
        P = GpuProblem(x, R, w.lo, w.hi)
        P.integrate(w.rk_order)
        P.assemble(om, wq, list(w.sigma_t), list(w.sigma_s), w.inv_c_dt, tau)
        P.set_state(psi0)
        opts = mlpg.mlpg_default_opts()
        opts.max_inner = 60
        opts.max_outer = 1
        mlpg.mlpg_solve(P.h, qs[0], None, opts, want_psi=False, raise_on_error=False, ws=P.solve_workspace(opts))
        P.close()
        src = torch.empty(32 * 1024 * 1024, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        return

    runs = {}
    for name, prec in (("fp64", mlpg.MLPG_FP64), ("mixed", mlpg.MLPG_MIXED)):
        if args.precision in (name, "both"):
            runs[name] = timed(prec)
    main_name = "fp64" if "fp64" in runs else "mixed"
    el, tot, pv, prof = runs[main_name]
    tot_its, tot_sw, tot_out, tot_solves = tot["its"], tot["sw"], tot["out"], tot["solves"]
    ms = el / max(args.steps, 1) * 1e3
    value = n * tot_its / el
    ex = W.mms_sin_phi(x, w.steps * w.dt)
    err = float(np.abs(pv.cpu().numpy() - ex).sum() / ex.sum())

    rec = {
        "metric": "DOF*ordinate*Krylov-iter/s", "value": value, "unit": "DOF*ord*iter/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"2d-mms-be20: {int(math.sqrt(n))}^2 jittered lattice, linear RK, R=2h, "
                               f"{M} ordinates, 20 BE steps dt=0.01", "points": n, "ordinates": M,
                   "be_steps": w.steps},
        "detail": {"p50_step_s": float(np.percentile(tot["step_s"], 50)),
                   "p99_step_s": float(np.percentile(tot["step_s"], 99)),
                   "precond": args.precond or "jacobi", "graphs": bool(args.graphs),
                   "sweep_launch_shapes": mlpg.mlpg_get_tuning(),
                   "inner_iters_per_step": tot_its / max(args.steps, 1),
                   "batched_sweeps_per_step": tot_sw / max(args.steps, 1),
                   "outer_iters_per_step": tot_out / max(args.steps, 1),
                   "direction_solves_per_s": tot_solves * M / el,
                   "kernel_classes": {k: {"avg_us": 1e3 * v["ms"] / max(v["launches"], 1),
                                          "timed_launches": v["launches"],
                                          "GB_s": (v["bytes"] / (v["ms"] * 1e-3) / 1e9) if v["ms"] > 0 else None}
                                      for k, v in prof.items()},
                   "rel_l1_phi_vs_manufactured": err},
        "roofline": roofline(prof, shape=next((e for e in mlpg.mlpg_get_tuning()
                                               if (e["n"], e["n_ord"], e["streams"], e["value_bytes"]) ==
                                               (n, M, 6, 8)), None) if main_name == "fp64" else None),
        "cpu_baseline": None,
    }
    if "mixed" in runs and main_name != "mixed":
        el2, tot2, pv2, prof2 = runs["mixed"]
        pv_np, pv2_np = pv.cpu().numpy(), pv2.cpu().numpy()
        rec["detail"]["mixed"] = {
            "value": n * tot2["its"] / el2, "ms_per_step": el2 / max(args.steps, 1) * 1e3,
            "direction_solves_per_s": tot2["solves"] * M / el2,
            "speedup_direction_solves_vs_fp64": (tot2["solves"] * M / el2) / (tot_solves * M / el),
            "p50_step_s": float(np.percentile(tot2["step_s"], 50)),
            "p99_step_s": float(np.percentile(tot2["step_s"], 99)),
            "inner_iters_per_step": tot2["its"] / max(args.steps, 1),
            "refinements_per_step": tot2["refinements"] / max(args.steps, 1),
            "fp64_completions_per_step": tot2["fp64_completions"] / max(args.steps, 1),
            "rel_l2_phi_point_vs_fp64": float(np.linalg.norm(pv2_np - pv_np) / np.linalg.norm(pv_np)),
            "roofline": roofline(prof2)}
    if not args.no_cpu_baseline:
        rec["cpu_baseline"], X, k = cpu_baseline(w, x, R, dx, om, wq, args.cpu_ordinates)
        rec["detail"]["error_vs_oracle"] = oracle_error(w, x, R, dx, om, wq, psi0, X, k)
    if args.serving_sample:
        rec["detail"]["serving_sample"] = serving_record(args.serving_sample, args.slots, serving_opts(args))
    print(json.dumps(rec), flush=True)


def other_workload(args):
    """One workload's whole path (geometry, integration, assembly, every solve of a repetition) timed
    phase by phase, with p50/p99 over repetitions; FP64 and mixed where the workload asks for both."""
    import torch
    from paper_2008_02205_amd import mlpg
    from paper_2008_02205_amd.problem import GpuProblem
    w = W.config(args.workload, args.scale)
    x, dx = W.points_for(w)
    R = W.radii_for(w, x, dx)
    n = x.shape[0]
    kind = mlpg.MLPG_QUAD_BEAM_DENSE if w.ord_kind == "beam-dense" else mlpg.MLPG_QUAD_PRODUCT
    om, wq = mlpg.mlpg_angular_quadrature(w.dim, w.n_ord, kind)
    M = om.shape[0]
    steps = w.steps if w.steps > 0 else 1
    if args.be_steps:
        steps = min(steps, args.be_steps)
    # moving points: the positions of every step are inputs (the caller's motion), made before timing
    xs = [x]
    for s in range(steps if w.velocity else 0):
        xs.append(W.advect_points(w, xs[-1], w.dt))
    qs = [torch.from_numpy(np.ascontiguousarray(
        W.source_values(w, xs[s + 1] if w.velocity else x, om, w.t0 + (s + 1) * w.dt))).cuda()
        for s in range(steps)]
    psi0 = torch.from_numpy(np.ascontiguousarray(W.initial_psi(w, x, om))).cuda()
    tau = torch.full((n,), dx, dtype=torch.float64, device="cuda")
    precs = {1: ("fp64",), 3: ("mixed",), 4: ("mixed", "fp64"), 6: ("fp64", "mixed"),
             7: ("fp64", "mixed"), 8: ("fp64", "mixed")}[args.workload]
    exact = None
    if w.source in ("paper-cos", "paper-wave"):
        exact = 4.0 * np.pi * W.paper_mms_psi(w, x, w.t0 + steps * w.dt)
    elif w.source == "mms-sin":
        exact = W.mms_sin_phi(xs[-1], w.t0 + steps * w.dt)
    if args.precision != "both":
        precs = (args.precision,)

    def sync_time():
        torch.cuda.synchronize()
        return time.perf_counter()

    t_start = time.perf_counter()

    def progress(level, iters, resid):
        print(f"[{w.name}] {'outer' if level else 'inner'} solve done: {iters} Krylov steps, residual {resid:.1e}, "
              f"{time.perf_counter() - t_start:.0f} s", file=sys.stderr, flush=True)

    mlpg.mlpg_set_progress(progress)

    def rep(prec):
        t = {}
        t0 = sync_time()
        P = GpuProblem(x, R, w.lo, w.hi, w.regions, w.fields)
        t1 = sync_time()
        info = P.integrate(w.rk_order)
        t2 = sync_time()
        P.assemble(om, wq, list(w.sigma_t), list(w.sigma_s), w.inv_c_dt, tau,
                   precision=mlpg.MLPG_FP64 if prec == "fp64" else mlpg.MLPG_MIXED)
        P.set_state(psi0)
        pb = None
        if w.inflow != "vacuum":
            y, _ = P.boundary_points()
            pb = torch.from_numpy(np.ascontiguousarray(W.inflow_values(w, y.cpu().numpy(), om))).cuda()
        t3 = sync_time()
        print(f"[{w.name} {prec}] setup: geometry {t1 - t0:.2f} s, integrate {t2 - t1:.2f} s, "
              f"assemble {t3 - t2:.2f} s", file=sys.stderr, flush=True)
        its = solves = outer = 0
        conv = True
        opts = mlpg.mlpg_default_opts()
        opts.precond = mlpg.MLPG_PRECOND_PATCH if args.precond == "patch" else mlpg.MLPG_PRECOND_JACOBI
        if args.accel:
            opts.accel = mlpg.MLPG_ACCEL_DSA
        if args.max_outer:
            opts.max_outer = args.max_outer
        if args.restart:
            opts.restart_inner = args.restart
        if args.max_inner:
            opts.max_inner = args.max_inner
        err = None
        mv = {"geometry_s": 0.0, "integrate_s": 0.0, "assemble_s": 0.0}
        for s in range(steps):
            if w.velocity:
                # the points have moved: neighbours, cells, integration and assembly again
                ta = sync_time()
                P.move(xs[s + 1], R)
                tb = sync_time()
                P.integrate(w.rk_order)
                tc = sync_time()
                P.assemble(om, wq, list(w.sigma_t), list(w.sigma_s), w.inv_c_dt, tau,
                           precision=mlpg.MLPG_FP64 if prec == "fp64" else mlpg.MLPG_MIXED)
                td = sync_time()
                mv["geometry_s"] += tb - ta; mv["integrate_s"] += tc - tb; mv["assemble_s"] += td - tc
            _, pv, _, inf = mlpg.mlpg_solve(P.h, qs[s], pb, opts, want_psi=False, raise_on_error=False,
                                            ws=P.solve_workspace(opts))
            conv = conv and inf["converged"] == 1
            its += inf["inner_iters"]
            solves += inf["inner_solves"]
            outer += inf["outer_iters"]
            print(f"[{w.name} {prec}] step {s + 1}/{steps}: outer {inf['outer_iters']}, inner solves "
                  f"{inf['inner_solves']}, Krylov steps {inf['inner_iters']}, {time.perf_counter() - t3:.1f} s",
                  file=sys.stderr, flush=True)
        t4 = sync_time()
        if w.velocity:
            # per-step rebuild times are reported separately from the solves
            t_solve = t4 - t3 - sum(mv.values())
        else:
            t_solve = t4 - t3
        if exact is not None:
            # relative error of the scalar flux at the centres (Sec. 5): sum |phi - phi_exact| / sum phi_exact
            err = float(np.abs(pv.cpu().numpy() - exact).sum() / exact.sum())
        P.close()
        return {"geometry_s": t1 - t0 + mv["geometry_s"], "integrate_s": t2 - t1 + mv["integrate_s"],
                "assemble_s": t3 - t2 + mv["assemble_s"], "solve_s": t_solve,
                "total_s": t4 - t0, "iters": its, "solves": solves, "outer": outer,
                "fallback_qps": info["fallback_qps"], "converged": conv, "rel_error": err,
                "rebuild_per_step_s": sum(mv.values()) / steps if w.velocity else None}

    out = {}
    for prec in precs:
        for _ in range(args.warmup):
            rep(prec)
        rs = [rep(prec) for _ in range(max(args.steps, 1))]
        tot = np.array([r["total_s"] for r in rs])
        out[prec] = {"value": float(np.mean([n * r["iters"] / r["total_s"] for r in rs])),
                     "direction_solves_per_s": float(np.mean([r["solves"] * M / r["total_s"] for r in rs])),
                     "p50_total_s": float(np.percentile(tot, 50)), "p99_total_s": float(np.percentile(tot, 99)),
                     "phases_s": {k: float(np.mean([r[k] for r in rs]))
                                  for k in ("geometry_s", "integrate_s", "assemble_s", "solve_s")},
                     "iters_per_rep": rs[0]["iters"], "outer_per_rep": rs[0]["outer"],
                     "fallback_qps": rs[0]["fallback_qps"], "converged": all(r["converged"] for r in rs),
                     "rel_error_vs_exact": rs[0]["rel_error"],
                     "rebuild_per_step_s": rs[0]["rebuild_per_step_s"],
                     "max_outer": args.max_outer, "max_inner": args.max_inner}
    main_p = precs[0]
    rec = {"metric": "DOF*ordinate*Krylov-iter/s", "value": out[main_p]["value"], "unit": "DOF*ord*iter/s",
           "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "higher_is_better": True,
           "dtype": "f64" if main_p == "fp64" else "f32+f64", "data": "synthetic",
           "config": {"workload": f"{w.name}: {n} points, {M} ordinates, rk order {w.rk_order}, "
                                  f"{'steady' if w.steps == 0 else f'{steps} BE steps'}", "points": n,
                      "ordinates": M, "dim": w.dim, "accel": "dsa" if args.accel else "none"},
           "detail": out}
    print(json.dumps(rec), flush=True)


ASTEROID_RESTART = 60


def asteroid_workload(args):
    """Sec. 5.4 asteroid at one tenth of the paper's lengths: an absorbing shell (20 mean free paths)
    lit by a small source through the Alg. 2 refined quadrature (goal 2048 ordinates), on points at
    the paper's graded spacing (0.1-1.0 in its units; ``--scale k`` coarsens it k times), one
    backward-Euler step from zero radiation long enough to cross the domain.  The error is taken where
    the refined ordinates resolve the flux (the lit cone in front of the asteroid), weighted by the
    points' shares of the area, against the exact line-source flux for the same polar levels with the
    step's 1/(c dt) added to the absorption."""
    import torch
    from paper_2008_02205_amd import mlpg
    from paper_2008_02205_amd.problem import GpuProblem
    a = W.asteroid(0.1)
    coarsen = float(args.scale) if args.scale else 1.0
    x, R, L = W.asteroid_graded_points(a, coarsen)
    shells, st, ss = W.asteroid_materials(a)
    a0 = W.asteroid_step_inv_c_dt(a)
    om, wq = mlpg.mlpg_refined_quadrature(0, 8, a.src, (0.0, 0.0), a.radius)
    n, M = x.shape[0], om.shape[0]
    q = torch.from_numpy(np.ascontiguousarray(W.asteroid_source(a, x, M))).cuda()
    tau = torch.from_numpy(L).cuda()
    xg, wg = np.polynomial.legendre.leggauss(4)
    exact = W.asteroid_phi_ordinates(a, x, xg[xg > 0], wg[xg > 0], a0)
    lit = W.asteroid_lit_region(a, x, 1.0)
    area = L * L
    precs = ("fp64", "mixed") if args.precision == "both" else (args.precision,)

    def sync_time():
        torch.cuda.synchronize()
        return time.perf_counter()

    def rep(prec):
        t0 = sync_time()
        P = GpuProblem(x, R, a.lo, a.hi, shells=shells)
        t1 = sync_time()
        info = P.integrate(1)
        t2 = sync_time()
        P.assemble(om, wq, list(st), list(ss), a0, tau, precision=mlpg.MLPG_FP64 if prec == "fp64" else mlpg.MLPG_MIXED)
        t3 = sync_time()
        opts = mlpg.mlpg_default_opts()
        opts.precond = mlpg.MLPG_PRECOND_JACOBI if args.precond == "jacobi" else mlpg.MLPG_PRECOND_PATCH
        # on the graded points restarted GMRES(30) stalls near a relative residual of 0.5 on some
        # ordinates of the oblique polar level (with point Jacobi at twice the paper's spacing, with
        # the patch preconditioner too at its own); GMRES(60) with the patch preconditioner converges
        # every ordinate within the library's default cap of 3,000 steps, so these are this
        # workload's defaults
        if args.max_inner:
            opts.max_inner = args.max_inner
        opts.restart_inner = args.restart or ASTEROID_RESTART
        if args.accel:
            opts.accel = mlpg.MLPG_ACCEL_DSA
        _, pv, _, inf = mlpg.mlpg_solve(P.h, q, None, opts, want_psi=False, raise_on_error=False,
                                        ws=P.solve_workspace(opts))
        t4 = sync_time()
        pv = pv.cpu().numpy()
        P.close()
        print(f"[asteroid {prec}] geometry {t1 - t0:.2f} s, integrate {t2 - t1:.2f} s, assemble {t3 - t2:.2f} s, "
              f"solve {t4 - t3:.2f} s, Krylov steps {inf['inner_iters']}", file=sys.stderr, flush=True)
        return {"geometry_s": t1 - t0, "integrate_s": t2 - t1, "assemble_s": t3 - t2, "solve_s": t4 - t3,
                "total_s": t4 - t0, "iters": inf["inner_iters"], "converged": inf["converged"] == 1,
                "lit_rel_error": float((area[lit] * np.abs(pv[lit] - exact[lit])).sum() / (area[lit] * exact[lit]).sum()),
                "negative_fraction": float(np.mean(pv < 0.0)), "negative_area_fraction": float(area[pv < 0.0].sum() / area.sum()),
                "fallback_qps": info["fallback_qps"]}

    out = {}
    for prec in precs:
        for _ in range(args.warmup):
            rep(prec)
        rs = [rep(prec) for _ in range(max(args.steps, 1))]
        tot = np.array([r["total_s"] for r in rs])
        out[prec] = {"value": float(np.mean([n * r["iters"] / r["total_s"] for r in rs])),
                     "direction_solves_per_s": float(np.mean([M / r["total_s"] for r in rs])),
                     "p50_total_s": float(np.percentile(tot, 50)), "p99_total_s": float(np.percentile(tot, 99)),
                     "phases_s": {k: float(np.mean([r[k] for r in rs]))
                                  for k in ("geometry_s", "integrate_s", "assemble_s", "solve_s")},
                     "iters_per_rep": rs[0]["iters"], "converged": all(r["converged"] for r in rs),
                     "lit_rel_error_vs_exact": rs[0]["lit_rel_error"], "lit_points": int(lit.sum()),
                     "negative_fraction": rs[0]["negative_fraction"],
                     "negative_area_fraction": rs[0]["negative_area_fraction"], "fallback_qps": rs[0]["fallback_qps"]}
    main_p = precs[0]
    rec = {"metric": "DOF*ordinate*Krylov-iter/s", "value": out[main_p]["value"], "unit": "DOF*ord*iter/s",
           "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "higher_is_better": True,
           "dtype": "f64" if main_p == "fp64" else "f32+f64", "data": "synthetic",
           "config": {"workload": f"asteroid (lengths x0.1, graded spacing x{coarsen:g}): {n} points, {M} refined "
                                  f"ordinates, one backward-Euler step (c dt = {1.0 / a0:.0f})",
                      "points": n, "ordinates": M, "dim": 2, "accel": "dsa" if args.accel else "none",
                      "precond": args.precond or "patch", "restart": args.restart or ASTEROID_RESTART},
           "detail": out}
    print(json.dumps(rec), flush=True)


def serving_record(k, slots, opts):
    """The first k requests of the seeded request stream (Poisson arrivals at 50/s, real time) through
    the request server: latency p50/p99 from arrival to result, offered and achieved load, aggregate
    iteration rate, and the exact device bytes of the requests against their admission bounds."""
    from paper_2008_02205_amd import mlpg
    from paper_2008_02205_amd.serving import Server, latency_summary

    def build(spec):
        x, R, dx = W.request_problem(spec)
        om, wq = mlpg.mlpg_angular_quadrature(2, spec.n_ord)
        return x, R, dx, om, wq, spec.sigma_t, spec.sigma_s, np.ones((x.shape[0], spec.n_ord))

    specs = W.request_stream(k)
    t0 = time.perf_counter()

    def done(r, nd):
        if nd % 25 == 0 or nd == k:
            print(f"[serving] {nd}/{k} requests done, {time.perf_counter() - t0:.0f} s", file=sys.stderr, flush=True)

    res = Server(slots=slots, opts=opts).run(specs, build, realtime=True, keep_fields=False, on_done=done)
    el = time.perf_counter() - t0
    summ = latency_summary(res)
    its = sum(r.info["inner_iters"] * r_spec.side ** 2 for r, r_spec in zip(res, specs) if r.info)
    errors = {}
    for r in res:
        if r.error is not None:
            errors[r.error[:160]] = errors.get(r.error[:160], 0) + 1
    return {"requests": k, "slots": slots, "p50_s": summ["p50_s"], "p99_s": summ["p99_s"],
            "mean_s": summ["mean_s"], "failed": summ["failed"], "errors": errors,
            "offered_req_s": len(specs) / specs[-1].arrival if specs[-1].arrival > 0 else None,
            "achieved_req_s": summ["throughput_req_s"], "DOF*ord*iter_per_s": its / el, "wall_s": el,
            "exact_bytes_over_admission_bound": summ["exact_over_reserved"],
            "workload": "steady 2D problems, N log-uniform in [1024, 65536] (square lattices), M in "
                        "{16,32,64,128}, sigma_t log-uniform [0.1,100], c uniform [0,0.95], mixed precision"}


def serving_opts(args):
    """Solver options of the served requests: the patch preconditioner unless --precond jacobi and the
    diffusion-synthetic acceleration unless --no-accel (on the first 120 requests of the stream: 1.80
    requests/s with neither, 2.76 with the patch preconditioner, 3.06 with both)."""
    from paper_2008_02205_amd import mlpg
    opts = mlpg.mlpg_default_opts()
    opts.precond = mlpg.MLPG_PRECOND_JACOBI if args.precond == "jacobi" else mlpg.MLPG_PRECOND_PATCH
    if not args.no_accel:
        opts.accel = mlpg.MLPG_ACCEL_DSA
    return opts


def serve(args):
    """Request-stream mode: continuous batching with HBM-budget admission."""
    r = serving_record(args.serving, args.slots, serving_opts(args))
    rec = {"metric": "request-stream latency (p50/p99) and throughput", "value": r["p50_s"], "unit": "s",
           "higher_is_better": False, "n_gpus": 1, "dtype": "f32+f64", "data": "synthetic",
           "config": {"workload": f"request stream: {args.serving} " + r["workload"] + ", Poisson arrivals at 50/s",
                      "slots": args.slots, "accel": "none" if args.no_accel else "dsa",
                      "precond": args.precond or "patch"},
           "serving": r}
    print(json.dumps(rec), flush=True)


def roofline(prof, shape=None):
    """Dominant kernel class of the profiled step against the HBM peak.

    achieved = algorithmic bytes per launch (each operand once; see the
    per-class byte model in the library) / average launch duration.  With
    `shape` (the sweep's tuned launch shape), traffic is the counters' HBM
    bytes per launch of the sweep in that shape."""
    name = max(prof, key=lambda k: prof[k]["ms"])
    v = prof[name]
    if v["launches"] == 0 or v["ms"] <= 0:
        return None
    avg_s = v["ms"] * 1e-3 / v["launches"]
    per_launch = v["bytes"] / v["launches"]
    achieved = per_launch / avg_s / 1e9
    traffic, key = measured_traffic(shape) if shape and name == "spmv_L" else (None, None)
    return {"kernel": name, "bound": "hbm", "achieved": achieved, "peak": PEAK_HBM_GBS, "unit": "GB/s",
            "frac": achieved / PEAK_HBM_GBS, "traffic": traffic, "traffic_shape": key,
            "avg_launch_us": avg_s * 1e6, "algorithmic_bytes_per_launch": per_launch}


def shape_key(e):
    """The counters file's key of a launch-shape table entry."""
    if e["form"] == 1:
        return f"form=1 waves={e['waves_per_block']} rounds={e['rounds']} xcd={e['xcd_split']}"
    if e["form"] == 2:
        return (f"form=2 ords={e['ords_per_lane']} waves={e['waves_per_block']} items={e['items_per_wave']} "
                f"xcd={e['xcd_split']}")
    return f"form=0 waves={e['waves_per_block']} items={e['items_per_wave']} xcd={e['xcd_split']}"


def measured_traffic(shape):
    """HBM bytes per launch of the operator sweep in launch shape `shape` (FETCH_SIZE and WRITE_SIZE
    scaled against a copy of known size) and the shape's key, or (None, key) when the kernel source has
    changed since the counters were taken or the shape was not measured."""
    import hashlib
    key = shape_key(shape)
    try:
        txt = open(COUNTERS).read()
        src = hashlib.sha256(open(SPMV_SOURCE, "rb").read()).hexdigest()
    except OSError:
        return None, key
    kv = dict(line.split(": ", 1) for line in txt.splitlines()
              if line.startswith(("source_sha256:", "traffic_bytes_per_launch ")))
    if kv.get("source_sha256", "").strip() != src:
        return None, key
    v = kv.get("traffic_bytes_per_launch " + key)
    return (float(v) if v is not None else None), key


def cpu_baseline(w, x, R, dx, om, wq, k, min_seconds=10.0):
    """The oracle on a bounded sample of the same workload: the first-flight
    inner solves L_m^-1 F of the first backward-Euler step for the first k
    ordinates (all by default), repeated until at least ``min_seconds`` of
    CPU work has been timed."""
    import oracle
    g = oracle.geometry(x, R, w.lo, w.hi)
    it = oracle.integrate(g, w.rk_order)
    tr = oracle.Transport(it, om, wq, w.sigma_t[0], w.sigma_s[0], w.inv_c_dt, dx)
    psi0 = W.initial_psi(w, x, om)
    F = tr.rhs(psi0, W.source_values(w, x, om, w.dt), None)
    th = oracle.num_threads()
    k = k or om.shape[0]
    its = 0
    reps = 0
    t0 = time.perf_counter()
    while True:
        X, i, _ = tr.inner_solve(F, 0, k)
        its += i
        reps += 1
        el = time.perf_counter() - t0
        if el >= min_seconds:
            break
    # the same sample on one thread (one ordinate's solves: the oracle runs one ordinate per thread)
    t1 = time.perf_counter()
    _, i1, _ = tr.inner_solve(F, 0, 1)
    el1 = time.perf_counter() - t1
    rec = {"value": x.shape[0] * its / el, "unit": "DOF*ord*iter/s", "cores": th, "kind": "oracle",
           "cpu_model": cpu_model(),
           "one_thread_value": x.shape[0] * i1 / el1,
           "sample": f"first-flight inner GMRES solves (right-Jacobi GMRES(30) to 1e-13) of BE step 1 for "
                     f"ordinates 0..{k - 1} of {om.shape[0]}, full {x.shape[0]}-point problem, x{reps}: "
                     f"{its} Arnoldi steps in {el:.1f} s on {th} threads; one thread: ordinate 0 alone, "
                     f"{i1} Arnoldi steps in {el1:.2f} s"}
    return rec, X, k


def oracle_error(w, x, R, dx, om, wq, psi0, X, k):
    """Relative L2 error of the GPU path against the oracle's solutions of the CPU
    sample, X = L_m^-1 (T psi^0 + r) for ordinates 0..k-1: the first backward-Euler
    step of the same problem without scattering (sigma_s = 0, which changes
    neither L_m nor the right-hand side), where the step's Psi is exactly X."""
    import torch
    from paper_2008_02205_amd import mlpg
    from paper_2008_02205_amd.problem import GpuProblem
    q = torch.from_numpy(np.ascontiguousarray(W.source_values(w, x, om, w.dt))).cuda()
    tau = torch.full((x.shape[0],), dx, dtype=torch.float64, device="cuda")
    out = {"sample": f"Psi of BE step 1 with sigma_s = 0 against the oracle's L_m^-1 F of the CPU sample, "
                     f"ordinates 0..{k - 1}"}
    ref = X[:, :k]
    for name, prec in (("fp64", mlpg.MLPG_FP64), ("mixed", mlpg.MLPG_MIXED)):
        P = GpuProblem(x, R, w.lo, w.hi)
        P.integrate(w.rk_order)
        P.assemble(om, wq, [w.sigma_t[0]], [0.0], w.inv_c_dt, tau, precision=prec)
        P.set_state(psi0)
        _, _, psi, _ = P.step(q, None, mlpg.mlpg_default_opts())
        got = psi.cpu().numpy()[:, :k]
        P.close()
        out[name] = float(np.linalg.norm(got - ref) / np.linalg.norm(ref))
    return out


def cpu_model():
    """The host CPU's model name (lscpu), or None."""
    import subprocess
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
    except (OSError, subprocess.SubprocessError):
        return None
    for line in out.splitlines():
        if line.startswith("Model name:"):
            return line.split(":", 1)[1].strip()
    return None


if __name__ == "__main__":
    main()
