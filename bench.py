#!/usr/bin/env python3
"""Benchmark: ms per Stokes solve to 1e-8 relative residual, 256^3, density ratio 1000.

One step = one full stokes_solve (FGMRES + projection preconditioner + multigrid)
of the seeded 256^3 air/water/solid workload (eval seed 900000) with inputs
resident in HBM; setup (coefficients, hierarchy) is timed separately.  Prints
one JSON line with a "roofline" object for the dominant kernel (the fused
finest-level pressure sweep, timed live with HIP events inside the library on
the solve's stream) and a "cpu_baseline" object (the C oracle on this host's
cores, on a bounded sample of the same workload).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--precision", type=int, default=0, help="0 FP64 multigrid, 1 FP32 multigrid")
    ap.add_argument("--n", type=int, default=256, help="cells per axis of the headline workload")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--opt", action="append", default=[],
                    help="solver option override key=value (fields of stokes_options)")
    ap.add_argument("--prof-kernel", type=int, default=1,
                    help="kernel class timed for the roofline (0 matvec, 1 pressure sweep, 2 multidot, 3 maxpy)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="first run a plain 1 GiB device copy (reference for HBM counter runs)")
    ap.add_argument("--no-forms", action="store_true",
                    help="skip the FP32-multigrid form timed after the plain FP64 solve")
    ap.add_argument("--traffic-from", nargs=2, metavar=("FETCH_DIR", "WRITE_DIR"),
                    help="no solve: turn the rocprofv3 FETCH_SIZE and WRITE_SIZE counter runs of "
                         "'bench.py --calibrate-copy' into profiles/traffic.json and print a summary")
    ap.add_argument("--no-configs", action="store_true",
                    help="skip the config 3 (128^3) and config 4 (1024x96x96) legs")
    ap.add_argument("--learned-study", type=int, default=0, metavar="SEEDS",
                    help="no bench line: measure what a (perfect or learned) initial guess is worth to the "
                         "pressure cycles on SEEDS fresh instances of the headline recipe, and the U-Net's "
                         "forward cost from 32^3 to 256^3; prints one JSON line")
    ap.add_argument("--velocity-mg-only", action="store_true",
                    help="no bench line: run only the viscous-dominated velocity-multigrid leg and print it")
    ap.add_argument("--verbose", action="store_true")
    return ap.parse_args()


def log(*a):
    print(*a, file=sys.stderr, flush=True)


class Legs:
    """Runs the measurements beside the headline one at a time, so that a failing
    leg (a solve that does not converge, missing weights, a host-side error) is
    reported in its own field and the headline line is still printed.  After a
    HIP error nothing more is launched on the GPU: the later GPU legs are
    recorded as skipped; host-only legs still run."""

    def __init__(self):
        self.gpu_ok = True

    def run(self, name, fn, *args, gpu=True):
        if gpu and not self.gpu_ok:
            return {"skipped": "an earlier leg hit a HIP error"}
        try:
            return fn(*args)
        except Exception as e:          # noqa: BLE001 -- reported, not swallowed
            msg = "%s: %s" % (type(e).__name__, e)
            log("leg %s failed: %s" % (name, msg))
            if gpu and ("HIP" in msg or getattr(e, "status", None) == -4):
                self.gpu_ok = False
            return {"error": msg}


def main():
    args = parse()
    if args.traffic_from:
        traffic_from_counters(*args.traffic_from, n=args.n, precision=args.precision)
        return
    if args.velocity_mg_only and args.gpus == 1:
        import paper_1901_07892_amd as S
        print(json.dumps(velocity_mg_leg(S)), flush=True)
        return
    if args.learned_study and args.gpus == 1:
        print(json.dumps(learned_study(args.learned_study, args.n)), flush=True)
        return
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the solve is a single-GPU kernel path "
              "(no multi-GPU sharding is built); use --gpus 1", file=sys.stderr)
        sys.exit(2)
    import torch
    import workloads as W
    import paper_1901_07892_amd as S

    if args.calibrate_copy:
        a = torch.empty(1 << 27, dtype=torch.float64, device="cuda")
        b = torch.empty_like(a)
        a.fill_(1.0)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        log("calibration copy: 3 x 1 GiB read + 1 GiB write")
        del a, b
    t0 = time.time()
    prob = W.config5(n_cells=args.n)
    log("workload %s generated in %.1fs; solids: %d" % (prob.name, time.time() - t0, len(prob.solids)))
    dev = torch.device("cuda:0")
    td = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    rho = [td(r) for r in prob.rho_faces[:3]]
    mu = td(prob.mu)
    rhs_u = [td(f) for f in prob.rhs_u[:3]]
    rhs_p = td(prob.rhs_p)
    xu = [torch.zeros_like(f) for f in rhs_u]
    xp = torch.zeros_like(rhs_p)
    torch.cuda.synchronize()

    ts = time.time()
    overrides = {"precision": args.precision}
    for kv in args.opt:
        k, v = kv.split("=")
        overrides[k] = float(v) if k in ("visc_scale", "cont_scale") else int(v)
    solver = S.StokesSolver(3, prob.n, prob.h, rho, mu, prob.dt, **overrides)
    torch.cuda.synchronize()
    setup_ms = (time.time() - ts) * 1e3
    log("setup %.1f ms, workspace %.2f GB" % (setup_ms, solver.ws_bytes / 1e9))

    def step():
        for a in xu:
            a.zero_()
        xp.zero_()
        st, stats = solver.solve(rhs_u, rhs_p, prob.tol, xu, xp)
        if st != 0:
            raise RuntimeError("solve did not converge: %s" % stats.as_dict())
        return stats

    for w in range(args.warmup):
        stats = step()
        log("warmup %d: iters %d res %.3e ms %.2f" % (w, stats.iters, stats.rel_res_true, stats.ms_total))
    torch.cuda.synchronize()
    S.stokes_profile_kernel(solver.ctx, args.prof_kernel)
    times = []
    iters = []
    t_all0 = time.perf_counter()
    for s in range(args.steps):
        t1 = time.perf_counter()
        stats = step()
        torch.cuda.synchronize()
        times.append((time.perf_counter() - t1) * 1e3)
        iters.append(stats.iters)
        log("step %d: %.2f ms iters %d res %.3e" % (s, times[-1], stats.iters, stats.rel_res_true))
    torch.cuda.synchronize()
    total_ms = (time.perf_counter() - t_all0) * 1e3
    ms = total_ms / args.steps
    n_cells = prob.n_cells
    kms, klaunch, kbytes = S.stokes_profile_read(solver.ctx)
    S.stokes_profile_kernel(solver.ctx, -1)
    names = {0: "k_apply3_z (Stokes matvec)", 1: "k_p_sweep3c (fused pressure red-black sweep, finest level)",
             2: "k_multidot", 3: "k_maxpy"}
    achieved = kbytes / (kms * 1e-3) / 1e9 if kms > 0 else None
    roofline = {"bound": "hbm", "kernel": names.get(args.prof_kernel),
                "achieved": achieved, "peak": 8000.0, "unit": "GB/s",
                "frac": achieved / 8000.0 if achieved else None,
                "traffic": traffic_per_launch(args.prof_kernel, args.n, args.precision),
                "launches": klaunch, "avg_launch_us": kms * 1e3 / max(klaunch, 1),
                "algorithmic_bytes_per_launch": kbytes / max(klaunch, 1)}
    # the other kernel classes, one solve each (outside the timed steps)
    kernels = {names[args.prof_kernel]: {"launches": klaunch, "avg_launch_us": kms * 1e3 / max(klaunch, 1),
                                         "algorithmic_GBps": achieved}}
    for kind in (0, 2, 3):
        if kind == args.prof_kernel:
            continue
        S.stokes_profile_kernel(solver.ctx, kind)
        step()
        torch.cuda.synchronize()
        a_ms, a_n, a_b = S.stokes_profile_read(solver.ctx)
        S.stokes_profile_kernel(solver.ctx, -1)
        kernels[names[kind]] = {"launches": a_n, "avg_launch_us": a_ms * 1e3 / max(a_n, 1),
                                "algorithmic_GBps": a_b / (a_ms * 1e-3) / 1e9 if a_ms > 0 else None}
    out = {
        "metric": "ms per Stokes solve to 1e-8 rel. residual, 256^3 rho-ratio 1000",
        "value": ms,
        "unit": "ms/solve",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.precision == 0 else "f64 (f32 multigrid)",
        "data": "synthetic",
        "config": {"workload": prob.name + " air/water/solids density ratio 1000, seed 900000",
                   "tol": prob.tol, "dt": prob.dt, "precision": args.precision,
                   "options": {k: getattr(solver.opts, k) for k, _ in solver.opts._fields_}},
        "solves_per_s": 1e3 / ms,
        "median_ms": float(np.median(times)),
        "fgmres_iters": int(np.median(iters)),
        "cell_updates_per_s": n_cells * float(np.median(iters)) / (ms * 1e-3),
        "setup_ms": setup_ms,
        "rel_res_true": stats.rel_res_true,
        "rel_res_plain": stats.rel_res_plain,
        "vcycles": stats.vcycles,
        "roofline": roofline,
        "kernels": kernels,
    }
    solver.close()
    # setup again into the same workspace, as a time-stepping caller does each step
    # with new coefficients (the timing above also covers allocating the workspace)
    ts = time.time()
    ctx2 = S._binding.stokes_setup(rho, mu, prob.dt, solver.grid, solver.opts, solver.workspace.data_ptr(),
                                   solver.ws_bytes)
    torch.cuda.synchronize()
    out["setup_ms_reused_workspace"] = (time.time() - ts) * 1e3
    S._binding.stokes_destroy(ctx2)
    log("setup into the same workspace: %.1f ms" % out["setup_ms_reused_workspace"])
    del solver
    legs = Legs()
    out["hbm_stream_copy"] = legs.run("hbm_stream_copy", stream_copy, S)
    out["coefficient_step"] = legs.run("coefficient_step", coefficient_step, S, prob)
    out["rigid_projection"] = legs.run("rigid_projection", rigid_step, S, prob, xu)
    out["explicit_rhs"] = legs.run("explicit_rhs", explicit_rhs_step, S, prob, rho, mu, xu)
    out["density_transport"] = legs.run("density_transport", density_transport_step, S, prob, xu)
    if not args.no_forms and args.precision == 0:
        out["forms"] = {"fp32_multigrid": legs.run("fp32_multigrid", fp32_form, S, prob, rho, mu, rhs_u, rhs_p,
                                                   xu, xp, overrides, ms, args.steps)}
        lf = legs.run("learned", learned_form, S, prob, rho, mu, rhs_u, rhs_p, xu, xp, overrides, ms,
                      args.steps)
        if lf is not None:
            out["forms"]["learned"] = lf
    if not args.no_configs:
        out["configs"] = {"config3_128^3 dam break": legs.run("config3", config_leg, S, 3),
                          "config4_1024x96x96 wave tank": legs.run("config4", config_leg, S, 4)}
        out["velocity_multigrid"] = legs.run("velocity_multigrid", velocity_mg_leg, S)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = legs.run("cpu_baseline", cpu_baseline, prob, int(np.median(iters)), gpu=False)
    print(json.dumps(out), flush=True)


def _cycles_to_reach(curve, target):
    """Fractional number of cycles after which a residual curve (entries k = 0, 1, ...)
    first reaches `target`, interpolating log-linearly between whole cycles; None
    if it never does."""
    for k, v in enumerate(curve):
        if v <= target:
            if k == 0:
                return 0.0
            a, b = np.log(curve[k - 1]), np.log(v)
            return k - 1 + (a - np.log(target)) / (a - b) if a > b else float(k)
    return None


def learned_study(nseeds, n=256, ref_cycles=30, max_cycles=8, k_first=4):
    """What an initial guess of the pressure cycles is worth, on fresh seeds of the
    headline recipe (seeds 910000 + i: neither the training seeds 0-1999 nor the
    headline's 900000).  For the first preconditioner application (k_first plain
    cycles from zero in the solve) it finds how many cycles each start needs to
    reach the residual of k_first plain cycles: from the trained network's guess
    (32^3 level) and from the ideal guess a perfect predictor on level l (128^3,
    64^3, 32^3, 16^3) could give (the converged solution averaged to that level,
    same fit and prolongation).  Next to it: the measured cost of one pressure
    cycle at this size and of one U-Net forward pass from 32^3 to 256^3 (BF16 on the
    matrix cores), so that a predictor on level l pays only if its cycles saved x
    cycle cost exceed its forward cost."""
    import torch
    import workloads as W
    import paper_1901_07892_amd as S
    from paper_1901_07892_amd import learned
    dev = torch.device("cuda:0")
    params, meta = learned.load_params()
    td = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    rows = ["zero", "network_32^3"] + ["ideal_level%d_%d^3" % (l, n >> l) for l in range(1, S._binding.STUDY_ROWS - 1)]
    seeds = []
    cycle_ms = []
    for i in range(nseeds):
        seed = 910000 + i
        t0 = time.time()
        prob = W.config5(n_cells=n, seed=seed)
        log("study seed %d: workload in %.1fs" % (seed, time.time() - t0))
        rho = [td(r) for r in prob.rho_faces[:3]]
        mu = td(prob.mu)
        rhs_u = [td(f) for f in prob.rhs_u[:3]]
        rhs_p = td(prob.rhs_p)
        solver = S.StokesSolver(3, prob.n, prob.h, rho, mu, prob.dt)
        net = None
        if params is not None:
            net = S.UNet(meta["grid"])
            net.set_params(params)
            S.stokes_attach_learned(solver.ctx, net, 0.9)
        curves = S.stokes_learned_study(solver.ctx, rhs_u, rhs_p, ref_cycles, max_cycles)
        # cost of one pressure cycle: the same call with 21 and with 1 reference cycles
        tt = []
        for rc in (1, 21):
            torch.cuda.synchronize()
            t = time.perf_counter()
            S.stokes_learned_study(solver.ctx, rhs_u, rhs_p, rc, 0)
            torch.cuda.synchronize()
            tt.append(time.perf_counter() - t)
        cycle_ms.append((tt[1] - tt[0]) * 1e3 / 20)
        # plain and learned solves of the same instance
        xu = [torch.zeros_like(f) for f in rhs_u]
        xp = torch.zeros_like(rhs_p)
        solves = {}
        for name, attach in (("plain", False), ("learned", True)):
            if attach and net is None:
                continue
            S.stokes_attach_learned(solver.ctx, net if attach else None, 0.9)
            for a in xu:
                a.zero_()
            xp.zero_()
            st, stats = solver.solve(rhs_u, rhs_p, prob.tol, xu, xp)
            torch.cuda.synchronize()
            t = time.perf_counter()
            for a in xu:
                a.zero_()
            xp.zero_()
            st, stats = solver.solve(rhs_u, rhs_p, prob.tol, xu, xp)
            torch.cuda.synchronize()
            solves[name] = {"ms": (time.perf_counter() - t) * 1e3, "fgmres_iters": stats.iters, "status": st,
                            "vcycles": stats.vcycles, "fell_back": stats.fell_back,
                            "rel_res_true": stats.rel_res_true}
        target = curves[0][k_first]
        rec = {"seed": seed, "solids": len(prob.psi or []),
               "target_residual_after_%d_plain_cycles" % k_first: target, "curves": {}, "cycles_to_target": {},
               "cycles_saved": {}, "solves": solves}
        for r, name in enumerate(rows):
            c = curves[r]
            if np.all(np.isnan(c)):
                continue
            rec["curves"][name] = [float(v) for v in c]
            k = _cycles_to_reach(list(c), target)
            rec["cycles_to_target"][name] = k
            rec["cycles_saved"][name] = (k_first - k) if k is not None else None
        log("seed %d: cycles to the residual of %d plain cycles: %s" % (
            seed, k_first, {k: (round(v, 2) if v is not None else None) for k, v in rec["cycles_to_target"].items()}))
        seeds.append(rec)
        if net is not None:
            net.close()
        solver.close()
        del solver
        torch.cuda.empty_cache()
    # U-Net forward cost by grid size
    fwd = {}
    for g in (32, 64, 128, 256):
        net = S.UNet(g)
        f = [torch.randn((g, g, g), dtype=torch.float32, device=dev) for _ in range(3)]
        pred = torch.zeros_like(f[0])
        net.forward(f[0], f[1], f[2], pred)
        reps = 20 if g <= 64 else 3
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            net.forward(f[0], f[1], f[2], pred)
        e1.record()
        torch.cuda.synchronize()
        us = e0.elapsed_time(e1) / reps * 1e3
        fl = S.stokes_unet_forward_flops(g)
        fwd["%d^3" % g] = {"us": us, "flops": fl, "TFLOPs": fl / (us * 1e-6) / 1e12,
                           "frac_of_bf16_peak": fl / (us * 1e-6) / 2.5e15}
        log("U-Net forward %d^3: %.1f us, %.1f TFLOP/s" % (g, us, fl / (us * 1e-6) / 1e12))
        net.close()
        del net, f, pred
        torch.cuda.empty_cache()
    saved = {}
    for name in rows:
        v = [r["cycles_saved"].get(name) for r in seeds if r["cycles_saved"].get(name) is not None]
        if v:
            saved[name] = {"mean": float(np.mean(v)), "min": float(np.min(v)), "max": float(np.max(v))}
    return {"study": "learned-stage bound", "grid": n, "ref_cycles": ref_cycles, "first_application_cycles": k_first,
            "pressure_cycle_ms": float(np.mean(cycle_ms)), "cycles_saved": saved, "unet_forward": fwd,
            "model": {k: meta.get(k) for k in ("instances", "epochs", "fine_grid", "level_grid")} if meta else None,
            "final_val_loss": meta["history"][-1]["val_loss"] if meta and meta.get("history") else None,
            "seeds": seeds}


def fp32_form(S, prob, rho, mu, rhs_u, rhs_p, xu64, xp64, overrides, ms64, steps):
    """Multigrid in FP32 inside FP64 FGMRES on the same workload: ms per solve, its
    FP64 residual, speedup over the plain FP64 solve and the relative difference of
    each field from the FP64 solution (both converged to the same tolerance)."""
    import torch
    ref_u = [a.clone() for a in xu64]
    ref_p = xp64.clone()
    o = dict(overrides)
    o["precision"] = 1
    solver = S.StokesSolver(3, prob.n, prob.h, rho, mu, prob.dt, **o)
    xu = [torch.zeros_like(a) for a in ref_u]
    xp = torch.zeros_like(ref_p)
    times = []
    for s in range(steps + 2):
        if s == 2:
            S.stokes_profile_kernel(solver.ctx, 1)
        for a in xu:
            a.zero_()
        xp.zero_()
        torch.cuda.synchronize()
        t = time.perf_counter()
        st, stats = solver.solve(rhs_u, rhs_p, prob.tol, xu, xp)
        torch.cuda.synchronize()
        if s >= 2:
            times.append((time.perf_counter() - t) * 1e3)
        if st != 0:
            raise RuntimeError("fp32-multigrid solve did not converge: %s" % stats.as_dict())
    kms, kn, kb = S.stokes_profile_read(solver.ctx)
    S.stokes_profile_kernel(solver.ctx, -1)
    solver.close()
    achieved = kb / (kms * 1e-3) / 1e9 if kms > 0 else None
    roofline = {"bound": "hbm", "kernel": "k_p_sweep3c<float> (fused pressure red-black sweep, finest level)",
                "achieved": achieved, "peak": 8000.0, "unit": "GB/s",
                "frac": achieved / 8000.0 if achieved else None, "launches": kn,
                "avg_launch_us": kms * 1e3 / max(kn, 1), "algorithmic_bytes_per_launch": kb / max(kn, 1)}
    diff = [float(torch.linalg.vector_norm(xu[c] - ref_u[c]) / torch.linalg.vector_norm(ref_u[c])) for c in range(3)]
    diff.append(float(torch.linalg.vector_norm(xp - ref_p) / torch.linalg.vector_norm(ref_p)))
    ms = float(np.mean(times))
    log("fp32-multigrid form: %.2f ms, %d iterations, residual %.2e" % (ms, stats.iters, stats.rel_res_true))
    return {"ms_per_solve": ms, "fgmres_iters": stats.iters, "rel_res_true": stats.rel_res_true,
            "speedup_vs_fp64": ms64 / ms, "rel_diff_vs_fp64_solution": diff, "roofline": roofline}


def learned_form(S, prob, rho, mu, rhs_u, rhs_p, xu64, xp64, overrides, ms64, steps):
    """Learned form: the trained U-Net (BF16 on the matrix cores) seeds the pressure
    cycles from the 32^3 level; plain multigrid takes over on stagnation.  Same
    FP64 outer solve and residual check.  None if no trained weights are present."""
    import torch
    from paper_1901_07892_amd import learned
    p, meta = learned.load_params()
    if p is None:
        return None
    net = S.UNet(meta["grid"])
    net.set_params(p)
    solver = S.StokesSolver(3, prob.n, prob.h, rho, mu, prob.dt, **overrides)
    S.stokes_attach_learned(solver.ctx, net, 0.9)
    xu = [torch.zeros_like(a) for a in xu64]
    xp = torch.zeros_like(xp64)
    times = []
    for s in range(steps + 2):
        for a in xu:
            a.zero_()
        xp.zero_()
        torch.cuda.synchronize()
        t = time.perf_counter()
        st, stats = solver.solve(rhs_u, rhs_p, prob.tol, xu, xp)
        torch.cuda.synchronize()
        if s >= 2:
            times.append((time.perf_counter() - t) * 1e3)
        if st != 0:
            raise RuntimeError("learned-form solve did not converge: %s" % stats.as_dict())
    solver.close()
    # the network alone: forward passes on the features of the 32^3 level
    n = meta["grid"]
    f = [torch.randn((n, n, n), dtype=torch.float32, device="cuda") for _ in range(3)]
    pred = torch.zeros_like(f[0])
    for _ in range(3):
        net.forward(f[0], f[1], f[2], pred)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(20):
        net.forward(f[0], f[1], f[2], pred)
    e1.record()
    torch.cuda.synchronize()
    fwd_us = e0.elapsed_time(e1) / 20 * 1e3
    flops = S.stokes_unet_forward_flops(n)
    tflops = flops / (fwd_us * 1e-6) / 1e12
    net.close()
    diff = [float(torch.linalg.vector_norm(xu[c] - xu64[c]) / torch.linalg.vector_norm(xu64[c])) for c in range(3)]
    diff.append(float(torch.linalg.vector_norm(xp - xp64) / torch.linalg.vector_norm(xp64)))
    ms = float(np.mean(times))
    log("learned form: %.2f ms, %d iterations, fell back %d" % (ms, stats.iters, stats.fell_back))
    return {"ms_per_solve": ms, "fgmres_iters": stats.iters, "fell_back": stats.fell_back,
            "rel_res_true": stats.rel_res_true, "speedup_vs_fp64": ms64 / ms,
            "rel_diff_vs_fp64_solution": diff,
            "training": {k: meta.get(k) for k in ("instances", "epochs", "fine_grid", "level_grid")},
            "final_val_loss": meta["history"][-1]["val_loss"] if meta.get("history") else None,
            "unet_forward": {"grid": n, "us": fwd_us, "flops": flops,
                             "roofline": {"bound": "mfma", "achieved": tflops, "peak": 2500.0, "unit": "TFLOP/s",
                                          "frac": tflops / 2500.0}}}


def kernel_source_hash() -> str:
    import hashlib
    h = hashlib.sha256()
    for f in ("paper_1901_07892_amd/csrc/kernels.hpp", "paper_1901_07892_amd/csrc/box.hpp"):
        h.update(open(os.path.join(ROOT, f), "rb").read())
    return h.hexdigest()[:16]


def traffic_per_launch(kernel, n, precision):
    """HBM bytes per launch of the timed kernel from rocprofv3 FETCH_SIZE + WRITE_SIZE
    counter runs (profiles/traffic.json), or None when absent or taken on other
    kernel sources."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    try:
        rec = json.load(open(path))
    except ValueError:
        return None
    key = "%d/%d/%d" % (kernel, n, precision)
    e = rec.get("entries", {}).get(key)
    if not e or e.get("kernel_source_hash") != kernel_source_hash():
        return None
    return e.get("bytes_per_launch")


def stream_copy(S):
    """Practical HBM bandwidth of the library's own streaming copy kernel
    (stokes_stream_copy): 1 GiB read + 1 GiB written per launch, 10 launches
    timed with events on the stream they run on."""
    import torch
    a = torch.empty(1 << 27, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    a.fill_(1.0)
    for _ in range(2):
        S.stokes_stream_copy(a, b)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(10):
        S.stokes_stream_copy(a, b)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / 10
    gbps = 2.0 * a.numel() * 8 / (ms * 1e-3) / 1e9
    del a, b
    log("stream copy: %.1f GB/s (%.1f%% of 8 TB/s)" % (gbps, gbps / 80.0))
    return {"kernel": "k_stream_copy (library)", "bytes_per_launch": 2 * (1 << 30), "avg_launch_us": ms * 1e3,
            "GBps": gbps, "frac_of_8TBps": gbps / 8000.0}


def coefficient_step(S, prob, launches=20):
    """The step before the solve on the same instance: face densities and cell
    viscosity from its level sets (stokes_coefficients), timed with events on
    the stream it runs on.  Algorithmic bytes: every level set read once, every
    output written once."""
    import torch
    import workloads as W
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    n, dim = prob.n, prob.dim
    phi = dev(prob.phi)
    psi = [dev(p) for p in prob.psi]
    rho = [torch.empty(W.face_shape(n, ax), dtype=torch.float64, device="cuda") for ax in range(dim)]
    mu = torch.empty(W.cell_shape(n), dtype=torch.float64, device="cuda")
    grid = S._binding.make_grid(dim, n, prob.h)
    fl = S.make_fluids(W.RHO_WATER, prob.rho_air, W.MU_WATER, W.MU_AIR, prob.heaviside_cells)
    mus = [W.MU_SOLID] * len(psi)
    run = lambda: S.stokes_coefficients(grid, fl, phi, psi, prob.rho_solid, mus, rho, mu)
    for _ in range(3):
        run()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(launches):
        run()
    e1.record()
    torch.cuda.synchronize()
    us = e0.elapsed_time(e1) / launches * 1e3
    nbytes = 8.0 * ((1 + len(psi)) * mu.numel() + mu.numel() + sum(r.numel() for r in rho))
    err = max([float(np.abs(mu.cpu().numpy() - prob.mu).max() / prob.mu.max())] +
              [float(np.abs(r.cpu().numpy() - pr).max() / pr.max()) for r, pr in zip(rho, prob.rho_faces)])
    gbps = nbytes / (us * 1e-6) / 1e9
    log("coefficient step: %.1f us, %.0f GB/s (%d solids), max rel diff vs generator %.1e" % (us, gbps, len(psi), err))
    return {"kernel": "k_coefficients<%d>" % len(psi), "solids": len(psi), "avg_launch_us": us,
            "bytes_per_launch": nbytes, "GBps": gbps, "frac_of_8TBps": gbps / 8000.0,
            "max_rel_diff_vs_generator": err}


def explicit_rhs_step(S, prob, rho, mu, u, launches=20):
    """The right-hand side of the next step from the solved velocity
    (stokes_explicit_rhs: mass term, Crank-Nicolson explicit viscous half,
    well-balanced gravity from the flow-only density), timed with events on its
    stream.  Algorithmic bytes: u^n (3), rho (3), rho_flow (3), mu read, f (3)
    written, each once."""
    import torch
    grid = S._binding.make_grid(prob.dim, prob.n, prob.h)
    rf = [torch.from_numpy(np.ascontiguousarray(a)).cuda() for a in prob.rho_flow_faces[:prob.dim]]
    f = [torch.empty_like(a) for a in u]
    gv = (0.0, 0.0, -9.81)
    run = lambda: S.stokes_explicit_rhs(grid, rho, mu, prob.dt, 0.5, u, f, rf, gv)
    for _ in range(3):
        run()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(launches):
        run()
    e1.record()
    torch.cuda.synchronize()
    us = e0.elapsed_time(e1) / launches * 1e3
    nbytes = 8.0 * (4 * sum(a.numel() for a in u) + mu.numel())     # u^n, rho, rho_flow, f; mu
    gbps = nbytes / (us * 1e-6) / 1e9
    log("explicit rhs: %.1f us, %.0f GB/s" % (us, gbps))
    return {"kernel": "k_explicit_rhs3_z", "theta": 0.5, "avg_launch_us": us, "bytes_per_launch": nbytes,
            "GBps": gbps, "frac_of_8TBps": gbps / 8000.0}


def density_transport_step(S, prob, u, reps=10):
    """SSP-RK3 face-density transport (three launches) on the instance's face densities,
    with the solved velocity as every stage's advecting velocity; algorithmic bytes =
    every face array each stage must read or write once (stage 1: rho_n, u, out;
    stages 2 and 3: rho_n, the stage density, u, out)."""
    import torch
    dev = torch.device("cuda:0")
    rho = [torch.from_numpy(np.ascontiguousarray(prob.rho_faces[c])).to(dev) for c in range(3)]
    out = [torch.empty_like(a) for a in rho]
    grid = S._binding.make_grid(3, prob.n, prob.h)
    ws = torch.empty(S.stokes_density_workspace_size(grid), dtype=torch.uint8, device=dev)
    umax = max(float(a.abs().max()) for a in u)
    dt = 0.3 * min(prob.h) / max(umax, 1e-30)
    stages = [u, u, u]
    for _ in range(2):
        S.stokes_density_rk3(grid, dt, rho, stages, out, ws)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        S.stokes_density_rk3(grid, dt, rho, stages, out, ws)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    faces = sum(float(a.numel()) for a in rho)
    nbytes = 8.0 * faces * (3 + 4 + 4)
    moved = max(float((out[c] - rho[c]).abs().max()) for c in range(3))
    log("density transport (SSP-RK3, 3 launches): %.3f ms, %.0f GB/s algorithmic" % (ms, nbytes / (ms * 1e-3) / 1e9))
    return {"kernel": "k_rk3_stage x 3", "ms_per_update": ms, "bytes_per_update": nbytes,
            "GBps": nbytes / (ms * 1e-3) / 1e9, "frac_of_8TBps": nbytes / (ms * 1e-3) / 8e12,
            "cfl": 0.3, "max_density_change": moved}


def rigid_step(S, prob, u, reps=10):
    """The step after the solve on the same instance: the free-body rigid
    projection of each solid (markers at the solid's cell centres) applied to
    the solved velocity, timed on the host around the call (it synchronises
    once to read the momentum sums)."""
    import time
    import torch
    import workloads as W
    Xc, Yc, Zc = W.cell_coords(prob.n, prob.h)
    grid = S._binding.make_grid(prob.dim, prob.n, prob.h)
    dV = float(np.prod(prob.h))
    bodies = []
    for q, psi in enumerate(prob.psi):
        m = psi < 0
        X = torch.from_numpy(np.ascontiguousarray(np.stack([Xc[m], Yc[m], Zc[m]], 1))).cuda()
        ws = torch.empty(S.stokes_rigid_workspace_size(3, X.shape[0]), dtype=torch.uint8, device="cuda")
        xc = X.mean(0).tolist()
        uu = [a.clone() for a in u]
        S.stokes_rigid_projection(grid, uu, X, dV, 1, S.make_body(xc), ws)
        torch.cuda.synchronize()
        ts = []
        for _ in range(reps):
            uu = [a.clone() for a in u]
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            b = S.stokes_rigid_projection(grid, uu, X, dV, 1, S.make_body(xc), ws)
            torch.cuda.synchronize()
            ts.append((time.perf_counter() - t0) * 1e3)
        bodies.append({"markers": int(X.shape[0]), "ms": float(np.median(ts)), "u_r": list(b.u_r),
                       "w_r": list(b.w_r)})
        log("rigid projection of solid %d: %d markers, %.3f ms" % (q, X.shape[0], bodies[-1]["ms"]))
    return {"bodies": bodies, "note": "free body, markers at the solid's cell centres, on the solved velocity"}


def _cpu_model():
    """Model name of the host CPU with its family / model / stepping numbers (some
    virtualised hosts report only a short model name)."""
    info = {}
    try:
        for line in open("/proc/cpuinfo"):
            if ":" not in line:
                continue
            k, v = (x.strip() for x in line.split(":", 1))
            if k in ("model name", "vendor_id", "cpu family", "model", "stepping", "cpu MHz") and k not in info:
                info[k] = v
    except OSError:
        return None
    if not info:
        return None
    return "%s (vendor %s, family %s, model %s, stepping %s, %s MHz)" % (
        info.get("model name"), info.get("vendor_id"), info.get("cpu family"), info.get("model"),
        info.get("stepping"), info.get("cpu MHz"))


def _counter_rows(d, counter):
    import csv
    rows = []
    for r in csv.DictReader(open(os.path.join(d, "run_counter_collection.csv"))):
        if r["Counter_Name"] == counter:
            rows.append((r["Kernel_Name"], int(r["Grid_Size"]), float(r["Counter_Value"])))
    return rows


def traffic_from_counters(fetch_dir, write_dir, n=256, precision=0, path=None):
    """HBM bytes per launch of the finest fused pressure sweep from two rocprofv3 runs
    (--pmc FETCH_SIZE, then --pmc WRITE_SIZE) of 'bench.py --calibrate-copy': each
    counter (KiB per dispatch) is scaled by what it reads for the plain 1 GiB device
    copy that run starts with.  Writes profiles/traffic.json; prints the summary."""
    import re
    fetch, write = _counter_rows(fetch_dir, "FETCH_SIZE"), _counter_rows(write_dir, "WRITE_SIZE")
    gib_kib = float(1 << 20)

    def calib(rows):
        # the calibration copies are the copy dispatches before the first solver kernel
        v = []
        for name, g, c in rows:
            if "stk::" in name:
                break
            if "copyBuffer" in name and c > 0.25 * gib_kib:
                v.append(c)
        if not v:
            raise SystemExit("no 1 GiB calibration copy in the counter run")
        return gib_kib / (sum(v) / len(v))

    ff, wf = calib(fetch), calib(write)
    R = 8 if precision == 0 else 4
    cells = float(n) ** 3
    kernels = [  # (label, name pattern, algorithmic bytes per launch on the finest level)
        ("k_p_sweep3c (finest fused pressure sweep)", r"k_p_sweep3\w*<%s, 64, 16(, \w+)?>" % ("double" if R == 8 else "float"),
         cells * R * 6.0),
        ("k_apply3_z (Stokes matvec)", r"k_apply3_z<", None),
        ("k_p_residual_restrict3_z (finest)", r"k_p_residual_restrict3_z<%s" % ("double" if R == 8 else "float"),
         cells * R * 5.0 + cells / 8 * R),
        ("k_precond_update_jac", r"k_precond_update_jac<", cells * 8 * 16.0),
        ("k_precond_div_jac", r"k_precond_div_jac<", cells * 8 * 9.0),
        ("k_scale", r"k_scale\b", None),
        # the steps around the solve (the headline instance has two solids)
        ("k_coefficients<2> (coefficient step)", r"k_coefficients<2>",
         8.0 * (4 * cells + 3 * (n + 1) * float(n) ** 2)),
        ("k_explicit_rhs (explicit right-hand side)", r"k_explicit_rhs", 8.0 * (12 * (n + 1) * float(n) ** 2 + cells)),
        ("k_rigid_interp (rigid projection gather)", r"k_rigid_interp<3>", None),
        ("k_rigid_spread (rigid projection scatter)", r"k_rigid_spread<3>", None),
    ]
    out = {}
    lines = []
    for label, pat, alg in kernels:
        def pick(rows):
            m = [(g, c) for name, g, c in rows if re.search(pat, name)]
            if not m:
                return None, 0
            gmax = max(g for g, _ in m)
            v = [c for g, c in m if g == gmax]
            return sum(v) / len(v), len(v)
        fk, nf = pick(fetch)
        wk, nw = pick(write)
        if fk is None or wk is None:
            continue
        fb, wb = fk * 1024 * ff, wk * 1024 * wf
        out[label] = (fk, wk, nf, fb, wb, alg)
        ratio = ("  -> %.2fx algorithmic %.3f GB" % ((fb + wb) / alg, alg / 1e9)) if alg else ""
        lines.append("  %-44s FETCH %10.1f KiB x %.3f = %.3f GB  WRITE %10.1f KiB x %.3f = %.3f GB  (%d dispatches)%s"
                     % (label, fk, ff, fb / 1e9, wk, wf, wb / 1e9, nf, ratio))
    label = kernels[0][0]
    if label not in out:
        raise SystemExit("finest sweep not found in the counter runs")
    fk, wk, nd, fb, wb, alg = out[label]
    entry = {"kernel": "k_p_sweep3c<%s,64,16> finest level" % ("double" if R == 8 else "float"),
             "fetch_kib_per_dispatch": fk, "write_kib_per_dispatch": wk, "dispatches": nd,
             "fetch_factor": ff, "write_factor": wf, "bytes_per_launch": fb + wb,
             "algorithmic_bytes_per_launch": alg, "kernel_source_hash": kernel_source_hash()}
    path = path or os.path.join(ROOT, "profiles", "traffic.json")
    rec = json.load(open(path)) if os.path.exists(path) else {}
    rec["description"] = ("HBM traffic per launch of the timed kernel from rocprofv3 --pmc FETCH_SIZE and "
                          "WRITE_SIZE runs, each scaled by the same counter on a plain 1 GiB device copy "
                          "(bench.py --calibrate-copy); written by bench.py --traffic-from.")
    rec["commands"] = [
        "rocprofv3 --pmc FETCH_SIZE --output-format csv -d %s -o run -- python3 -u bench.py --steps 1 "
        "--warmup 0 --no-cpu-baseline --no-forms --no-configs --calibrate-copy" % fetch_dir,
        "rocprofv3 --pmc WRITE_SIZE --output-format csv -d %s -o run -- python3 -u bench.py --steps 1 "
        "--warmup 0 --no-cpu-baseline --no-forms --no-configs --calibrate-copy" % write_dir,
        "python3 bench.py --traffic-from %s %s" % (fetch_dir, write_dir)]
    rec.setdefault("entries", {})["1/%d/%d" % (n, precision)] = entry
    with open(path, "w") as f:
        json.dump(rec, f, indent=1)
    print("calibration (1 GiB copy): FETCH_SIZE factor %.3f, WRITE_SIZE factor %.3f" % (ff, wf))
    print("\n".join(lines))
    print("wrote", path)
    return entry


def cpu_baseline(prob, gpu_iters):
    """The C oracle (OpenMP) on this host: ONE full solve of the same 256^3 workload
    to the same tolerance, timed by the wall clock around the call (setup of its
    hierarchy included).  Restart 20 keeps its Krylov basis within host memory;
    three pressure V-cycles per preconditioner step.  The one-core figure is an
    estimate: the value times the one-/all-thread time ratio of a full 64^3 solve."""
    import workloads as W
    from oracle import native
    nth = native.num_threads()
    log("cpu baseline: full oracle solve of %s on %d threads ..." % (prob.name, nth))
    t0 = time.time()
    _, _, info = native.solve_problem(prob, tol=prob.tol, restart=20, p_cycles=3, max_iters=200)
    wall = time.time() - t0
    log("cpu baseline: %d oracle iterations, rel residual %.2e, setup %.1fs, FGMRES %.1fs, wall %.1fs"
        % (info["iters"], info["rel_res_true"], info["setup_s"], info["solve_s"], wall))
    tiny = W.config5(n_cells=64)
    tiny.dt = prob.dt
    t1 = time.time()
    native.solve_problem(tiny, tol=prob.tol, p_cycles=3)
    t_all = time.time() - t1
    native.set_threads(1)
    t1 = time.time()
    native.solve_problem(tiny, tol=prob.tol, p_cycles=3)
    t_one = time.time() - t1
    native.set_threads(nth)
    return {"value": wall * 1e3, "unit": "ms/solve", "cores": nth, "kind": "oracle",
            "sample": "one full solve of the same %s workload by the C oracle (FP64, OpenMP for matvec/BLAS, "
                      "lexicographic Gauss-Seidel multigrid, three pressure V-cycles per preconditioner step, "
                      "restart 20) to tol %.0e, wall clock around the call (hierarchy setup %.1f s, FGMRES %.1f s; "
                      "the GPU solve takes %d iterations)" % (prob.name, prob.tol, info["setup_s"], info["solve_s"],
                                                            gpu_iters),
            "oracle_iters": int(info["iters"]), "oracle_status": int(info["status"]),
            "oracle_rel_res_true": info["rel_res_true"],
            "cpu_model": _cpu_model(), "nproc": os.cpu_count(),
            "one_core_estimate": {"value": wall * 1e3 * t_one / t_all, "unit": "ms/solve",
                                  "sample": "estimate, not timed: the value above times the one-thread / "
                                            "%d-thread time ratio of a full 64^3 oracle solve of the same recipe "
                                            "(%.2f s / %.2f s)" % (nth, t_one, t_all)}}


def velocity_mg_leg(S, n=128, dt=1.0, steps=5):
    """A viscous-dominated solve, where the automatic rule runs the velocity
    multigrid (at the workload configs the velocity operator is mass-dominated and
    one diagonal step replaces it): the headline recipe at n^3 with dt = 1 (viscous
    / mass diagonal ratio above 1e-2 in the air), tol 1e-8, FP64 and FP32
    multigrid; ms per solve, iterations and cycles, against the same solve with
    the diagonal velocity step forced (vel_levels = 1)."""
    import torch
    import workloads as W
    prob = W.config5(n_cells=n, dt=dt)
    dev = torch.device("cuda:0")
    td = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    rho = [td(r) for r in prob.rho_faces[:3]]
    mu = td(prob.mu)
    rhs_u = [td(f) for f in prob.rhs_u[:3]]
    rhs_p = td(prob.rhs_p)
    leg = {"grid": list(prob.n), "dt": dt, "tol": prob.tol}
    for name, over in (("fp64", {}), ("fp32_multigrid", {"precision": 1}),
                       ("fp64_diagonal_velocity_step", {"vel_levels": 1, "max_iters": 60})):
        solver = S.StokesSolver(3, prob.n, prob.h, rho, mu, dt, **over)
        xu = [torch.zeros_like(f) for f in rhs_u]
        xp = torch.zeros_like(rhs_p)
        times = []
        for it in range(steps + 1):
            for a in xu:
                a.zero_()
            xp.zero_()
            torch.cuda.synchronize()
            t = time.perf_counter()
            st, stats = solver.solve(rhs_u, rhs_p, prob.tol, xu, xp)
            torch.cuda.synchronize()
            if it > 0:
                times.append((time.perf_counter() - t) * 1e3)
        leg[name] = {"ms_per_solve": float(np.median(times)), "status": st, "fgmres_iters": stats.iters,
                     "cycles": stats.vcycles, "rel_res_true": stats.rel_res_true}
        log("velocity multigrid leg %s: %.2f ms, status %d, %d iterations, %d cycles, res %.2e"
            % (name, leg[name]["ms_per_solve"], st, stats.iters, stats.vcycles, stats.rel_res_true))
        solver.close()
        del solver
    return leg


def config_leg(S, num, steps=5, warmup=2):
    """Configs 3 and 4 at their stated sizes (FP64 and FP32 multigrid, each to its tol):
    ms per solve, iterations, the finest fused sweep's roofline (HIP events on the
    solve's stream), and the solutions checked by the oracle -- error against its
    FP64 solution at tol 1e-13 for config 3, its own operator's residual for config 4
    (its FGMRES at tol 1e-13 takes minutes of host time at 1024x96x96)."""
    import torch
    import workloads as W
    from oracle import native
    prob = W.config3() if num == 3 else W.config4()
    dev = torch.device("cuda:0")
    td = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    rho = [td(r) for r in prob.rho_faces[:3]]
    mu = td(prob.mu)
    rhs_u = [td(f) for f in prob.rhs_u[:3]]
    rhs_p = td(prob.rhs_p)
    leg = {"grid": list(prob.n), "tol": prob.tol, "dt": prob.dt}
    sols = {}
    for precision in (0, 1):
        solver = S.StokesSolver(3, prob.n, prob.h, rho, mu, prob.dt, precision=precision)
        xu = [torch.zeros_like(f) for f in rhs_u]
        xp = torch.zeros_like(rhs_p)

        def step():
            for a in xu:
                a.zero_()
            xp.zero_()
            st, stats = solver.solve(rhs_u, rhs_p, prob.tol, xu, xp)
            if st != 0:
                raise RuntimeError("config %d solve did not converge: %s" % (num, stats.as_dict()))
            return stats

        for _ in range(warmup):
            step()
        torch.cuda.synchronize()
        S.stokes_profile_kernel(solver.ctx, 1)
        t0 = time.perf_counter()
        for _ in range(steps):
            stats = step()
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / steps
        kms, kn, kb = S.stokes_profile_read(solver.ctx)
        S.stokes_profile_kernel(solver.ctx, -1)
        achieved = kb / (kms * 1e-3) / 1e9 if kms > 0 else None
        name = "fp64" if precision == 0 else "fp32_multigrid"
        leg[name] = {"ms_per_solve": ms, "fgmres_iters": stats.iters, "rel_res_true": stats.rel_res_true,
                     "rel_res_plain": stats.rel_res_plain,
                     "sweep_roofline": {"bound": "hbm", "kernel": "k_p_sweep3c finest level", "achieved": achieved,
                                        "peak": 8000.0, "unit": "GB/s",
                                        "frac": achieved / 8000.0 if achieved else None, "launches": kn,
                                        "avg_launch_us": kms * 1e3 / max(kn, 1)}}
        sols[name] = ([a.cpu().numpy() for a in xu], xp.cpu().numpy())
        log("config %d %s: %.2f ms, %d iterations, sweep %.1f us (%.0f GB/s)"
            % (num, name, ms, stats.iters, kms * 1e3 / max(kn, 1), achieved or 0))
        solver.close()
        del solver
    if num == 3:
        t0 = time.time()
        ou, op, info = native.solve_problem(prob, tol=1e-13, max_iters=400, restart=20)
        leg["oracle"] = {"tol": 1e-13, "iters": int(info["iters"]), "rel_res_true": info["rel_res_true"],
                         "wall_s": time.time() - t0}
        for name, (xu, xp) in sols.items():
            errs = [float(np.linalg.norm(xu[c] - ou[c]) / np.linalg.norm(ou[c])) for c in range(3)]
            pm, om = xp - xp.mean(), op - op.mean()
            errs.append(float(np.linalg.norm(pm - om) / np.linalg.norm(om)))
            leg[name]["rel_error_vs_oracle"] = errs
    else:
        sigma = native.auto_sigma(prob)
        b2 = sum(float(np.sum(prob.rhs_u[c] ** 2)) for c in range(3))
        for name, (xu, xp) in sols.items():
            yu, yp = native.apply_problem(prob, xu, xp)
            r2 = sum(float(np.sum((prob.rhs_u[c] - yu[c]) ** 2)) for c in range(3))
            rp2 = float(np.sum(yp ** 2))
            leg[name]["oracle_residual"] = {"plain": float(np.sqrt((r2 + rp2) / b2)),
                                            "weighted": float(np.sqrt((r2 + sigma ** 2 * rp2) / b2)),
                                            "sigma": sigma}
    return leg


if __name__ == "__main__":
    main()
