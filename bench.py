#!/usr/bin/env python3
"""Benchmark: ms per Stokes solve to 1e-8 relative residual, 256^3, density ratio 1000.

One step = one full stokes_solve (FGMRES + projection preconditioner + multigrid)
of the seeded 256^3 air/water/solid workload (eval seed 900000) with inputs
resident in HBM; setup (coefficients, hierarchy) is timed separately.  Prints
one JSON line.
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
    ap.add_argument("--verbose", action="store_true")
    return ap.parse_args()


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the solve is a single-GPU kernel path "
              "(no multi-GPU sharding is built); use --gpus 1", file=sys.stderr)
        sys.exit(2)
    import torch
    import workloads as W
    import paper_1901_07892_amd as S

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
    }
    solver.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
