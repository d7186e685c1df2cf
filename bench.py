"""Benchmark: Poisson unknowns/s to relative residual 1e-10 on the
paper-scale spherical shell (192 r x 256 theta x 512 phi cells, tanh radial
clustering with stretching factor 2.0, cone walls at 0.05 and pi - 0.05,
right-hand side = seeded N(0,1) field smoothed by 3 Jacobi passes, mean
removed), one MI355X.

A step is one complete cps_solve (FP64 hierarchy, Krylov-accelerated
V(2,2) multigrid) from the right-hand side resident in HBM to 1e-10.  The
FP32-multigrid + FP64-refinement form is timed on the same input and
reported beside it.  Prints one JSON line.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Poisson unknowns/s to 1e-10 residual, FP64 vs FP32-MG+IR; serve p50/p99 ms"
HBM_PEAK_GBS = 8000.0
TOL = 1e-10


def gs_bytes_per_launch(shape, ncol, word, phi_invariant, mode_terms):
    """Algorithmic HBM bytes of one finest-level Gauss-Seidel colour pass:
    each updated cell reads its right-hand side and writes itself once, every
    other cell is read once as a neighbour, and the metric arrays are read
    once (per (r, theta) when phi-invariant)."""
    nr, nt, np_ = shape
    n = nr * nt * np_
    upd = n // ncol
    field = upd * 2 * word + (n - upd) * word
    coef = mode_terms * (nr * nt if phi_invariant else n) * word
    return field + coef


def run_form(cps, torch, g, rhs, precision, steps, warmup):
    s = cps.Solver(g, precision=precision, accel=1, max_iters=400)
    p = torch.empty_like(rhs)
    for _ in range(warmup):
        res = s.solve(rhs, TOL, out=p)
    torch.cuda.synchronize()
    cps.cps_profile_enable(s.h, True)
    t0 = time.perf_counter()
    iters = []
    for _ in range(steps):
        res = s.solve(rhs, TOL, out=p)
        iters.append(res.iterations)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    prof = {k: cps.cps_profile_read(s.h, k) for k in range(5)}
    cps.cps_profile_enable(s.h, False)
    out = dict(solver=s, p=p, res=res, sec=dt, iters=iters, prof=prof)
    return out


def cpu_baseline(g, rhs_np, gpu_iters, accel=1):
    """The oracle's multigrid (same levels, smoother, transfers, coarse
    solve and Krylov method) on the full grid, timed for two outer
    iterations on the host cores and scaled to the iteration count the same
    algorithm needs to reach 1e-10."""
    import oracle as O
    og = O.Grid(g.n_r, g.n_theta, g.n_phi, map=g.map, r_inner=g.r_inner, r_outer=g.r_outer,
                theta0=g.theta0, theta1=g.theta1, radial_stretch=g.radial_stretch)
    mg = O.Multigrid(og)
    k = 2
    t0 = time.perf_counter()
    mg.solve(rhs_np, tol=1e-300, max_iters=k, accel=accel)
    per_iter = (time.perf_counter() - t0) / k
    n = g.n_r * g.n_theta * g.n_phi
    threads = O.max_threads()
    return {"value": n / (per_iter * gpu_iters), "unit": "unknowns/s", "cores": threads,
            "kind": "oracle",
            "sample": f"{k} PCG iterations of the oracle's V(2,2) multigrid on the full "
                      f"{g.n_r}x{g.n_theta}x{g.n_phi} grid ({per_iter:.2f} s each, "
                      f"{threads} OpenMP threads), scaled to the {gpu_iters} iterations "
                      f"the same algorithm needs to reach 1e-10"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-mixed", action="store_true")
    a = ap.parse_args()
    if a.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {a.gpus}): the solve of one "
              "grid is not sharded across devices in this build", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2305_17875_amd import cps, inputs

    torch.cuda.set_device(0)
    g = inputs.config2()
    n = g.cells
    print(f"[bench] generating rhs {g.shape}", file=sys.stderr, flush=True)
    rhs_np = inputs.smoothed_noise(g.shape, seed=0)
    rhs = torch.from_numpy(rhs_np).cuda().flatten()

    print("[bench] fp64 solves", file=sys.stderr, flush=True)
    f64 = run_form(cps, torch, g, rhs, 0, a.steps, a.warmup)
    s64 = f64["solver"]
    word = 8
    gs_ms, gs_n = f64["prof"][cps.KERNEL_GS]
    avg_gs_ms = gs_ms / max(gs_n, 1)
    terms = {2: 3, 4: 5}[s64.ncolours] if s64.phi_invariant else 9
    gs_bytes = gs_bytes_per_launch(g.shape, s64.ncolours, word, s64.phi_invariant, terms)
    achieved = gs_bytes / (avg_gs_ms * 1e-3) / 1e9
    kern = {}
    for k, name in enumerate(["gs_pass", "residual", "apply", "restrict", "prolong"]):
        ms, cnt = f64["prof"][k]
        kern[name] = {"launches_per_step": cnt / a.steps,
                      "avg_us": (ms / cnt * 1e3) if cnt else None}

    line = {
        "metric": METRIC,
        "value": n / f64["sec"],
        "unit": "unknowns/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": f64["sec"] * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "sphere shell 192(r)x256(theta)x512(phi), tanh radial "
                               "clustering 2.0, smoothed N(0,1) rhs seed 0, tol 1e-10",
                   "cells": n, "levels": len(s64.levels), "accel": "pcg",
                   "colours": s64.ncolours},
        "iterations": f64["iters"][-1],
        "rel_residual": f64["res"].rel_residual,
        "roofline": {"bound": "hbm", "kernel": "k_gs (finest level, one colour pass)",
                     "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                     "avg_us": avg_gs_ms * 1e3, "algorithmic_bytes": gs_bytes},
        "kernels_fp64": kern,
    }
    if not a.no_mixed:
        print("[bench] mixed solves", file=sys.stderr, flush=True)
        mx = run_form(cps, torch, g, rhs, 1, a.steps, a.warmup)
        x64 = f64["p"].double()
        err = float(torch.linalg.norm(mx["p"] - x64) / torch.linalg.norm(x64))
        line["mixed"] = {"value": n / mx["sec"], "ms_per_step": mx["sec"] * 1e3,
                         "iterations": mx["iters"][-1],
                         "rel_residual": mx["res"].rel_residual,
                         "rel_diff_vs_fp64": err, "dtype": "f32 V-cycles, f64 outer"}
        mx["solver"].close()
    if not a.no_cpu_baseline:
        print("[bench] cpu baseline (oracle)", file=sys.stderr, flush=True)
        line["cpu_baseline"] = cpu_baseline(g, rhs_np, f64["iters"][-1])
    s64.close()
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
