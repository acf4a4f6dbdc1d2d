"""Throughput of the cRKDG step on one MI355X.

One "step" is one pass of the whole hot path over the 2D Euler shock
workload (4096 x 1024 cells, Q^2, scheme (eq:3), Lax--Friedrichs flux, Mach-3
shock into a smoothed density field; see paper_2307_06471_amd/workloads.py):
  dt from the cell averages (device reduction, no host sync)
  -> inner stages (local operator)
  -> final stage (DG operator, face fluxes, conservative update)
  -> TVB minmod limiter (M = 50).
The timed region holds K such steps with the state resident in HBM; the
result is DOF-updates/s (cells x modes x components per step).

Prints one JSON line.  `roofline` covers the kernel with the largest share
of the step time, from HIP events recorded around every launch on the
library's stream during the timed region; `cpu_baseline` times the serial
oracle on a bounded patch of the same workload.
"""
import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "2D Euler cRKDG DOF-updates/s: FP32+learned limiter vs FP64 plain, equal L2 err"
HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFLOPS = 78.6


def algorithmic_bytes(cls, state_bytes, ncells, stages_final):
    """bytes a kernel class must move per launch (its inputs and outputs):
    inner: read u^n, write the stored stage state(s); final: read u^n and the
    final-stage states, write u^{n+1}; limiter: read the state, write one
    flag byte per cell; dt: read the cell averages."""
    if cls == "inner":
        return state_bytes * (1 + (stages_final - 1))
    if cls == "final":
        return state_bytes * (stages_final + 1)
    if cls == "limit":
        return state_bytes + ncells
    if cls == "dt":
        return state_bytes // 9
    return None


def make_solver(K, W, scale=1, precision=0):
    import torch
    cfg = W.config("c5", scale=scale)
    params, xi = W.shock_problem(2000, cfg["nx"], cfg["ny"])
    ghost = W.post_shock_conserved(params[0])
    x0, x1, y0, y1 = cfg["box"]
    mesh = K.make_mesh(2, cfg["nx"], cfg["ny"], x0=x0, x1=x1, y0=y0, y1=y1, bc=(2, 1, 1, 1),
                       bc_state=[ghost] * 4, equation=K.EQ_EULER, gamma=W.GAMMA,
                       precision=precision)
    s = K.Solver(mesh, cfg["k"], K.FLUX_LLF, 3)
    s.crkdg_project(K.IC_SHOCK, params, aux=torch.from_numpy(xi).cuda())
    s.crkdg_limit(cfg["limiter"][1])  # the projected shock overshoots: limit once
    return s, cfg, params, xi


def cpu_baseline(W, seconds=12.0):
    """serial oracle on a 128 x 32 patch of the same workload (same cell size,
    same physics, same boundary types): one warm-up step, then as many steps
    (dt + step + limiter) as fit in `seconds`"""
    import oracle as O
    nx, ny = 128, 32
    cfg = W.config("c5")
    dx = (cfg["box"][1] - cfg["box"][0]) / cfg["nx"]
    params, xi = W.shock_problem(2000, nx, ny)
    params = list(params)
    params[4], params[5] = 0.5 * nx * dx, 0.5 * ny * dx  # shock through the patch centre
    ghost = W.post_shock_conserved(params[0])
    om = O.Mesh(2, nx, ny, x0=0.0, x1=nx * dx, y0=0.0, y1=ny * dx, bc=(2, 1, 1, 1),
                bc_state=[ghost] * 4, equation=O.EQ_EULER, gamma=W.GAMMA, flux=O.FLUX_LLF)
    k = cfg["k"]
    A, b, c = (np.array(v, float) for v in W.TABLEAU["eq3"])
    u = O.project(om, k, O.IC_SHOCK, params, xi)
    u, _, _ = O.limit_tvb(om, k, 50.0, u)

    def one(u):
        dt = cfg["cfl"] / O.max_wavespeed(om, k, u)
        u = O.step_crkdg(om, k, (A, b, c), 0.0, dt, u)
        u, _, _ = O.limit_tvb(om, k, 50.0, u)
        return u

    u = one(u)
    t0 = time.perf_counter()
    n = 0
    while time.perf_counter() - t0 < seconds or n < 2:
        u = one(u)
        n += 1
    el = time.perf_counter() - t0
    dofs = nx * ny * (k + 1) ** 2 * 4
    return {"value": dofs * n / el, "unit": "DOF-updates/s", "cores": 1, "kind": "oracle",
            "sample": f"{nx}x{ny}-cell patch of the same workload (Q2, eq3, LLF, TVB M=50, "
                      f"same cell size and boundary types), {n} steps after 1 warm-up, "
                      f"serial FP64 C oracle, {el:.1f} s"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--scale", type=int, default=1, help="divide the cell counts (debug only)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU; this build has no multi-GPU path (--gpus {args.gpus})",
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2307_06471_amd import crkdg as K
    from paper_2307_06471_amd import workloads as W

    forms = {}
    for name, prec in (("fp32-bulk + TVB", K.FP32_MIXED), ("fp64 + TVB", K.FP64)):
        forms[name] = run_form(K, W, args, prec)
        print(f"# {name}: {forms[name]['ms_per_step']:.3f} ms/step", file=sys.stderr, flush=True)
    head = forms["fp32-bulk + TVB"]
    plain = forms["fp64 + TVB"]
    out = {
        "metric": METRIC, "value": head["value"], "unit": "DOF-updates/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": head["ms_per_step"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"2D Euler Mach-3 shock into a smoothed density field, "
                               f"{head['nx']}x{head['ny']} Q2 cells on [0,4]x[0,1], cRKDG scheme "
                               f"eq3, Lax-Friedrichs flux, TVB minmod M=50 (FP64 test), "
                               f"per-step dt (CFL 0.1)",
                   "form": "fp32-bulk (FP32 contractions and fluxes, FP64 cell averages and "
                           "face-flux sums) + TVB limiter",
                   "cells": head["cells"], "dofs": head["dofs"], "parallelism": "1 GPU"},
        "roofline": head["roofline"],
        "kernels": head["kernels"],
        "fp64_plain": {"value": plain["value"], "ms_per_step": plain["ms_per_step"],
                       "roofline": plain["roofline"], "kernels": plain["kernels"]},
        "speedup_vs_fp64_plain": head["value"] / plain["value"],
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(W)
    print(json.dumps(out), flush=True)


def run_form(K, W, args, precision):
    import torch
    s, cfg, params, xi = make_solver(K, W, args.scale, precision)
    stream = s.stream
    dt_dev = torch.zeros(1, dtype=torch.float64, device="cuda")
    flags = torch.zeros(s.ncells, dtype=torch.uint8, device="cuda")
    M = cfg["limiter"][1]

    def step():
        s.crkdg_compute_dt(cfg["cfl"], dt_dev)
        s.crkdg_step_dev(dt_dev)
        s.crkdg_limit(M, flags, count=False)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    s.crkdg_profile_begin(8 * args.steps + 8)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    with torch.cuda.stream(stream):
        e0.record(stream)
        for _ in range(args.steps):
            step()
        e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    prof = s.crkdg_profile_end()
    n_flag = s.crkdg_limit(M, None, count=True)  # raises if a cell average went non-physical

    dofs = s.ncells * s.nmodes * s.ncomp
    stages_final = 2  # scheme (eq:3): b = (1/4, 0, 3/4)
    kern = {}
    for cls, (tms, cnt) in prof.items():
        by = algorithmic_bytes(cls, s.state_bytes, s.ncells, stages_final)
        kern[cls] = {"ms_per_launch": tms / cnt, "launches": cnt, "share": tms / ms,
                     "achieved_GBs": None if by is None else by / (tms / cnt * 1e-3) / 1e9}
    dom = max(prof, key=lambda c: prof[c][0])
    by = algorithmic_bytes(dom, s.state_bytes, s.ncells, stages_final)
    achieved = by / (prof[dom][0] / prof[dom][1] * 1e-3) / 1e9
    roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None, "kernel": dom,
            "bytes_per_launch": by}
    return {"value": dofs * args.steps / (ms / 1e3), "ms_per_step": ms / args.steps,
            "roofline": roof, "kernels": kern, "flagged_cells_end": n_flag,
            "cells": s.ncells, "dofs": dofs, "nx": cfg["nx"], "ny": cfg["ny"]}


if __name__ == "__main__":
    main()
