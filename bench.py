"""Throughput of the cRKDG step on one MI355X.

One "step" is one pass of the whole hot path over the 2D Euler shock
workload (4096 x 1024 cells, Q^2, scheme (eq:3), Lax--Friedrichs flux, Mach-3
shock into a smoothed density field; see paper_2307_06471_amd/workloads.py):
  inner stages (local operator)
  -> final stage (DG operator, face fluxes, conservative update)
  -> final-stage limiter (M = 50), which also reduces the cell wave speeds
     for the next step's dt (device reduction, no host sync).
The timed region holds K such steps with the state resident in HBM; the
result is DOF-updates/s (cells x modes x components per step).

The last line of stdout is one compact JSON line (a few KB): the headline
rate, `roofline` for the kernel with the largest share of the step time
(from HIP events recorded around every launch on the library's stream during
the timed region), `cpu_baseline` (the serial oracle on a bounded patch of
the same workload), the FP64 plain form and the equal-error verdict.  The
full report (every form's kernels, per-seed errors, the indicator's training
report) goes to the file named by --detail.
"""
import argparse
import json
import math
import os
import sys
import tempfile
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "2D Euler cRKDG DOF-updates/s: FP32+learned limiter vs FP64 plain, equal L2 err"
FN_TARGET = 0.005  # band: false negatives against TVB on validation (1% is the goal in use)
HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFLOPS = 78.6
FP32_PEAK_TFLOPS = 157.3  # MI355X vector FP32 (256 CUs x 4 SIMDs x 32 FMA lanes x 2 x 2.4 GHz)
# FP32 vector flops one step needs per cell (Q2 Euler, scheme eq3), every
# cell's stages evaluated once and u^n's volume integral shared by the first
# inner stage and the final stage: I + F, where I = 3686 is the inner-stage
# kernel's count per cell (1.546e10 per launch over 4194304 lanes) and F = 2862
# the one-pass kernel's final-stage part, from its 2.986e10 per launch over
# 67 strips x 64 lanes x (1024 full rows x (I + F) + 70 strip-end rows x I)
# (profiles/shock_4096x1024_q2_flop_counters.txt; the split schedule, which
# evaluates u^n's volume integral twice and the halo's traces again, executes
# 7529 per cell)
STEP_FLOP_PER_CELL = 6548.0


def algorithmic_bytes(cls, state_bytes, stage_bytes, ncells, stages_final, scheme="crkdg"):
    """bytes a kernel class must move per launch (its inputs and outputs):
    inner: read u^n, write the stored stage state(s); final: read u^n and the
    stored stage states, write u^{n+1}; limiter: read the state, write one
    flag byte per cell; dt: the final max over the limiter's per-block
    wave-speed maxima.  Original RKDG (SSP order 3): three DG-operator passes
    per step, the first reading u^n once (2 states moved), the others u^n and
    the previous stage (3 states): 8/3 states per launch on average; its
    limiter reads the state (no flags)."""
    if scheme == "rkdg3":
        if cls == "final":
            return 8 * state_bytes / 3
        if cls == "limit":
            return state_bytes
        return None
    if cls == "fused":  # the one-pass step: read u^n, write u^{n+1}
        return 2 * state_bytes
    if cls == "inner":
        return state_bytes + stage_bytes * (stages_final - 1)
    if cls == "final":
        return 2 * state_bytes + stage_bytes * (stages_final - 1)
    if cls == "limit":
        return state_bytes + ncells
    if cls == "dt":
        return ((ncells + 255) // 256) * 8  # the limiter's per-block maxima
    return None


def shock_mesh(K, W, cfg, theta, precision):
    x0, x1, y0, y1 = cfg["box"]
    ghost = W.post_shock_conserved(theta)
    return K.make_mesh(2, cfg["nx"], cfg["ny"], x0=x0, x1=x1, y0=y0, y1=y1, bc=(2, 1, 1, 1),
                       bc_state=[ghost] * 4, equation=K.EQ_EULER, gamma=W.GAMMA,
                       precision=precision)


def make_solver(K, W, scale=1, precision=0, field_grid=None, seed=2000, refine=1):
    import torch
    cfg = W.config("c5", scale=scale)
    cfg["nx"], cfg["ny"] = cfg["nx"] * refine, cfg["ny"] * refine
    params, xi = W.shock_problem(seed, cfg["nx"], cfg["ny"], field_grid=field_grid)
    s = K.Solver(shock_mesh(K, W, cfg, params[0], precision), cfg["k"], K.FLUX_LLF, 3)
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
    host, nproc = host_info()
    return {"value": dofs * n / el, "unit": "DOF-updates/s", "cores": 1, "kind": "oracle",
            "host": host, "nproc": nproc,
            "sample": f"{nx}x{ny}-cell patch of the same workload (Q2, eq3, LLF, TVB M=50, "
                      f"same cell size and boundary types), {n} steps after 1 warm-up, "
                      f"serial FP64 C oracle on one thread, {el:.1f} s"}


def log(msg):
    print(f"# {msg}", file=sys.stderr, flush=True)


def train_indicator(K, ML):
    """train the learned troubled-cell indicator with the library's own kernels
    on runs labelled by the FP64 TVB test (M = 50): four-quadrant Riemann
    problems and planar-shock problems with seeds other than the benchmark's.
    Pass 1 learns from runs limited by the TVB test; pass 2 adds runs
    limited by the pass-1 indicator (labels still from the TVB test on the
    same states) and retrains on both, so the network sees the states it
    meets in use.  The decision band comes from held-out seeds."""
    t0 = time.perf_counter()
    rep = {}

    def data(policy, seed_off):
        tr = [ML.generate(range(0, 32 if policy is None else 16), n=128, report=rep,
                          policy=policy, sample_seed=seed_off),
              ML.generate(range(2100, 2108), n=4, family="shock", policy=policy,
                          sample_seed=seed_off),
              ML.generate(range(2100, 2104), n=1, family="shock", max_steps=400, samples=10,
                          policy=policy, sample_seed=seed_off)]
        va = [ML.generate(range(64, 72), n=128, policy=policy, sample_seed=seed_off + 1),
              ML.generate(range(2200, 2202), n=4, family="shock", policy=policy,
                          sample_seed=seed_off + 1),
              ML.generate([2200], n=1, family="shock", max_steps=400, samples=10, policy=policy,
                          sample_seed=seed_off + 1)]
        return tr, va

    cat = lambda parts: (np.concatenate([p[0] for p in parts]),
                         np.concatenate([p[1] for p in parts]))
    # the band is chosen per problem family, on the shock family's own
    # validation runs (the workload the indicator serves); a pooled choice is
    # dominated by the more numerous quadrant samples and misses its
    # false-negative target on the shock workload
    tr1, va1 = data(None, 0)
    Xtr, ytr = cat(tr1)
    P1, _ = ML.train(Xtr, ytr, epochs=10, batch=4096, seed=0)
    lo1, hi1 = ML.choose_band(P1, *cat(va1[1:]), fn_target=FN_TARGET)
    tr2, va2 = data((P1, lo1, hi1), 10)
    Xtr, ytr = cat(tr1 + tr2)
    Xva, yva = cat(va1[1:] + va2[1:])
    t1 = time.perf_counter()
    P, info = ML.train(Xtr, ytr, epochs=10, batch=4096, seed=0)
    lo0, hi0 = ML.choose_band(P, Xva, yva, fn_target=FN_TARGET)
    # last round: the band on validation runs in the form of use (FP32 bulk)
    # limited by this network with that band, where its states come from
    va3 = [ML.generate(range(2200, 2202), n=4, family="shock", policy=(P, lo0, hi0),
                       sample_seed=30, precision=K.FP32_MIXED)]
    Xva3, yva3 = cat(va3)
    lo, hi = ML.choose_band(P, Xva3, yva3, fn_target=FN_TARGET)
    rv = ML.rates(P, Xva3, yva3, lo, hi)
    rv2 = ML.rates(P, Xva, yva, lo, hi)
    rq = ML.rates(P, *cat([va1[0], va2[0]]), lo, hi)
    t2 = time.perf_counter()
    return P, lo, hi, {
        "train": "pass 1: four-quadrant Riemann problems (seeds 0-31, 128x128 Q2, to 0.25 "
                 "domain crossings) + planar-shock problems (seeds 2100-2107 at 1024x256 to "
                 "T=0.25; seeds 2100-2103 at 4096x1024, 400 steps), limited by the TVB test; "
                 "pass 2: the same shock runs and quadrant seeds 0-15 limited by the pass-1 "
                 "indicator; labels always the FP64 TVB test, M=50",
        "validation_sets": "band: shock seeds 2200-2201 at 1024x256 in FP32 bulk, limited by "
                           "the trained network with a first band chosen on the FP64 shock "
                           "validation runs (2200-2201 at 1024x256, 2200 at 4096x1024 for 400 "
                           "steps, both policies); quadrant seeds 64-71 reported with the same "
                           "band",
        "band_round2": [lo0, hi0],
        "fn_target": FN_TARGET, "validation_quadrant": rq,
        "samples": int(len(ytr)), "positives": int(ytr.sum()),
        "runs_stopped_nonphysical": sorted(set(rep.get("stopped", []))),
        "adam_steps": info["steps"], "epochs": 10, "batch": 4096,
        "tau_lo": lo, "tau_hi": hi, "validation": rv, "validation_fp64_runs": rv2,
        "data_s": round(t1 - t0, 2), "train_s": round(t2 - t1, 2)}


def c4_study(K, ML, train_seeds=range(0, 64), val_seeds=range(64, 80), test_seeds=range(80, 96),
             n_test=1024):
    """the four-quadrant protocol of the learned indicator: training data from
    FP64 TVB runs of seeds 0-63 at 256^2 and 512^2, the band chosen on
    validation seeds 64-79 at 512^2 (runs limited by TVB, then by the network
    with that band), and the held-out seeds 80-95 at 1024^2 run twice in FP64,
    limited by TVB and by the network with the TVB fallback band; errors of
    both against an FP64 TVB run at 2048^2."""
    t0 = time.perf_counter()
    rep = {}
    X1, y1 = ML.generate(train_seeds, n=256, report=rep)
    log(f"c4 study: training runs at 256^2 done, {time.perf_counter() - t0:.0f} s")
    X2, y2 = ML.generate(train_seeds, n=512, sample_seed=1)
    log(f"c4 study: training runs at 512^2 done, {time.perf_counter() - t0:.0f} s")
    Xtr, ytr = np.concatenate([X1, X2]), np.concatenate([y1, y2])
    P, info = ML.train(Xtr, ytr, epochs=10, batch=4096, seed=0)
    log(f"c4 study: trained, {time.perf_counter() - t0:.0f} s")
    Xva, yva = ML.generate(val_seeds, n=512, sample_seed=2)
    lo0, hi0 = ML.choose_band(P, Xva, yva, fn_target=FN_TARGET)
    log(f"c4 study: first band ({lo0:.4g}, {hi0:.4g}), {time.perf_counter() - t0:.0f} s")
    Xvp, yvp = ML.generate(val_seeds, n=512, sample_seed=3, policy=(P, lo0, hi0))
    lo, hi = ML.choose_band(P, Xvp, yvp, fn_target=FN_TARGET)
    log(f"c4 study: {len(ytr)} training samples, band ({lo:.4g}, {hi:.4g}), "
        f"{time.perf_counter() - t0:.0f} s")
    rows, stopped = [], []
    for seed in test_seeds:
        r = ML.compare_with_tvb("quadrant", seed, n_test, P, lo, hi)
        if "stopped" in r:
            stopped.append(seed)
            log(f"c4 seed {seed}: the {r['stopped']} run left the physical set")
            continue
        rows.append(r)
        log(f"c4 seed {seed} ({time.perf_counter() - t0:.0f} s): "
            f"{json.dumps({k: r[k] for k in ('tvb', 'learned')})}")
    pos = sum(r["learned"]["tvb_positives_sampled"] for r in rows)
    agg = {
        "fn_rate_vs_tvb": sum(r["learned"]["fn_rate_vs_tvb"] * r["learned"]["tvb_positives_sampled"]
                              for r in rows) / max(1, pos),
        "fp_rate_vs_tvb_mean": float(np.mean([r["learned"]["fp_rate_vs_tvb"] for r in rows])),
        "L1_ratio_mean": float(np.mean([r["learned"]["L1"] / r["tvb"]["L1"] for r in rows])),
        "L2_ratio_mean": float(np.mean([r["learned"]["L2"] / r["tvb"]["L2"] for r in rows])),
        "limit_ms_tvb": float(np.mean([r["tvb"]["limit_ms_per_step"] for r in rows])),
        "limit_ms_learned": float(np.mean([r["learned"]["limit_ms_per_step"] for r in rows])),
        "flagged_tvb": float(np.mean([r["tvb"]["flagged_fraction"] for r in rows])),
        "flagged_learned": float(np.mean([r["learned"]["flagged_fraction"] for r in rows])),
        "fallback": float(np.mean([r["learned"]["fallback_fraction"] for r in rows])),
    }
    return {"train": "quadrant seeds 0-63 at 256^2 and 512^2, FP64 TVB labels",
            "samples": int(len(ytr)), "positives": int(ytr.sum()),
            "band": [lo, hi], "band_tvb_limited_validation": [lo0, hi0],
            "validation": ML.rates(P, Xvp, yvp, lo, hi), "test_mesh": f"{n_test}^2",
            "tested_seeds": len(rows), "stopped_nonphysical": stopped, "aggregate": agg,
            "per_seed": rows, "seconds": round(time.perf_counter() - t0, 1)}


def c3_rates(K, W, steps=100, warmup=20):
    """DOF-updates/s of the scaled density-wave workload (Section 4.1.2's
    example at 1024^2, Q^3, classical RK4, periodic, no limiter) in FP64 and
    in the FP32-bulk form: fixed dt (CFL 0.05) from the initial state, 100
    steps timed with HIP events after 20 warm-up steps"""
    import torch
    cfg = W.config("c3")
    x0, x1, y0, y1 = cfg["box"]
    out = {}
    for name, prec in (("fp64", K.FP64), ("fp32_bulk", K.FP32_MIXED)):
        mesh = K.make_mesh(2, cfg["nx"], cfg["ny"], x0=x0, x1=x1, y0=y0, y1=y1,
                           equation=K.EQ_EULER, gamma=W.GAMMA, precision=prec)
        s = K.Solver(mesh, cfg["k"], K.FLUX_LLF, W.RK_STAGES[cfg["tableau"]])
        s.crkdg_project(K.IC_EULER_WAVE, cfg["ic_params"])
        dt = torch.full((1,), cfg["cfl"] / s.crkdg_max_wavespeed(), dtype=torch.float64,
                        device="cuda")
        for _ in range(warmup):
            s.crkdg_step_dev(dt)
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        with torch.cuda.stream(s.stream):
            e0.record(s.stream)
            for _ in range(steps):
                s.crkdg_step_dev(dt)
            e1.record(s.stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / steps
        dofs = s.ncells * s.nmodes * s.ncomp
        out[name] = {"value": dofs / (ms * 1e-3), "ms_per_step": round(ms, 5)}
        del s
        torch.cuda.empty_cache()
    out["workload"] = (f"2D Euler density wave, {cfg['nx']}x{cfg['ny']} Q3, RK4, periodic, "
                       f"fixed dt (CFL {cfg['cfl']}), no limiter")
    return out


def dmr_run(K, k, nx, ny, precision, rkdg, T=0.2, M=50.0, cfl=0.1):
    """the paper's double Mach reflection (Section 4): projection, one limiter
    pass on the projected jump, then steps to T with dt = cfl / s_max; the
    limiter after every step (cRKDG) or inside every stage (RKDG).  Both keep
    dt and the time on the device (cRKDG: crkdg_step_dev + crkdg_limit_dt;
    RKDG: crkdg_step_rkdg with dt in device memory + crkdg_compute_dt), read
    the time back every 256 steps and take host steps only to land on T.
    Wall time covers the whole run, host synchronisation included."""
    import torch
    lm = K.make_mesh(2, nx, ny, x0=0.0, x1=4.0, y0=0.0, y1=1.0, bc=(2, 1, 2, 2),
                     bc_exact=K.IC_DMR, equation=K.EQ_EULER, gamma=1.4, precision=precision)
    s = K.Solver(lm, k, K.FLUX_LLF, 3)
    s.crkdg_project(K.IC_DMR)
    s.crkdg_limit(M)
    torch.cuda.synchronize()
    t, n = 0.0, 0
    t0 = time.perf_counter()
    chunk = 256
    dt_dev = torch.zeros(1, dtype=torch.float64, device="cuda")
    s.crkdg_compute_dt(cfl, dt_dev)
    while t + 2 * chunk * float(dt_dev.item()) < T:
        for _ in range(chunk):
            if rkdg:
                s.crkdg_step_rkdg(3, 0.0, M=M, dt_tensor=dt_dev)
                s.crkdg_compute_dt(cfl, dt_dev)
            else:
                s.crkdg_step_dev(dt_dev)
                s.crkdg_limit_dt(M, cfl, dt_dev)
        n += chunk
        t = s.crkdg_get_time()
    while t < T:
        dt = min(cfl / s.crkdg_max_wavespeed(), T - t)
        if rkdg:
            s.crkdg_step_rkdg(3, dt, M=M)
        else:
            s.crkdg_step(dt)
            s.crkdg_limit(M, count=False)
        t += dt
        n += 1
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    s.crkdg_limit(M)  # raises if a cell average went non-physical
    rho = s.crkdg_get_state()[0, 0]
    dofs = s.ncells * s.nmodes * s.ncomp
    return {"steps": n, "seconds": round(wall, 3), "ms_per_step": 1e3 * wall / n,
            "dof_updates_per_s": dofs * n / wall, "rho_min": float(rho.min()),
            "rho_max": float(rho.max())}, rho


def dmr_study(K):
    """1920 x 480 with Q1 and Q2 (the paper's fine runs): cRKDG and the
    original RKDG in FP64, FP32-bulk cRKDG with Q2"""
    out = {}
    for k in (1, 2):
        res = {}
        rho = {}
        forms = [("fp64 cRKDG", K.FP64, False), ("fp64 RKDG SSP3", K.FP64, True)]
        if k == 2:
            forms.append(("fp32-bulk cRKDG", K.FP32_MIXED, False))
        for name, prec, rk in forms:
            res[name], rho[name] = dmr_run(K, k, 1920, 480, prec, rk)
            log(f"dmr Q{k} 1920x480 {name}: {res[name]}")
        ref = rho["fp64 RKDG SSP3"]
        for name in rho:
            res[name]["rel_L1_density_vs_rkdg"] = float(np.abs(rho[name] - ref).sum() /
                                                        np.abs(ref).sum())
        out[f"Q{k}"] = res
    return out


def fehlberg_study(K, steps=10, warmup=2):
    """degree 4 with the six-stage fifth-order Runge--Kutta--Fehlberg method
    (Section 4 pairs them), FP64: 2D advection Q4 on 4096 x 1024 cells
    (upwind flux, periodic, velocity (1, 0.5)), fixed dt.  The full tableau
    takes one pass per inner stage i = 1..5: it reads u^(i-1), u^n (once for
    i = 1) and the i - 1 earlier loc outputs, and writes loc(u^(i-1)) (not
    for i = 5: no later stage uses it) and u^(i): 3 + 5 + 6 + 7 + 7 = 28
    states; the final pass reads u^n and the four other stages with
    b_i != 0 and writes u^{n+1}: 6 states."""
    import torch
    per_launch = {"inner": 28.0 / 5.0, "final": 6.0}  # states per launch
    cases = [
        ("2D advection Q4 4096x1024", K.make_mesh(2, 4096, 1024, x0=0.0, x1=4.0, y0=0.0, y1=1.0,
                                                   equation=K.EQ_ADVECTION, adv=(1.0, 0.5)),
         K.FLUX_UPWIND, K.IC_ADV_SIN, 0.02 / (1.0 * 1024 + 0.5 * 1024)),  # CFL 0.02
    ]
    out = {}
    for name, lm, flux, ic, dt in cases:
        s = K.Solver(lm, 4, flux, K.RK_FEHLBERG5)
        s.crkdg_project(ic)
        for _ in range(warmup):
            s.crkdg_step(dt)
        torch.cuda.synchronize()
        s.crkdg_profile_begin(16 * steps)
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        with torch.cuda.stream(s.stream):
            e0.record(s.stream)
            for _ in range(steps):
                s.crkdg_step(dt)
            e1.record(s.stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1)
        prof = s.crkdg_profile_end()
        dofs = s.ncells * s.nmodes * s.ncomp
        kern = {}
        for cls, (tms, cnt) in prof.items():
            if cnt == 0:
                continue
            by = per_launch.get(cls, 0.0) * s.state_bytes
            kern[cls] = {"ms_per_launch": tms / cnt, "launches": cnt, "share": tms / ms,
                         "achieved_GBs": by / (tms / cnt * 1e-3) / 1e9 if by else None}
        out[name] = {"value": dofs * steps / (ms / 1e3), "unit": "DOF-updates/s",
                     "ms_per_step": ms / steps, "dofs": dofs, "state_bytes": s.state_bytes,
                     "kernels": kern}
        log(f"fehlberg k=4 {name}: {ms / steps:.3f} ms/step, "
            f"{out[name]['value']:.3e} DOF-updates/s, "
            + ", ".join(f"{c} {v['achieved_GBs']:.0f} GB/s" for c, v in kern.items()
                        if v["achieved_GBs"]))
        del s
        torch.cuda.empty_cache()
    return out


def stream_copy_gbs(nbytes=1 << 30, reps=10):
    """achievable HBM bandwidth on this device: a device-to-device copy of
    `nbytes` (read once, written once), the best of `reps` event-timed
    copies, in GB/s of bytes moved"""
    import torch
    x = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    y = torch.empty_like(x)
    for _ in range(3):
        y.copy_(x)
    best = None
    for _ in range(reps):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        y.copy_(x)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1)
        best = ms if best is None else min(best, ms)
    del x, y
    torch.cuda.empty_cache()
    return 2 * nbytes / (best * 1e-3) / 1e9


def save_indicator(path, P, lo, hi, info):
    """a trained indicator as .npz: parameters, band, training report (JSON)"""
    np.savez(path, P=np.asarray(P, dtype=np.float32), lo=lo, hi=hi,
             info=np.array(json.dumps(info)))


def load_indicator(path):
    z = np.load(path)  # numeric and text arrays only (no pickles)
    info = json.loads(str(z["info"]))
    info["loaded_from"] = os.path.basename(path)
    return z["P"].astype(np.float32), float(z["lo"]), float(z["hi"]), info


def short_kernels(kern):
    """per-kernel-class ms per launch and achieved GB/s, rounded (compact line)"""
    return {c: {"ms": round(v["ms_per_launch"], 4), "launches": v["launches"],
                "GBs": None if v["achieved_GBs"] is None else round(v["achieved_GBs"], 1)}
            for c, v in kern.items()}


def host_info():
    host = "unknown CPU"
    try:
        with open("/proc/cpuinfo") as f:
            host = next(l.split(":", 1)[1].strip() for l in f if l.startswith("model name"))
    except (OSError, StopIteration):
        pass
    return host, os.cpu_count()


def write_detail(detail, path):
    """the full report (per-seed errors, training report, every form's kernels)
    goes to a file; stdout carries only the compact line"""
    d = os.path.dirname(path)
    if d:
        os.makedirs(d, exist_ok=True)
    with open(path, "w") as f:
        json.dump(detail, f, indent=1)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-equal-error", action="store_true")
    ap.add_argument("--equal-error-scale", type=int, default=4,
                    help="the equal-error runs use the workload with cell counts divided by this")
    ap.add_argument("--equal-error-full", action="store_true",
                    help="six seeds and every precision form in the equal-error study "
                         "(default: three seeds, the headline form against FP64 + TVB)")
    ap.add_argument("--all-forms", action="store_true",
                    help="also time the FP32-inner and FP32-increments forms")
    ap.add_argument("--scale", type=int, default=1, help="divide the cell counts (debug only)")
    ap.add_argument("--no-mlp", action="store_true",
                    help="profiling runs only: skip the learned indicator (training and form)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="end with a plain 256 MiB device copy (traffic counter calibration)")
    ap.add_argument("--no-c3", action="store_true",
                    help="skip the density-wave workload's rates (1024^2 Q3 RK4, FP64 and FP32 bulk)")
    ap.add_argument("--no-rkdg", action="store_true",
                    help="profiling runs only: skip the original-RKDG form")
    ap.add_argument("--fehlberg", action="store_true",
                    help="also run degree 4 with the six-stage fifth-order Runge-Kutta-Fehlberg "
                         "method (2D advection Q4)")
    ap.add_argument("--fehlberg-only", action="store_true",
                    help="profiling runs: only the degree-4 Fehlberg runs (prints their JSON)")
    ap.add_argument("--dmr", action="store_true",
                    help="also run the double Mach reflection at 1920x480 (Q1, Q2) to t = 0.2")
    ap.add_argument("--c4-study-only", action="store_true",
                    help="the learned indicator's four-quadrant protocol (train 0-63, validate "
                         "64-79, test 80-95 at 1024^2 against TVB; prints its JSON)")
    ap.add_argument("--full-size-study", action="store_true",
                    help="the shock workload at full size (4096x1024), seed 2000 unless "
                         "--full-size-seeds says otherwise: FP64 + TVB, "
                         "its 1e-7 control, the fused FP32-bulk forms and FP32-inner + TVB "
                         "against FP64 + TVB at 8192x2048 (prints its JSON; needs --indicator "
                         "or trains one)")
    ap.add_argument("--full-size-seeds", type=int, nargs="+", default=[2000],
                    help="seeds of --full-size-study (default 2000)")
    ap.add_argument("--full-size-forms", nargs="+",
                    default=["fp64 + TVB, perturbed 1e-7", "fp32-bulk fused + TVB",
                             "fp32-bulk fused + MLP", "fp32-inner + TVB"],
                    help="forms of --full-size-study besides FP64 + TVB (equal_error's names)")
    ap.add_argument("--dmr-only", action="store_true",
                    help="profiling runs: only the double Mach reflection study (prints its JSON)")
    ap.add_argument("--indicator", default=None,
                    help="profiling runs: .npz of a trained indicator, loaded if the file "
                         "exists, else written after training")
    ap.add_argument("--detail",
                    default=os.path.join(tempfile.gettempdir(), "crkdg_bench_detail.json"),
                    help="where the full report goes (the compact line is printed on stdout)")
    args = ap.parse_args()
    if args.equal_error_scale < 2:
        ap.error("--equal-error-scale must be at least 2 (the reference is twice as fine)")
    if args.gpus != 1:
        print(f"bench.py measures one GPU; this build has no multi-GPU path (--gpus {args.gpus})",
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2307_06471_amd import crkdg as K
    from paper_2307_06471_amd import mlp as ML
    from paper_2307_06471_amd import workloads as W

    if args.dmr_only:
        print(json.dumps({"double_mach_reflection": dmr_study(K)}), flush=True)
        return
    if args.c4_study_only:
        res = c4_study(K, ML)
        try:
            write_detail(res, args.detail)
        except OSError as e:
            log(f"could not write {args.detail}: {e}")
        print(json.dumps({k: v for k, v in res.items() if k != "per_seed"}), flush=True)
        return
    if args.fehlberg_only:
        print(json.dumps({"fehlberg_k4": fehlberg_study(K)}), flush=True)
        return

    mlp = None
    if not args.no_mlp:
        if args.indicator and os.path.exists(args.indicator):
            Pn, lo, hi, mlp_info = load_indicator(args.indicator)
            P = torch.from_numpy(Pn).cuda()
        else:
            P, lo, hi, mlp_info = train_indicator(K, ML)
            if args.indicator:
                save_indicator(args.indicator, P.cpu().numpy(), lo, hi, mlp_info)
        log(f"indicator trained: {mlp_info['samples']} samples, band ({lo:.4g}, {hi:.4g}), "
            f"validation {mlp_info['validation']}")
        mlp = (P, lo, hi)

    if args.full_size_study:
        if mlp is None:
            sys.exit("--full-size-study needs the learned indicator (drop --no-mlp)")
        res = equal_error(K, W, 1, mlp, seeds=tuple(args.full_size_seeds), full=True,
                          forms=("fp64 + TVB",) + tuple(args.full_size_forms))
        try:
            write_detail(res, args.detail)
        except OSError as e:
            log(f"could not write {args.detail}: {e}")
        print(json.dumps({k: v for k, v in res.items() if k != "per_seed"}), flush=True)
        return

    forms = {}
    F, S = K.SCHED_FUSED, K.SCHED_SPLIT
    plan = [("fp32-bulk fused + MLP", K.FP32_MIXED, mlp, F),
            ("fp32-bulk + MLP", K.FP32_MIXED, mlp, S)] if mlp is not None else []
    plan += [("fp64 + TVB", K.FP64, None, F), ("fp64 split + TVB", K.FP64, None, S),
             ("fp32-bulk fused + TVB", K.FP32_MIXED, None, F),
             ("fp32-bulk + TVB", K.FP32_MIXED, None, S)]
    if args.all_forms:
        plan += [("fp32-inner + TVB", K.FP32_INNER, None, S)]
        plan += [("fp32-increments + MLP", K.FP32_INCREMENTS, mlp, S)] if mlp is not None else []
        plan += [("fp32-increments + TVB", K.FP32_INCREMENTS, None, S)]
    head_name = "fp32-bulk fused + MLP" if mlp is not None else "fp32-bulk fused + TVB"
    other_name = head_name.replace("fp32-bulk fused", "fp32-bulk")
    for name, prec, ind, sched in plan:
        forms[name] = run_form(K, W, args, prec, ind, repeats=4 if name == head_name else 0,
                               schedule=sched)
        log(f"{name}: {forms[name]['ms_per_step']:.3f} ms/step, kernels "
            f"{json.dumps(short_kernels(forms[name]['kernels']))}")
    rk = None
    if not args.no_rkdg:
        rk = run_form(K, W, args, K.FP64, None, scheme="rkdg3")
        log(f"fp64 RKDG SSP3 + TVB every stage: {rk['ms_per_step']:.3f} ms/step")
    c3 = None
    if not args.no_c3:
        c3 = c3_rates(K, W)
        log(f"c3 density wave: {json.dumps(c3)}")
    head = forms[head_name]
    # (not in counter runs: their one large copy is the traffic calibration)
    copy_gbs = None if args.calibrate_copy else round(stream_copy_gbs(), 1)
    plain = forms["fp64 + TVB"]
    tvb32 = forms["fp32-bulk fused + TVB"]
    other = forms[other_name]
    workload = (f"2D Euler Mach-3 shock into a smoothed density field, {head['nx']}x{head['ny']} "
                f"Q2 cells on [0,4]x[0,1], cRKDG scheme eq3, Lax-Friedrichs flux, final-stage "
                f"limiter M=50, per-step dt (CFL 0.1)")
    form_text = ("fp32-bulk (FP32 contractions and fluxes, FP64 cell averages and face-flux sums) "
                 "+ learned troubled-cell indicator (12-32-32-1 MLP, FP64 TVB test inside its "
                 "uncertainty band)") if mlp is not None else \
        "fp32-bulk + TVB (profiling run without the learned indicator)"
    detail = {"metric": METRIC, "workload": workload, "form": form_text, "steps": args.steps,
              "warmup": args.warmup, "forms": forms, "stream_copy_GBs": copy_gbs}
    if rk is not None:
        detail["fp64_rkdg_ssp3"] = rk
    if c3 is not None:
        detail["c3_density_wave"] = c3
    if mlp is not None:
        detail["mlp"] = mlp_info
    ee = None
    if not args.no_equal_error and mlp is not None:
        ee = equal_error(K, W, args.equal_error_scale, mlp, full=args.equal_error_full)
        detail["equal_error"] = ee
        log(f"equal error: {ee['verdict']} {json.dumps(ee['mean_error_ratio_vs_fp64_tvb'])}")
    if args.fehlberg:
        detail["fehlberg_k4"] = fehlberg_study(K)
    if args.dmr:
        detail["double_mach_reflection"] = dmr_study(K)
    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(W)
        detail["cpu_baseline"] = cpu
    if args.calibrate_copy:
        x = torch.ones(1 << 26, dtype=torch.float32, device="cuda")
        y = torch.empty_like(x)
        for _ in range(3):
            y.copy_(x)
        torch.cuda.synchronize()
    try:
        write_detail(detail, args.detail)
    except OSError as e:
        log(f"could not write {args.detail}: {e}")

    roof = dict(head["roofline"])
    line = {
        "metric": METRIC, "value": head["value"], "unit": "DOF-updates/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(head["ms_per_step"], 5),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": workload, "form": head_name, "cells": head["cells"],
                   "dofs": head["dofs"], "parallelism": "1 GPU"},
        "roofline": roof,
        "cpu_baseline": None if cpu is None else {
            k: cpu[k] for k in ("value", "unit", "cores", "kind", "sample", "host", "nproc")},
        "kernels": short_kernels(head["kernels"]),
        "repeats_ms_per_step": [round(v, 5) for v in head["repeat_ms_per_step"]],
        "fp64_plain": {"value": plain["value"], "ms_per_step": round(plain["ms_per_step"], 5),
                       "roofline": {k: plain["roofline"][k]
                                    for k in ("kernel", "bound", "achieved", "unit", "frac")},
                       "kernels": short_kernels(plain["kernels"]),
                       "split_ms_per_step": round(forms["fp64 split + TVB"]["ms_per_step"], 5)},
        "fp32_bulk_fused_tvb": {"value": tvb32["value"],
                                "ms_per_step": round(tvb32["ms_per_step"], 5),
                                "limit_ms": round(tvb32["kernels"]["limit"]["ms_per_launch"], 5)},
        "split_schedule": {"form": other_name, "value": other["value"],
                           "ms_per_step": round(other["ms_per_step"], 5),
                           "kernels": short_kernels(other["kernels"]),
                           "roofline": {k: other["roofline"][k]
                                        for k in ("kernel", "achieved", "frac")}},
        "speedup_vs_fp64_plain": round(head["value"] / plain["value"], 4),
        "stream_copy_GBs": copy_gbs,
        "detail": args.detail,
    }
    if c3 is not None:
        line["c3_density_wave"] = {k: ({"value": v["value"], "ms_per_step": v["ms_per_step"]}
                                       if isinstance(v, dict) else v) for k, v in c3.items()
                                   if k != "workload"}
    if rk is not None:
        line["fp64_rkdg_ssp3"] = {"value": rk["value"], "ms_per_step": round(rk["ms_per_step"], 5),
                                  "crkdg_over_rkdg_fp64": round(plain["value"] / rk["value"], 4)}
    if mlp is not None:
        line["mlp"] = {"tau_lo": mlp_info["tau_lo"], "tau_hi": mlp_info["tau_hi"],
                       "validation": mlp_info["validation"],
                       "train_s": mlp_info.get("train_s"), "data_s": mlp_info.get("data_s")}
    if ee is not None:
        line["equal_error"] = {"mesh": ee["mesh"], "seeds": ee["seeds"],
                               "ratio_at_T": ee["mean_error_ratio_vs_fp64_tvb"][head_name]
                               [f"t={ee['checkpoints'][-1]}"],
                               "verdict": ee["verdict"], "indicator_vs_tvb": ee["indicator_rates"]}
    sys.stderr.flush()
    print(json.dumps(line, separators=(",", ":")), flush=True)


def measured_traffic(kernel, precision_tag):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter
    summary, if it was taken on the current kernel sources; else None"""
    from paper_2307_06471_amd import profsummary as PS
    d = PS.read_traffic(os.path.join(ROOT, "profiles", f"k_{kernel}_{precision_tag}_traffic.txt"))
    if not d or d.get("kernel source hash") != PS.kernel_source_hash():
        return None
    return float(d["traffic_bytes_per_launch"])


def run_form(K, W, args, precision, mlp=None, scheme="crkdg", repeats=0, schedule=None):
    """warm-up, then exactly args.steps timed steps (the reported rate);
    `repeats` further timed regions of args.steps steps each, continuing the
    same run, give the run-to-run spread (reported beside, not in, the rate).
    schedule: the library's step schedule (split or fused one-pass step)"""
    import torch
    s, cfg, params, xi = make_solver(K, W, args.scale, precision)
    s.crkdg_set_schedule(K.SCHED_SPLIT if schedule is None else schedule)
    stream = s.stream
    dt_dev = torch.zeros(1, dtype=torch.float64, device="cuda")
    flags = torch.zeros(s.ncells, dtype=torch.uint8, device="cuda")
    M = cfg["limiter"][1]

    P, lo, hi = mlp if mlp is not None else (None, 0.0, 0.0)

    def step():
        if scheme == "rkdg3":
            # the original RKDG: DG operator and limiter in each of three
            # stages, then the next step's dt from the new averages
            s.crkdg_step_rkdg(3, 0.0, M, dt_tensor=dt_dev)
            s.crkdg_compute_dt(cfg["cfl"], dt_dev)
            return
        # one step, then the limiter, which also leaves the next step's dt
        # (from the cell averages it reads; the limiter does not change them)
        s.crkdg_step_dev(dt_dev)
        s.crkdg_limit_dt(M, cfg["cfl"], dt_dev, flags, params=P, tau_lo=lo, tau_hi=hi)

    s.crkdg_compute_dt(cfg["cfl"], dt_dev)  # dt of the first step
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
    rep_ms = []
    for _ in range(repeats):
        r0 = torch.cuda.Event(enable_timing=True)
        r1 = torch.cuda.Event(enable_timing=True)
        with torch.cuda.stream(stream):
            r0.record(stream)
            for _ in range(args.steps):
                step()
            r1.record(stream)
        torch.cuda.synchronize()
        rep_ms.append(r0.elapsed_time(r1) / args.steps)
    n_flag = s.crkdg_limit(M, None, count=True)  # raises if a cell average went non-physical

    dofs = s.ncells * s.nmodes * s.ncomp
    stages_final = 2  # scheme (eq:3): b = (1/4, 0, 3/4)
    stage_bytes = s.state_bytes  # stored stages use the state's layout
    kern = {}
    for cls, (tms, cnt) in prof.items():
        by = algorithmic_bytes(cls, s.state_bytes, stage_bytes, s.ncells, stages_final, scheme)
        kern[cls] = {"ms_per_launch": tms / cnt, "launches": cnt, "share": tms / ms,
                     "achieved_GBs": None if by is None else by / (tms / cnt * 1e-3) / 1e9}
    dom = max(prof, key=lambda c: prof[c][0])
    by = algorithmic_bytes(dom, s.state_bytes, stage_bytes, s.ncells, stages_final, scheme)
    achieved = by / (prof[dom][0] / prof[dom][1] * 1e-3) / 1e9
    traffic = None if scheme != "crkdg" else measured_traffic(
        {"final": "final2", "inner": "inner", "limit": "limit", "fused": "fused2"}.get(dom, dom),
        {K.FP32_MIXED: "fp32", K.FP64: "fp64"}.get(precision, "fp32inner"))
    roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic, "kernel": dom,
            "bytes_per_launch": by}
    if traffic is not None:
        roof["traffic_over_algorithmic"] = round(traffic / by, 3)
    if dom == "fused" and cfg["k"] == 2:
        # the one-pass step does all of a step's arithmetic for 2S bytes per
        # cell: 20.5 flop/B in the FP32-bulk form (the FP32 ridge is 19.7
        # flop/B), 11.4 flop/B in FP64 (ridge 9.8 flop/B): ALU-bound
        fl = STEP_FLOP_PER_CELL * s.ncells
        peak = FP64_PEAK_TFLOPS if precision == K.FP64 else FP32_PEAK_TFLOPS
        tf = fl / (prof[dom][0] / prof[dom][1] * 1e-3) / 1e12
        roof = {"bound": "alu", "achieved": round(tf, 2), "peak": peak,
                "unit": "TFLOP/s", "frac": round(tf / peak, 4), "traffic": traffic,
                "kernel": dom, "flop_per_launch": fl, "bytes_per_launch": by,
                "hbm_achieved_GBs": round(achieved, 1),
                "hbm_frac": round(achieved / HBM_PEAK_GBS, 4)}
        if traffic is not None:
            roof["traffic_over_algorithmic"] = round(traffic / by, 3)
    return {"value": dofs * args.steps / (ms / 1e3), "ms_per_step": ms / args.steps,
            "repeat_ms_per_step": rep_ms,
            "roofline": roof, "kernels": kern, "flagged_cells_end": n_flag,
            "cells": s.ncells, "dofs": dofs, "nx": cfg["nx"], "ny": cfg["ny"]}


def equal_error(K, W, scale, mlp, full=False, checkpoints=(0.05, 0.1, 0.25), samples=10,
                seeds=None, forms=None):
    """the shock workload with cell counts divided by `scale`, run to T = 0.25
    by FP64 + TVB, the original RKDG (SSP-RK3, limiter every stage, FP64),
    FP32-inner + TVB, FP32-bulk + TVB, FP32-bulk + learned indicator and the
    two FP32-increments forms, for each seed; L1/L2 density errors of the cell averages against FP64 + TVB on the
    2x finer mesh restricted to this one (same initial density function), at
    each checkpoint time (the runs land on them exactly).

    The flow behind the shock is chaotic: a perturbation of 1e-12 of the
    initial state grows to an L1 difference of a few percent of the error by
    T.  A control run (FP64 + TVB from the initial state scaled by
    1 + 1e-7 noise, about the size of FP32 rounding) measures that spread.
    At about `samples` steps of the learned-indicator run its decisions are
    compared with the FP64 TVB test on the same (pre-limiter) state.
    `seeds` and `forms` (names from the list below) narrow the study."""
    import torch
    P, lo, hi = mlp
    T = checkpoints[-1]
    coarse = W.config("c5", scale)
    grid = (coarse["nx"], coarse["ny"])  # the reference sees the same initial density field

    def run(seed, refine, precision, indicator, at_checkpoint, rates=False, perturb=False,
            scheme="crkdg"):
        s, cfg, params, xi = make_solver(K, W, scale, precision, field_grid=grid, seed=seed,
                                         refine=refine)
        s.crkdg_set_schedule(K.SCHED_FUSED if scheme == "crkdg-fused" else K.SCHED_SPLIT)
        if perturb:
            u = s.crkdg_get_state()
            rng = np.random.default_rng(seed)
            s.crkdg_set_state(u * (1.0 + 1e-7 * rng.standard_normal(u.shape)))
        M = cfg["limiter"][1]
        flags = torch.zeros(s.ncells, dtype=torch.uint8, device="cuda")
        clone = None
        if rates:  # an FP64 copy of the state takes the TVB decisions for comparison
            clone = K.Solver(shock_mesh(K, W, cfg, params[0], K.FP64), cfg["k"], K.FLUX_LLF, 3)
            tflags = torch.zeros(s.ncells, dtype=torch.uint8, device="cuda")
        t, n, ci = 0.0, 0, 0
        tot = {"flagged": 0, "fallback": 0, "cells": 0, "tvb_pos": 0, "fn": 0, "fp": 0,
               "sampled": 0}
        nsteps_est = None
        t0 = tlog = time.perf_counter()
        while ci < len(checkpoints):
            if time.perf_counter() - tlog > 30.0:
                tlog = time.perf_counter()
                log(f"    {s.mesh.nx}x{s.mesh.ny} seed {seed}: step {n}, t = {t:.5f}")
            target = checkpoints[ci]
            dt = min(cfg["cfl"] / s.crkdg_max_wavespeed(), target - t)
            if nsteps_est is None:
                nsteps_est = int(T / dt) + 1
            if scheme == "rkdg3":
                s.crkdg_step_rkdg(3, dt, M)  # the limiter runs inside every stage
            else:
                s.crkdg_step(dt)
            t = t + dt if target - t - dt > 1e-14 else target
            n += 1
            sample = rates and n % max(1, nsteps_est // samples) == 0
            if sample:
                clone.crkdg_set_state(s.crkdg_get_state())
                clone.crkdg_limit(M, tflags)
            if scheme == "rkdg3":
                pass
            elif indicator is None:
                tot["flagged"] += s.crkdg_limit(M, flags if sample else None)
            else:
                nf, nb = s.crkdg_limit_mlp(M, P, lo, hi, flags if sample else None)
                tot["flagged"] += nf
                tot["fallback"] += nb
            tot["cells"] += s.ncells
            if sample:
                tv = (tflags & 1).bool()
                ml = (flags & 1).bool()
                tot["tvb_pos"] += int(tv.sum())
                tot["fn"] += int((tv & ~ml).sum())
                tot["fp"] += int((ml & ~tv).sum())
                tot["sampled"] += s.ncells
            if t == target:
                at_checkpoint(ci, s)
                ci += 1
        torch.cuda.synchronize()
        return s, n, tot, time.perf_counter() - t0

    if seeds is None:
        seeds = (2000, 2001, 2002, 2003, 2004, 2005) if full else (2000, 2001, 2002)
    only = forms
    forms = (("fp64 + TVB", K.FP64, None, False, "crkdg-fused"),
             ("fp64 + TVB, perturbed 1e-7", K.FP64, None, True, "crkdg-fused"),
             ("fp32-bulk + TVB", K.FP32_MIXED, None, False, "crkdg"),
             ("fp32-bulk fused + MLP", K.FP32_MIXED, mlp, False, "crkdg-fused"))
    if full:
        forms += (("fp64 RKDG SSP3 + TVB every stage", K.FP64, None, False, "rkdg3"),
                  ("fp32-inner + TVB", K.FP32_INNER, None, False, "crkdg"),
                  ("fp32-increments + TVB", K.FP32_INCREMENTS, None, False, "crkdg"),
                  ("fp32-increments + MLP", K.FP32_INCREMENTS, mlp, False, "crkdg"))
    if only is not None:
        forms = tuple(f for f in forms + (("fp32-bulk fused + TVB", K.FP32_MIXED, None, False,
                                           "crkdg-fused"),) if f[0] in only)
    per_seed = {}
    for seed in seeds:
        snaps = []
        ref, nref, _, tref = run(seed, 2, K.FP64, None,
                                 lambda ci, s: snaps.append(s.crkdg_get_state()),
                                 scheme="crkdg-fused")
        log(f"equal-error seed {seed}: reference {ref.mesh.nx}x{ref.mesh.ny}, {nref} steps, "
            f"{tref:.1f} s")
        res = {}
        base_snaps = []
        for name, prec, ind, pert, sch in forms:
            errs = []
            diffs = []

            def at_cp(ci, s):
                ref.crkdg_set_state(snaps[ci])
                e = s.crkdg_error_ref(ref, 0)
                errs.append((float(e[0]), float(e[1])))
                if name == "fp64 + TVB":
                    base_snaps.append(s.crkdg_get_state())
                else:
                    ref.crkdg_set_state(snaps[ci])  # keep ref for the next checkpoint

            s, n, tot, el = run(seed, 1, prec, ind, at_cp, rates=ind is not None,
                                perturb=pert, scheme=sch)
            r = {"L1": [e[0] for e in errs], "L2": [e[1] for e in errs], "steps": n,
                 "flagged_fraction": None if sch == "rkdg3" else tot["flagged"] / tot["cells"],
                 "seconds": round(el, 2)}
            if ind is not None:
                r["fallback_fraction"] = tot["fallback"] / tot["cells"]
                r["fn_rate_vs_tvb"] = tot["fn"] / max(1, tot["tvb_pos"])
                r["fp_rate_vs_tvb"] = tot["fp"] / max(1, tot["sampled"] - tot["tvb_pos"])
            res[name] = r
            log(f"  {name}: L1 {['%.4e' % v for v in r['L1']]} L2 {['%.4e' % v for v in r['L2']]} "
                f"flagged {r['flagged_fraction']}")
            del s
        per_seed[str(seed)] = res
        del ref

    def mean_ratio(name, norm, ci):
        return float(np.mean([per_seed[k][name][norm][ci] / per_seed[k]["fp64 + TVB"][norm][ci]
                              for k in per_seed]))

    ratios = {name: {f"t={tc}": {"L1": mean_ratio(name, "L1", ci), "L2": mean_ratio(name, "L2", ci)}
                     for ci, tc in enumerate(checkpoints)}
              for name, *_ in forms[1:]}
    def verdict(name):
        cand = ratios[name][f"t={T}"]
        return {"L2": "equal" if cand["L2"] <= 1.05 else "not equal",
                "L1": "equal" if cand["L1"] <= 1.05 else "not equal", "at": f"t={T}"}

    head = "fp32-bulk fused + MLP"
    rates = None
    if head in ratios:
        mlp_runs = [per_seed[k][head] for k in per_seed]
        rates = {key: float(np.mean([r[key] for r in mlp_runs]))
                 for key in ("fn_rate_vs_tvb", "fp_rate_vs_tvb", "fallback_fraction",
                             "flagged_fraction")}
        rates["fn_rate_vs_tvb_max"] = float(max(r["fn_rate_vs_tvb"] for r in mlp_runs))
        rates["tvb_flagged_fraction"] = float(np.mean(
            [per_seed[k]["fp64 + TVB"]["flagged_fraction"] for k in per_seed]))
    return {"mesh": f"{coarse['nx']}x{coarse['ny']}", "indicator_rates": rates,
            "reference": "FP64 + TVB on the 2x finer mesh, restricted; same initial density",
            "checkpoints": list(checkpoints), "seeds": list(seeds),
            "criterion": "mean over seeds of the density-error ratio to FP64 + TVB at most 1.05",
            "mean_error_ratio_vs_fp64_tvb": ratios, "per_seed": per_seed,
            "verdict": verdict(head) if head in ratios else None,
            "verdict_fp32_increments_mlp": (verdict("fp32-increments + MLP")
                                            if "fp32-increments + MLP" in ratios else None),
            "verdict_fp32_inner": (verdict("fp32-inner + TVB")
                                   if "fp32-inner + TVB" in ratios else None)}


if __name__ == "__main__":
    main()
