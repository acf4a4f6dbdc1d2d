"""Learned troubled-cell indicator: data generation, training and the
decision band (not part of the paper's method).

Everything numeric runs in the library's HIP kernels through the C ABI:
the FP64 cRKDG solver with the TVB limiter generates the labels, the
feature kernel the inputs, the MLP kernels the training (forward, backward,
Adam).  This module only orchestrates: seeds, sampling, minibatch order.

Labels: the FP64 TVB troubled-cell decision (flag bit 1) on the pre-limiter
state after each sampled step, on seeded four-quadrant Riemann problems and
seeded planar-shock problems.  Negatives are subsampled to at most 10 per
positive (seeded).
"""
import math

import numpy as np

from . import crkdg as K
from . import workloads as W

NPAR = 12 * 32 + 32 + 32 * 32 + 32 + 32 + 1


def quadrant_solver(seed, n, precision=K.FP64, split=None):
    cfg = W.config("c4", scale=1)
    cfg["nx"] = cfg["ny"] = n
    x0, x1, y0, y1 = cfg["box"]
    mesh = K.make_mesh(2, n, n, x0=x0, x1=x1, y0=y0, y1=y1, bc=(1, 1, 1, 1), equation=K.EQ_EULER,
                       gamma=W.GAMMA, precision=precision)
    s = K.Solver(mesh, cfg["k"], K.FLUX_LLF, 3)
    rng = np.random.default_rng(10_000 + seed)
    sp = split if split is not None else (0.5 + 0.02 * rng.uniform(-1, 1),
                                          0.5 + 0.02 * rng.uniform(-1, 1))
    s.crkdg_project(K.IC_QUADRANT, W.quadrant_params(seed, split=sp))
    return s, cfg


def shock_solver(seed, scale, precision=K.FP64):
    """the planar-shock workload (Mach 3 into a smoothed density field) with
    cell counts divided by `scale` and the shock angle and noise from `seed`"""
    import torch
    cfg = W.config("c5", scale=scale)
    params, xi = W.shock_problem(seed, cfg["nx"], cfg["ny"])
    x0, x1, y0, y1 = cfg["box"]
    ghost = W.post_shock_conserved(params[0])
    mesh = K.make_mesh(2, cfg["nx"], cfg["ny"], x0=x0, x1=x1, y0=y0, y1=y1, bc=(2, 1, 1, 1),
                       bc_state=[ghost] * 4, equation=K.EQ_EULER, gamma=W.GAMMA,
                       precision=precision)
    s = K.Solver(mesh, cfg["k"], K.FLUX_LLF, 3)
    s.crkdg_project(K.IC_SHOCK, params, aux=torch.from_numpy(xi).cuda())
    return s, cfg


def generate(seeds, n=128, samples=20, t_frac=0.25, M=50.0, neg_ratio=10, sample_seed=0,
             report=None, family="quadrant", max_steps=None, max_pos=20000, policy=None,
             precision=K.FP64):
    """features X (float32 [S, 12]) and TVB labels y (uint8 [S]) from FP64
    TVB runs with the given seeds, sampled at about `samples` evenly spaced
    steps.

    family "quadrant": four-quadrant problems on n x n cells, each run until
    the fastest initial wave has crossed t_frac of the domain.  family
    "shock": the planar-shock workload with cell counts divided by n, run to
    its final time or for max_steps steps.

    policy = (params, tau_lo, tau_hi): the runs are limited by the learned
    indicator instead of the TVB test (the states it will meet in use); the
    labels stay the FP64 TVB decisions, taken on an FP64 copy of each
    sampled state.

    Per sampled step at most max_pos positives are kept, and negatives are
    subsampled to neg_ratio per positive (at least 256).

    precision: the form the runs step in (the limiter's tests are FP64 in
    every form, so the labels are the FP64 TVB decisions on the run's own
    states).

    Some random quadrant states (strong collisions of low-pressure gas) drive
    a cell average out of the physical set, which neither the TVB limiter nor
    the positivity safeguard can repair; such a run stops there and keeps the
    samples taken before.  `report` (a dict, optional) receives the list of
    those seeds under "stopped"."""
    import torch
    Xs, ys = [], []
    stopped = []
    rng = np.random.default_rng(sample_seed)
    for seed in seeds:
        if family == "quadrant":
            s, cfg = quadrant_solver(seed, n, precision=precision)
            s.crkdg_limit(M)  # the projected jumps overshoot
            smax = s.crkdg_max_wavespeed()          # sum over directions of speed / h
            h = (cfg["box"][1] - cfg["box"][0]) / n
            T = t_frac / (smax * h / 2.0)
            nsteps = int(math.ceil(T / (cfg["cfl"] / smax)))
        elif family == "shock":
            s, cfg = shock_solver(seed, n, precision=precision)
            s.crkdg_limit(M)
            T = cfg["T"]
            nsteps = int(math.ceil(T / (cfg["cfl"] / s.crkdg_max_wavespeed())))
        else:
            raise ValueError(family)
        if max_steps is not None and nsteps > max_steps:
            nsteps = max_steps
        stride = max(1, nsteps // samples)
        t, step = 0.0, 0
        flags = torch.zeros(s.ncells, dtype=torch.uint8, device="cuda")
        X = torch.empty((s.ncells, 12), dtype=torch.float32, device="cuda")
        clone = None
        if policy is not None:
            clone = K.Solver(s.mesh, cfg["k"], K.FLUX_LLF, 3)
        while t < T - 1e-14 and step < nsteps:
            dt = min(cfg["cfl"] / s.crkdg_max_wavespeed(), T - t)
            s.crkdg_step(dt)
            t += dt
            step += 1
            sample = step % stride == 0
            if sample:
                s.crkdg_mlp_features(M, X)
            try:
                if policy is None:
                    s.crkdg_limit(M, flags if sample else None)
                else:
                    if sample:  # labels: the TVB decision on the same state
                        clone.crkdg_set_state(s.crkdg_get_state())
                        clone.crkdg_limit(M, flags)
                    s.crkdg_limit_mlp(M, policy[0], policy[1], policy[2], None)
            except K.CrkdgError as e:
                if e.code != K.CRKDG_ENONPHYSICAL:
                    raise
                stopped.append(seed)
                break
            if sample:
                lab = ((flags & 1) != 0).cpu().numpy()
                pos = np.nonzero(lab)[0]
                neg = np.nonzero(~lab)[0]
                if len(pos) > max_pos:
                    pos = rng.choice(pos, max_pos, replace=False)
                take = min(len(neg), max(neg_ratio * len(pos), 256))
                neg = rng.choice(neg, take, replace=False)
                idx = np.sort(np.concatenate([pos, neg]))
                Xs.append(X[torch.from_numpy(idx).cuda()].cpu().numpy())
                ys.append(lab[idx].astype(np.uint8))
        del s
    if report is not None:
        report["stopped"] = stopped
    if not Xs:
        return np.zeros((0, 12), np.float32), np.zeros(0, np.uint8)
    return np.concatenate(Xs).astype(np.float32), np.concatenate(ys).astype(np.uint8)


def init_params(seed=0):
    """He-uniform weights (suited to ReLU layers), zero biases (float64 host
    array)"""
    rng = np.random.default_rng(seed)
    P = np.zeros(NPAR)
    o = 0
    for fan_out, fan_in in ((32, 12), (32, 32)):
        lim = math.sqrt(6.0 / fan_in)
        P[o:o + fan_out * fan_in] = rng.uniform(-lim, lim, fan_out * fan_in)
        o += fan_out * fan_in + fan_out
    lim = math.sqrt(6.0 / 32)
    P[o:o + 32] = rng.uniform(-lim, lim, 32)
    return P


def train(X, y, epochs=10, batch=4096, lr=1e-3, pos_weight=None, seed=0):
    """Adam on the weighted BCE; deterministic given the seed.  Returns the
    device parameters and the per-epoch mean loss."""
    import torch
    dev = "cuda"
    if pos_weight is None:
        npos = max(1, int(y.sum()))
        pos_weight = (len(y) - npos) / npos
    Xd = torch.from_numpy(np.ascontiguousarray(X, dtype=np.float32)).to(dev)
    yd = torch.from_numpy(np.ascontiguousarray(y, dtype=np.uint8)).to(dev)
    P = torch.from_numpy(init_params(seed).astype(np.float32)).to(dev)
    m1 = torch.zeros_like(P)
    m2 = torch.zeros_like(P)
    grad = torch.empty_like(P)
    loss = torch.empty(1, dtype=torch.float32, device=dev)
    work = torch.empty(K.lib().crkdg_mlp_work_bytes(batch), dtype=torch.uint8, device=dev)
    rng = np.random.default_rng(seed + 1)
    step = 0
    hist = []
    for _ in range(epochs):
        perm = torch.from_numpy(rng.permutation(len(y))).to(dev)
        tot, nb = 0.0, 0
        for b0 in range(0, len(y) - batch + 1, batch):
            idx = perm[b0:b0 + batch]
            xb = Xd.index_select(0, idx).contiguous()
            yb = yd.index_select(0, idx).contiguous()
            K.crkdg_mlp_grad(P, xb, yb, pos_weight, grad, loss, work)
            step += 1
            K.crkdg_mlp_adam(P, m1, m2, grad, step, lr)
            tot += float(loss.item()) if nb % 16 == 0 else 0.0
            nb += 1
        hist.append(tot)
    return P, {"steps": step, "pos_weight": pos_weight, "loss_samples": hist}


def probabilities(P, X):
    import torch
    Xd = torch.from_numpy(np.ascontiguousarray(X, dtype=np.float32)).cuda()
    z = K.crkdg_mlp_forward(P, Xd).cpu().numpy().astype(np.float64)
    return 1.0 / (1.0 + np.exp(-z))


def choose_band(P, Xval, yval, fn_target=0.01, fp_target=0.01):
    """tau_lo: the largest threshold with at most fn_target of the TVB
    positives at or below it (those would be missed); tau_hi: the smallest
    threshold with at most fp_target of the negatives at or above it.  Cells
    in between go to the FP64 TVB test.  Thresholds are taken among the
    distinct probabilities, so tied values cannot push a rate past its target."""
    p = probabilities(P, Xval)
    pos = np.sort(p[yval == 1])
    neg = np.sort(p[yval == 0])
    k = int(math.floor(fn_target * len(pos)))
    vals = np.unique(pos)
    le = np.searchsorted(pos, vals, side="right")        # positives <= each value
    ok = vals[le <= k]
    tau_lo = float(ok[-1]) if ok.size else float(np.nextafter(pos[0], -np.inf))
    j = int(math.floor(fp_target * len(neg)))
    vals = np.unique(neg)
    ge = len(neg) - np.searchsorted(neg, vals, side="left")  # negatives >= each value
    ok = vals[ge <= j]
    tau_hi = float(ok[0]) if ok.size else float(np.nextafter(neg[-1], np.inf))
    tau_hi = max(tau_hi, tau_lo)
    return tau_lo, tau_hi


def rates(P, X, y, tau_lo, tau_hi):
    p = probabilities(P, X)
    pos = y == 1
    smooth = p <= tau_lo
    trouble = p >= tau_hi
    band = ~smooth & ~trouble
    return {"fn_rate": float((smooth & pos).sum() / max(1, pos.sum())),
            "fp_rate": float((trouble & ~pos).sum() / max(1, (~pos).sum())),
            "fallback_fraction": float(band.mean()),
            "n": int(len(y)), "positives": int(pos.sum())}


def compare_with_tvb(family, seed, n, P, tau_lo, tau_hi, M=50.0, samples=10, t_frac=0.25,
                     reference=True, precision=K.FP64):
    """what the learned indicator changes against the TVB test alone on one
    problem (the gain test): the same problem run to the same final time
    with the limiter deciding by the TVB test (M) and by the network with
    the FP64 TVB fallback band, in `precision`.  Reported: the limiter's
    device time per step, the flagged and fallback fractions, the false
    negative / positive rates of the network's decisions against the FP64
    TVB test taken on the same pre-limiter states (an FP64 copy, at about
    `samples` steps), and with `reference` the L1 / L2 errors of the density
    cell averages against an FP64 TVB run on the 2x finer mesh restricted to
    this one.  family: "quadrant" (n x n cells) or "shock" (cell counts
    divided by n).  If a run drives a cell average out of the physical set
    the result holds only "stopped" (the run that stopped)."""
    import torch

    def build(nn, prec):
        if family == "quadrant":
            s, cfg = quadrant_solver(seed, nn, precision=prec)
        else:
            s, cfg = shock_solver(seed, nn, precision=prec)
        s.crkdg_limit(M)  # the projected jumps overshoot
        return s, cfg

    s0, cfg = build(n, precision)
    if family == "quadrant":
        smax = s0.crkdg_max_wavespeed()
        h = (cfg["box"][1] - cfg["box"][0]) / n
        T = t_frac / (smax * h / 2.0)
    else:
        T = cfg["T"]
    del s0

    def run(nn, prec, learned, compare):
        s, cfg = build(nn, prec)
        flags = torch.zeros(s.ncells, dtype=torch.uint8, device="cuda")
        clone = tflags = None
        if compare:
            clone = K.Solver(s.mesh if prec == K.FP64 else
                             K.make_mesh(2, s.mesh.nx, s.mesh.ny, x0=s.mesh.x0, x1=s.mesh.x1,
                                         y0=s.mesh.y0, y1=s.mesh.y1, bc=tuple(s.mesh.bc),
                                         bc_state=[list(r) for r in s.mesh.bc_state],
                                         equation=K.EQ_EULER, gamma=s.mesh.gamma,
                                         precision=K.FP64), cfg["k"], K.FLUX_LLF, 3)
            tflags = torch.zeros(s.ncells, dtype=torch.uint8, device="cuda")
        t, step = 0.0, 0
        est = None
        tot = {"flagged": 0, "fallback": 0, "cells": 0, "tvb_pos": 0, "fn": 0, "fp": 0,
               "neg": 0, "limit_ms": 0.0}
        while t < T:
            dt = min(cfg["cfl"] / s.crkdg_max_wavespeed(), T - t)
            if est is None:
                est = max(1, int(T / dt) // samples)
            s.crkdg_step(dt)
            t = t + dt if T - t - dt > 1e-14 else T
            step += 1
            sample = compare and step % est == 0
            if sample:
                clone.crkdg_set_state(s.crkdg_get_state())
                clone.crkdg_limit(M, tflags)
            s.crkdg_profile_begin(4)
            if learned:
                nf, nb = s.crkdg_limit_mlp(M, P, tau_lo, tau_hi, flags if sample else None)
                tot["fallback"] += nb
            else:
                nf = s.crkdg_limit(M, flags if sample else None)
            prof = s.crkdg_profile_end()
            tot["limit_ms"] += prof.get("limit", (0.0, 0))[0]
            tot["flagged"] += nf
            tot["cells"] += s.ncells
            if sample:
                tv = (tflags & 1).bool()
                ml = (flags & 1).bool()
                tot["tvb_pos"] += int(tv.sum())
                tot["neg"] += int((~tv).sum())
                tot["fn"] += int((tv & ~ml).sum())
                tot["fp"] += int((ml & ~tv).sum())
        torch.cuda.synchronize()
        return s, step, tot

    out = {"family": family, "seed": seed, "mesh": None, "T": T}
    runs = {}
    for name, learned in (("tvb", False), ("learned", True)):
        try:
            s, nsteps, tot = run(n, precision, learned, compare=learned)
        except K.CrkdgError as e:
            # a cell average left the physical set (as some random quadrant
            # states do under any limiter): no comparison for this problem
            if e.code != K.CRKDG_ENONPHYSICAL:
                raise
            out["stopped"] = name
            return out
        out["mesh"] = f"{s.mesh.nx}x{s.mesh.ny}"
        r = {"steps": nsteps, "limit_ms_per_step": tot["limit_ms"] / nsteps,
             "flagged_fraction": tot["flagged"] / tot["cells"]}
        if learned:
            r["fallback_fraction"] = tot["fallback"] / tot["cells"]
            r["fn_rate_vs_tvb"] = tot["fn"] / max(1, tot["tvb_pos"])
            r["fp_rate_vs_tvb"] = tot["fp"] / max(1, tot["neg"])
            r["tvb_positives_sampled"] = tot["tvb_pos"]
        runs[name] = (s, r)
    if reference:
        fine = 2 * n if family == "quadrant" else max(1, n // 2)
        ref, _, _ = run(fine, K.FP64, False, compare=False)
        for name, (s, r) in runs.items():
            e = s.crkdg_error_ref(ref, 0)
            r["L1"], r["L2"] = float(e[0]), float(e[1])
    for name, (s, r) in runs.items():
        out[name] = r
    return out
