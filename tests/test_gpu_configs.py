"""Full-length runs of the smooth workloads at their full sizes.

C2: 2D Euler isentropic vortex, 256 x 256 Q^2, scheme (eq:3) of Section 2.2,
    Lax--Friedrichs flux, periodic, CFL 0.1 with a fixed dt, to T = 1 (about
    1,400 steps), FP64.  Compared with the oracle's own full run stored in
    tests/golden/c2_vortex_256.json (written by make_c2_vortex.py, which
    calls only the oracle): a sample of cells, per-(component, mode) sums and
    sums of squares over all cells and the conserved totals within 1e-12
    relative (the FP64 tolerance; the two sides differ only in rounding
    order), and the density errors against the exact vortex within what a
    state difference of that size can move them.
C3: 2D Euler density wave of Section 4.1.2 scaled to 1024 x 1024 Q^3, RK4,
    CFL 0.05 with a fixed dt, to T = 0.5, in FP64 and in the FP32-bulk form:
    the FP32-bulk state within 1e-5 relative L2 of the FP64 state, and both
    against the exact solution.
"""
import json
import math
import os

import numpy as np
import pytest

import oracle as O
from paper_2307_06471_amd import workloads as W

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def K():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_2307_06471_amd import crkdg
    return crkdg


def test_c2_vortex_full_run_against_the_oracle(K):
    with open(os.path.join(HERE, "golden", "c2_vortex_256.json")) as f:
        G = json.load(f)
    cfg = W.config("c2")
    nx, ny, k = cfg["nx"], cfg["ny"], cfg["k"]
    assert (G["nx"], G["ny"], G["k"]) == (nx, ny, k)
    x0, x1, y0, y1 = cfg["box"]
    om = O.Mesh(2, nx, ny, x0=x0, x1=x1, y0=y0, y1=y1, equation=O.EQ_EULER, gamma=W.GAMMA,
                flux=O.FLUX_LLF)
    mesh = K.make_mesh(2, nx, ny, x0=x0, x1=x1, y0=y0, y1=y1, equation=K.EQ_EULER,
                       gamma=W.GAMMA, precision=K.FP64)
    s = K.Solver(mesh, k, K.FLUX_LLF, W.RK_STAGES[cfg["tableau"]])
    u0 = O.project(om, k, O.IC_VORTEX, cfg["ic_params"])   # the oracle's initial DOFs
    s.crkdg_set_state(u0)
    dt = cfg["cfl"] / s.crkdg_max_wavespeed()
    assert abs(dt - G["dt"]) <= 1e-14 * G["dt"]
    dt = G["dt"]                                             # the same bits on both sides
    n = G["steps"]
    print(f"[c2] {nx}x{ny} Q{k}: {n} steps of dt {dt:.6g}", flush=True)
    for step in range(n - 1):
        s.crkdg_step(dt)
    s.crkdg_step(G["last_dt"])
    u = s.crkdg_get_state()
    cells = np.array(G["cells"])
    want = np.array(G["state"])                              # [cell][comp][mode]
    got = u[:, :, cells].transpose(2, 0, 1)
    err = np.abs(got - want).max() / np.abs(want).max()
    sums = np.array(G["sum"])
    sumsq = np.array(G["sumsq"])
    e_sum = np.abs(u.sum(axis=2) - sums).max() / np.abs(sums).max()
    e_sq = np.abs((u * u).sum(axis=2) - sumsq).max() / np.abs(sumsq).max()
    tot = [s.crkdg_total(c) for c in range(4)]
    e_tot = max(abs(tot[c] - G["total_T"][c]) / max(1.0, abs(G["total_T"][c])) for c in range(4))
    drift = max(abs(tot[c] - G["total_t0"][c]) / max(1.0, abs(G["total_t0"][c])) for c in range(4))
    e = s.crkdg_error(K.IC_VORTEX, cfg["ic_params"], t=cfg["T"])
    # the errors are small differences of O(1) values: a state difference
    # d moves L1 by at most |domain| d, L2 by sqrt(|domain|) d, Linf by d;
    # with d at the FP64 tolerance 1e-12 max|rho|
    area = (x1 - x0) * (y1 - y0)
    d = 1e-12 * np.abs(want[:, 0, 0]).max()
    e_err = max(abs(e[i] - G["errors_density"][i]) / (d * (area, np.sqrt(area), 1.0)[i])
                for i in range(3))
    print(f"[c2] sampled cells {err:.2e}, mode sums {e_sum:.2e}, sums of squares {e_sq:.2e}, "
          f"totals {e_tot:.2e} (drift from t=0 {drift:.2e}), density errors {e_err:.2e} of "
          f"their bound "
          f"(L1/L2/Linf {e[0]:.4e} {e[1]:.4e} {e[2]:.4e})", flush=True)
    assert err < 1e-12
    assert e_sum < 1e-12 and e_sq < 1e-12
    assert e_tot < 1e-12 and drift < 1e-13
    assert e_err <= 1.0


def run_fixed(K, s, dt, T):
    n = int(math.ceil(T / dt - 1e-12))
    for _ in range(n - 1):
        s.crkdg_step(dt)
    s.crkdg_step(T - (n - 1) * dt)
    return n


def test_c3_density_wave_fp32_bulk_against_fp64(K):
    cfg = W.config("c3")
    nx, ny, k = cfg["nx"], cfg["ny"], cfg["k"]
    x0, x1, y0, y1 = cfg["box"]
    out = {}
    dt = None
    for name, prec in (("fp64", K.FP64), ("fp32-bulk", K.FP32_MIXED)):
        mesh = K.make_mesh(2, nx, ny, x0=x0, x1=x1, y0=y0, y1=y1, equation=K.EQ_EULER,
                           gamma=W.GAMMA, precision=prec)
        s = K.Solver(mesh, k, K.FLUX_LLF, W.RK_STAGES[cfg["tableau"]])
        s.crkdg_project(K.IC_EULER_WAVE, cfg["ic_params"])
        if dt is None:
            dt = cfg["cfl"] / s.crkdg_max_wavespeed()
        print(f"[c3] {name} {nx}x{ny} Q{k} RK4, dt {dt:.6g}", flush=True)
        n = run_fixed(K, s, dt, cfg["T"])
        out[name] = (s.crkdg_get_state(), s.crkdg_error(K.IC_EULER_WAVE, cfg["ic_params"],
                                                         t=cfg["T"]))
        print(f"[c3] {name}: {n} steps, density L1/L2/Linf vs exact "
              f"{out[name][1][0]:.4e} {out[name][1][1]:.4e} {out[name][1][2]:.4e}", flush=True)
        del s
    u64, e64 = out["fp64"]
    u32, e32 = out["fp32-bulk"]
    rel = np.sqrt(((u32 - u64) ** 2).sum() / (u64 ** 2).sum())
    print(f"[c3] FP32-bulk vs FP64 relative L2 {rel:.3e}", flush=True)
    assert rel <= 1e-5
    # fourth order on a fine mesh: the FP64 error is far below FP32 round-off;
    # the FP32-bulk error is round-off (the density's L2 norm over [0, 2]^2 is
    # about 2, so 2e-5 is 1e-5 relative)
    assert e64[1] < 1e-9
    assert e32[1] < 2e-5
