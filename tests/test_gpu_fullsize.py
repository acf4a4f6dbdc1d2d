"""GPU parity at the full workload sizes, on sampled cells.

The oracle cannot step a million-cell mesh in seconds, but the method's
stencil is compact (Section 3.1): u^{n+1} of a cell depends only on u^n of
the cell and its four face neighbours, because the inner stages are element
local and only the final stage reaches across faces.  So for each sampled
cell the oracle steps the 3 x 3 patch of u^n around it (taken from the GPU
run, with the patch's true coordinates and the domain's boundary types on
the sides where the patch touches the boundary) and the patch centre must
equal the GPU's cell.  The limiter is checked the same way on the
pre-limiter state (its stencil is the four face neighbours too).

Each case runs the library in the launch configuration the benchmark times
(dt from the device reduction, crkdg_step_dev, then the limiter) for a few
steps before the checked step.

Tolerances: FP64 path 1e-12 relative to the largest value in the cell;
FP32-bulk and FP32-increments paths 1e-5 relative (FP32 arithmetic, one
step).
Limiter decisions are compared where the oracle's decision margin is above
1e-9 of the compared values' scale (both sides decide in FP64).
"""
import numpy as np
import pytest

import oracle as O
from paper_2307_06471_amd import workloads as W
from tests.helpers import BC, mlp_fp32_bound, tableau

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def K():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_2307_06471_amd import crkdg
    return crkdg


def build(K, name, precision, seed=None):
    """full-size solver of workload `name` with its initial condition"""
    import torch
    cfg = W.config(name)
    x0, x1, y0, y1 = cfg["box"]
    bc = tuple(BC[b] for b in cfg["bc"])
    bc_state = None
    aux = None
    if name == "c2":
        ic, params = K.IC_VORTEX, cfg["ic_params"]
    elif name == "c3":
        ic, params = K.IC_EULER_WAVE, cfg["ic_params"]
    elif name == "c4":
        ic, params = K.IC_QUADRANT, W.quadrant_params(seed)
    else:
        params, xi = W.shock_problem(seed, cfg["nx"], cfg["ny"])
        ic, aux = K.IC_SHOCK, torch.from_numpy(xi).cuda()
        bc_state = [W.post_shock_conserved(params[0])] * 4
    mesh = K.make_mesh(2, cfg["nx"], cfg["ny"], x0=x0, x1=x1, y0=y0, y1=y1, bc=bc,
                       bc_state=bc_state, equation=K.EQ_EULER, gamma=W.GAMMA,
                       precision=precision)
    s = K.Solver(mesh, cfg["k"], K.FLUX_LLF, W.RK_STAGES[cfg["tableau"]])
    if aux is not None:
        s.crkdg_project(ic, params, aux=aux)
    else:
        s.crkdg_project(ic, params)
    if cfg["limiter"] is not None:
        s.crkdg_limit(cfg["limiter"][1])  # projected jumps overshoot
    return s, cfg, bc, bc_state


def patch(cfg, bc, bc_state, u, i, j):
    """oracle mesh and state of the (up to) 3 x 3 patch around cell (i, j);
    returns the mesh, the patch state, and the centre's index in the patch"""
    nx, ny = cfg["nx"], cfg["ny"]
    x0, x1, y0, y1 = cfg["box"]
    dx, dy = (x1 - x0) / nx, (y1 - y0) / ny
    per_x, per_y = bc[0] == 0, bc[2] == 0
    ii = [i + d for d in (-1, 0, 1) if per_x or 0 <= i + d < nx]
    jj = [j + d for d in (-1, 0, 1) if per_y or 0 <= j + d < ny]
    cells = np.array([(b % ny) * nx + (a % nx) for b in jj for a in ii])
    pbc = (bc[0] if ii[0] == 0 and not per_x else 0,
           bc[1] if ii[-1] == nx - 1 and not per_x else 0,
           bc[2] if jj[0] == 0 and not per_y else 0,
           bc[3] if jj[-1] == ny - 1 and not per_y else 0)
    om = O.Mesh(2, len(ii), len(jj), x0=x0 + ii[0] * dx, x1=x0 + (ii[-1] + 1) * dx,
                y0=y0 + jj[0] * dy, y1=y0 + (jj[-1] + 1) * dy, bc=pbc, bc_state=bc_state,
                equation=O.EQ_EULER, gamma=W.GAMMA, flux=O.FLUX_LLF)
    centre = jj.index(j) * len(ii) + ii.index(i)
    return om, np.ascontiguousarray(u[:, :, cells]), centre


def sample_cells(cfg, rng, extra=()):
    nx, ny = cfg["nx"], cfg["ny"]
    fixed = [(0, 0), (nx - 1, 0), (0, ny - 1), (nx - 1, ny - 1), (nx // 2, 0), (0, ny // 2),
             (nx - 1, ny // 2), (nx // 2, ny - 1), (63, 3), (64, 4), (65, 7)]
    rnd = [(int(a), int(b)) for a, b in zip(rng.integers(0, nx, 120), rng.integers(0, ny, 120))]
    return fixed + rnd + list(extra)


CASES = [
    # name, precision, seed, steps before the checked one
    ("c2", "fp64", None, 4),
    ("c3", "fp64", None, 2),
    ("c3", "mixed", None, 2),
    ("c4", "fp64", 1000, 4),
    ("c4", "mixed", 1001, 4),
    ("c5", "fp64", 2000, 3),
    ("c5", "mixed", 2000, 3),
    ("c5", "incr", 2000, 3),
    # the fused one-pass step (same form, one kernel for the whole step)
    ("c4", "mixed-fused", 1001, 4),
    ("c5", "mixed-fused", 2000, 3),
]


@pytest.mark.parametrize("case", CASES, ids=lambda c: f"{c[0]}-{c[1]}")
def test_full_size_sampled_parity(K, case):
    import torch
    name, prec, seed, pre = case
    precision = {"fp64": K.FP64, "mixed": K.FP32_MIXED, "incr": K.FP32_INCREMENTS,
                 "mixed-fused": K.FP32_MIXED}[prec]
    tol = 1e-12 if prec == "fp64" else 1e-5
    s, cfg, bc, bc_state = build(K, name, precision, seed)
    s.crkdg_set_schedule(K.SCHED_FUSED if prec == "mixed-fused" else K.SCHED_SPLIT)
    print(f"[fullsize] {name} {prec} {cfg['nx']}x{cfg['ny']} k={cfg['k']}", flush=True)
    k = cfg["k"]
    tab = tableau(cfg["tableau"])
    lim = cfg["limiter"]
    dt_dev = torch.zeros(1, dtype=torch.float64, device="cuda")
    flags = torch.zeros(s.ncells, dtype=torch.uint8, device="cuda")

    def advance():
        s.crkdg_compute_dt(cfg["cfl"], dt_dev)
        s.crkdg_step_dev(dt_dev)

    for _ in range(pre):
        advance()
        if lim is not None:
            s.crkdg_limit(lim[1], flags, count=False)
    u0 = s.crkdg_get_state()
    advance()
    dt = float(dt_dev.item())
    u1 = s.crkdg_get_state()
    assert np.isfinite(u1).all()
    rng = np.random.default_rng(7)
    extra = ()
    if lim is not None:
        n = s.crkdg_limit(lim[1], flags)
        u2 = s.crkdg_get_state()
        fl = flags.cpu().numpy()
        troubled = np.nonzero(fl & 1)[0]
        assert n > 0 and len(troubled) > 0
        pick = rng.choice(troubled, min(60, len(troubled)), replace=False)
        extra = [(int(c % cfg["nx"]), int(c // cfg["nx"])) for c in pick]
    worst = 0.0
    agree = checked = 0
    for (i, j) in sample_cells(cfg, rng, extra):
        cell = j * cfg["nx"] + i
        om, up, c = patch(cfg, bc, bc_state, u0, i, j)
        ref = O.step_crkdg(om, k, tab, 0.0, dt, up)[:, :, c]
        got = u1[:, :, cell]
        err = np.abs(got - ref).max() / np.abs(ref).max()
        worst = max(worst, err)
        assert err < tol, (i, j, err)
        if lim is None:
            continue
        om, up, c = patch(cfg, bc, bc_state, u1, i, j)
        lo, flo, _ = O.limit_tvb(om, k, lim[1], up)
        _, margin, _ = O.tvb_flags(om, k, lim[1], up)
        if margin[c] <= 1e-9 * max(1.0, np.abs(up[:, 0]).max()):
            continue
        checked += 1
        assert (fl[cell] & 1) == (flo[c] & 1), (i, j, fl[cell], flo[c])
        if fl[cell] == flo[c]:
            agree += 1
            e2 = np.abs(u2[:, :, cell] - lo[:, :, c]).max() / np.abs(lo[:, :, c]).max()
            assert e2 < tol, (i, j, e2)
    print(f"[fullsize] {name} {prec}: worst step error {worst:.2e}; limiter cells checked "
          f"{checked}, identical flags {agree}", flush=True)
    if lim is not None:
        assert checked > 50 and agree >= 0.95 * checked


def test_full_size_learned_indicator_parity(K):
    """the benchmark's launch configuration of the headline form at full size
    (4096 x 1024 Q2 shock, FP32-bulk state, dt from the device, crkdg_step_dev,
    then crkdg_limit_dt with the learned indicator; a fixed random network
    and band (0.35, 0.65) stand in for the trained one).  On sampled cells the
    decision is the oracle's FP64 network on the oracle's features of the
    cell's 3 x 3 patch, and the FP64 TVB test inside the band; compared where
    the logit is further than the binary32 error bound from a threshold's
    logit and, in the band, the TVB margin above 1e-9 of the averages' scale.
    Limited states are compared where the decision equals the TVB test's;
    the sample holds 150 cells both the network and the TVB test flag and
    50 band cells the TVB test flags (besides cells the network alone flags,
    other band cells and random cells), so that more than 100 limited states
    are compared."""
    import torch
    s, cfg, bc, bc_state = build(K, "c5", K.FP32_MIXED, 2000)
    k, M, cfl = cfg["k"], cfg["limiter"][1], cfg["cfl"]
    rng = np.random.default_rng(5)
    P = 0.5 * rng.standard_normal(O.N_MLP_PARAMS)
    P[-1] = 0.3
    Pf = P.astype(np.float32)
    Pd = torch.from_numpy(Pf).cuda()
    lo, hi = 0.35, 0.65
    dt_dev = torch.zeros(1, dtype=torch.float64, device="cuda")
    flags = torch.zeros(s.ncells, dtype=torch.uint8, device="cuda")
    print(f"[fullsize] c5 learned indicator {cfg['nx']}x{cfg['ny']}", flush=True)
    s.crkdg_compute_dt(cfl, dt_dev)
    for _ in range(3):
        s.crkdg_step_dev(dt_dev)
        s.crkdg_limit_dt(M, cfl, dt_dev, flags, params=Pd, tau_lo=lo, tau_hi=hi)
    s.crkdg_step_dev(dt_dev)
    u1 = s.crkdg_get_state()
    s.crkdg_limit_dt(M, cfl, dt_dev, flags, params=Pd, tau_lo=lo, tau_hi=hi)
    u2 = s.crkdg_get_state()
    fl = flags.cpu().numpy()
    nx = cfg["nx"]
    # the TVB test's flags on the same pre-limiter state (a second handle):
    # limited states are compared where both tests flag a cell, so the sample
    # takes cells flagged by both, band cells, and cells the network alone flags
    tv = K.Solver(s.mesh, k, K.FLUX_LLF, 3)
    tv.crkdg_set_state(u1)
    tflags = torch.zeros(s.ncells, dtype=torch.uint8, device="cuda")
    tv.crkdg_limit(M, tflags)
    tf = tflags.cpu().numpy()
    del tv
    extra = []
    for sel, want in (((fl & 1) & (tf & 1), 150), ((fl & 8) & ((tf & 1) << 3), 50),
                      ((fl & 1) & ~tf & 1, 40), (fl & 8, 40)):
        cells = np.nonzero(sel)[0]
        assert len(cells) > 0, want
        extra += [(int(c % nx), int(c // nx)) for c in rng.choice(cells, min(want, len(cells)),
                                                                   replace=False)]
    P64 = Pf.astype(np.float64)
    zlo, zhi = np.log(lo / (1 - lo)), np.log(hi / (1 - hi))
    checked = states = 0
    for (i, j) in sample_cells(cfg, rng, extra):
        cell = j * nx + i
        om, up, c = patch(cfg, bc, bc_state, u1, i, j)
        X = O.mlp_features(om, k, M, up)[c:c + 1]
        z = O.mlp_forward(P64, X)[0]
        zb = mlp_fp32_bound(P64, X)[0]
        fo, margin, _ = O.tvb_flags(om, k, M, up)
        band = zlo < z < zhi
        scale = max(1.0, np.abs(up[:, 0]).max())
        if min(abs(z - zlo), abs(z - zhi)) <= zb or (band and margin[c] <= 1e-9 * scale):
            continue
        dec = int(fo[c] & 1) if band else int(z >= zhi)
        checked += 1
        assert (fl[cell] & 1) == dec, (i, j, z, fl[cell])
        assert ((fl[cell] & 8) != 0) == band, (i, j, z, fl[cell])
        if dec == (fo[c] & 1):
            lim, flo, _ = O.limit_tvb(om, k, M, up)
            if (fl[cell] & 7) == (flo[c] & 7):
                states += 1
                e = np.abs(u2[:, :, cell] - lim[:, :, c]).max() / np.abs(lim[:, :, c]).max()
                assert e < 1e-5, (i, j, e)
    print(f"[fullsize] learned indicator: decisions checked {checked}, limited states "
          f"checked {states}", flush=True)
    assert checked > 300 and states > 100
