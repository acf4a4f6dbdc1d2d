"""GPU parity of the HIP path (through the C ABI) against the CPU oracle.

Sizes span several 64x4 tiles and ragged tails.  Tolerance for the FP64
path: 1e-12 relative to the largest magnitude of the compared quantity
(the stated FP64 tolerance of the build); the two sides differ only in
rounding order (the GPU contracts a*b+c into FMAs, the oracle does not).
"""
import numpy as np
import pytest

import oracle as O
from paper_2307_06471_amd import workloads as W
from tests.helpers import BC, rel_err

pytestmark = pytest.mark.gpu

TOL = 1e-12


@pytest.fixture(scope="module")
def K():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_2307_06471_amd import crkdg
    return crkdg


def meshes(K, dim, nx, ny, equation, bc=(0, 0, 0, 0), bc_state=None, adv=(0.8, -0.6),
           box=(0.0, 1.0, 0.0, 1.0), bc_exact=0, flux="llf"):
    eqo = O.EQ_EULER if equation == "euler" else O.EQ_ADVECTION
    om = O.Mesh(dim, nx, ny, x0=box[0], x1=box[1], y0=box[2], y1=box[3], bc=bc,
                bc_state=bc_state, bc_exact=bc_exact, equation=eqo, adv=adv,
                flux=O.FLUX_LLF if flux == "llf" else O.FLUX_UPWIND)
    lm = K.make_mesh(dim, nx, ny, x0=box[0], x1=box[1], y0=box[2], y1=box[3], bc=bc,
                     bc_state=bc_state, bc_exact=bc_exact,
                     equation=K.EQ_EULER if equation == "euler" else K.EQ_ADVECTION, adv=adv)
    return om, lm


def random_state(equation, shape, seed):
    rng = np.random.default_rng(seed)
    if equation == "euler":
        return W.random_euler_modes(rng, shape[1], shape[2])
    return rng.standard_normal(shape)


def solver(K, lm, k, flux, stages=3):
    return K.Solver(lm, k, K.FLUX_LLF if flux == "llf" else K.FLUX_UPWIND, stages)


OP_CASES = [
    # dim, equation, nx, ny, bc, flux
    (2, "euler", 70, 9, (0, 0, 0, 0), "llf"),
    (2, "euler", 67, 5, (1, 1, 1, 1), "llf"),
    (2, "euler", 64, 4, (2, 1, 1, 2), "llf"),
    (2, "advection", 65, 6, (0, 0, 0, 0), "upwind"),
    (2, "advection", 33, 11, (1, 1, 0, 0), "llf"),
    (1, "advection", 300, 1, (0, 0, 0, 0), "upwind"),
    (1, "advection", 257, 1, (1, 1, 0, 0), "llf"),
]


@pytest.mark.parametrize("k", [0, 1, 2, 3])
@pytest.mark.parametrize("case", OP_CASES, ids=lambda c: f"{c[0]}d-{c[1]}-{c[2]}x{c[3]}-bc{c[4]}")
def test_operators(K, case, k):
    import torch
    dim, eq, nx, ny, bc, flux = case
    bcs = [[1.1, 0.2, -0.1, 2.7]] * 4 if eq == "euler" else [[0.3]] * 4
    om, lm = meshes(K, dim, nx, ny, eq, bc=bc, bc_state=bcs, flux=flux)
    s = solver(K, lm, k, flux)
    u = random_state(eq, om.shape(k), 11 * k + nx)
    x = torch.from_numpy(u.copy()).cuda()
    for op, oop in ((K.OP_LOC, O.OP_LOC), (K.OP_DG, O.OP_DG)):
        got = s.crkdg_apply_op(op, x).cpu().numpy()
        ref = O.apply(om, k, oop, u)
        assert rel_err(got, ref) < TOL, (op, rel_err(got, ref))


def test_combine(K):
    import torch
    om, lm = meshes(K, 2, 37, 5, "euler")
    s = solver(K, lm, 2, "llf")
    rng = np.random.default_rng(0)
    arrs = [rng.standard_normal(om.shape(2)) for _ in range(4)]
    coefs = [0.3, -1.25, 2.0, 1e-3]
    t = [torch.from_numpy(a).cuda() for a in arrs]
    out = s.crkdg_combine(t[0], coefs[:3], t[1:]).cpu().numpy()
    ref = arrs[0] + coefs[0] * arrs[1] + coefs[1] * arrs[2] + coefs[2] * arrs[3]
    assert rel_err(out, ref) < 1e-15
    out = s.crkdg_combine(None, coefs, t).cpu().numpy()
    ref = sum(c * a for c, a in zip(coefs, arrs))
    assert rel_err(out, ref) < 1e-15


def test_combine_odd_length_and_many_arrays(K):
    """an odd number of doubles (the last one takes the scalar tail path),
    up to six arrays, with and without a base, on a mesh whose vector count
    is not a multiple of the two vectors each thread handles per pass"""
    import torch
    om, lm = meshes(K, 1, 257, 1, "advection", flux="upwind")
    s = solver(K, lm, 0, "upwind")
    rng = np.random.default_rng(1)
    arrs = [rng.standard_normal(om.shape(0)) for _ in range(7)]
    assert arrs[0].size % 2 == 1
    t = [torch.from_numpy(a).cuda() for a in arrs]
    coefs = [0.3, -1.25, 2.0, 1e-3, -0.7, 0.25]
    out = s.crkdg_combine(t[0], coefs, t[1:]).cpu().numpy()
    ref = arrs[0] + sum(c * a for c, a in zip(coefs, arrs[1:]))
    assert rel_err(out, ref) < 1e-15
    out = s.crkdg_combine(None, coefs[:1], t[1:2]).cpu().numpy()
    assert rel_err(out, coefs[0] * arrs[1]) < 1e-15


TABS = ["fe", "eq2", "eq3", "rk4", "ssp3"]


@pytest.mark.parametrize("tab", TABS)
@pytest.mark.parametrize("k", [1, 2, 3])
def test_one_step_euler(K, tab, k):
    om, lm = meshes(K, 2, 70, 9, "euler", box=(0.0, 2.0, 0.0, 1.0))
    s = solver(K, lm, k, "llf")
    A, b, c = (np.array(v, float) for v in W.TABLEAU[tab])
    s.crkdg_set_tableau(A, b, c)
    u = random_state("euler", om.shape(k), 5 + k)
    s.crkdg_set_state(u)
    dt = 2e-3
    s.crkdg_step(dt)
    got = s.crkdg_get_state()
    ref = O.step_crkdg(om, k, (A, b, c), 0.0, dt, u)
    assert rel_err(got, ref) < TOL


@pytest.mark.parametrize("tab", TABS)
@pytest.mark.parametrize("dim", [1, 2])
def test_one_step_advection(K, tab, dim):
    k = 2
    om, lm = meshes(K, dim, 70 if dim == 2 else 300, 9, "advection", flux="upwind")
    s = solver(K, lm, k, "upwind")
    A, b, c = (np.array(v, float) for v in W.TABLEAU[tab])
    s.crkdg_set_tableau(A, b, c)
    u = random_state("advection", om.shape(k), 3)
    s.crkdg_set_state(u)
    s.crkdg_step(1e-3)
    ref = O.step_crkdg(om, k, (A, b, c), 0.0, 1e-3, u)
    assert rel_err(s.crkdg_get_state(), ref) < TOL


def test_c1_full_run(K):
    """1D advection workload: 640 steps, SSP-RK3 Butcher tableau, periodic"""
    cfg = W.config("c1")
    om, lm = meshes(K, 1, cfg["nx"], 1, "advection", box=cfg["box"], adv=(1.0, 0.0), flux="upwind")
    s = solver(K, lm, 2, "upwind")
    A, b, c = (np.array(v, float) for v in W.TABLEAU["ssp3"])
    s.crkdg_set_tableau(A, b, c)
    s.crkdg_project(K.IC_ADV_SIN)
    u0 = O.project(om, 2, O.IC_ADV_SIN)
    assert rel_err(s.crkdg_get_state(), u0) < 1e-14
    h = (cfg["box"][1] - cfg["box"][0]) / cfg["nx"]
    dt = cfg["dt_over_h"] * h
    u = u0.copy()
    for n in range(cfg["steps"]):
        s.crkdg_step(dt)
        u = O.step_crkdg(om, 2, (A, b, c), n * dt, dt, u)
    assert rel_err(s.crkdg_get_state(), u) < TOL
    e_gpu = s.crkdg_error(K.IC_ADV_SIN, (), t=cfg["steps"] * dt)
    e_or = O.errors(om, 2, u, O.IC_ADV_SIN, t=cfg["steps"] * dt)
    assert rel_err(e_gpu, e_or) < 1e-10


def test_small_vortex_run_and_conservation(K):
    cfg = W.config("c2", scale=8)  # 32 x 32
    om, lm = meshes(K, 2, cfg["nx"], cfg["ny"], "euler", box=cfg["box"])
    s = solver(K, lm, 2, "llf")
    s.crkdg_project(K.IC_VORTEX, cfg["ic_params"])
    u = O.project(om, 2, O.IC_VORTEX, cfg["ic_params"])
    assert rel_err(s.crkdg_get_state(), u) < 1e-13
    smax = s.crkdg_max_wavespeed()
    assert abs(smax - O.max_wavespeed(om, 2, u)) < 1e-14 * smax
    dt = cfg["cfl"] / smax
    m0 = [s.crkdg_total(c) for c in range(4)]
    for c in range(4):
        assert abs(m0[c] - O.total_mass(om, 2, u, c)) < 1e-13 * max(1, abs(m0[c]))
    A, b, cc = (np.array(v, float) for v in W.TABLEAU["eq3"])
    for n in range(40):
        s.crkdg_step(dt)
        u = O.step_crkdg(om, 2, (A, b, cc), n * dt, dt, u)
    assert rel_err(s.crkdg_get_state(), u) < TOL
    for c in range(4):
        assert abs(s.crkdg_total(c) - m0[c]) < 1e-13 * max(1, abs(m0[c]))
    e = s.crkdg_error(K.IC_VORTEX, cfg["ic_params"], t=40 * dt)
    eo = O.errors(om, 2, u, O.IC_VORTEX, cfg["ic_params"], t=40 * dt)
    assert rel_err(e, eo) < 1e-10


def test_bitwise_determinism(K):
    cfg = W.config("c2", scale=8)
    om, lm = meshes(K, 2, cfg["nx"], cfg["ny"], "euler", box=cfg["box"])
    outs = []
    for _ in range(2):
        s = solver(K, lm, 2, "llf")
        s.crkdg_project(K.IC_VORTEX, cfg["ic_params"])
        for _ in range(10):
            s.crkdg_step(0.01)
        outs.append(s.crkdg_get_state())
    assert np.array_equal(outs[0], outs[1])


@pytest.mark.parametrize("ic", ["const", "adv1", "adv2", "wave", "vortex", "quadrant", "shock",
                                "shock_coarse_field"])
def test_projection(K, ic):
    k = 2
    if ic in ("adv1",):
        om, lm = meshes(K, 1, 100, 1, "advection", box=(0.0, 2 * np.pi, 0, 1), adv=(1.0, 0.0))
        p, oid, lid, aux = [], O.IC_ADV_SIN, K.IC_ADV_SIN, None
    elif ic == "adv2":
        om, lm = meshes(K, 2, 40, 30, "advection", box=(-1.0, 1.0, -1.0, 1.0), adv=(1.0, 1.0))
        p, oid, lid, aux = [], O.IC_ADV_SIN, K.IC_ADV_SIN, None
    else:
        box = (0.0, 4.0, 0.0, 1.0) if ic == "shock" else (0.0, 2.0, 0.0, 2.0)
        om, lm = meshes(K, 2, 130, 33, "euler", box=box)
        aux = None
        if ic == "const":
            p, oid, lid = [1.0, 0.3, -0.2, 2.5], O.IC_CONST, K.IC_CONST
        elif ic == "wave":
            p, oid, lid = [0.7, 0.3, 1.0], O.IC_EULER_WAVE, K.IC_EULER_WAVE
        elif ic == "vortex":
            p, oid, lid = [5.0, 1.0, 1.0, 2.0, 2.0], O.IC_VORTEX, K.IC_VORTEX
        elif ic == "quadrant":
            p, oid, lid = W.quadrant_params(3, split=(1.03, 0.97)), O.IC_QUADRANT, K.IC_QUADRANT
        elif ic == "shock":
            p, aux = W.shock_problem(2000, 130, 33)
            oid, lid = O.IC_SHOCK, K.IC_SHOCK
        else:  # the noise field on a coarser grid than the mesh
            p, aux = W.shock_problem(2000, 130, 33, field_grid=(45, 17))
            oid, lid = O.IC_SHOCK, K.IC_SHOCK
    s = solver(K, lm, k, "llf" if ic not in ("adv1", "adv2") else "upwind")
    if aux is not None:
        import torch
        s.crkdg_project(lid, p, aux=torch.from_numpy(aux).cuda())
    else:
        s.crkdg_project(lid, p)
    ref = O.project(om, k, oid, p if p else None, aux)
    assert rel_err(s.crkdg_get_state(), ref) < 1e-13


def test_inflow_boundary_stage_times(K):
    """1D advection with inflow data sin(-t) on the left, evaluated at the
    final-stage times (Section 3.4); 100 steps of scheme (eq:3)"""
    N, k = 80, 2
    L = 4 * np.pi
    om, lm = meshes(K, 1, N, 1, "advection", box=(0.0, L, 0, 1), adv=(1.0, 0.0), bc=(2, 1, 0, 0),
                    bc_exact=O.IC_ADV_SIN, flux="upwind")
    s = solver(K, lm, k, "upwind", stages=3)
    s.crkdg_project(K.IC_ADV_SIN)
    u = O.project(om, k, O.IC_ADV_SIN)
    A, b, c = (np.array(v, float) for v in W.TABLEAU["eq3"])
    dt = 0.16 * L / N
    for n in range(100):
        s.crkdg_step(dt)
        u = O.step_crkdg(om, k, (A, b, c), n * dt, dt, u)
    assert rel_err(s.crkdg_get_state(), u) < TOL


@pytest.mark.parametrize("k", [1, 2, 3])
def test_limiter(K, k):
    """one limiter application on a projected quadrant state with jumps that
    cut cells; flags compared where the decision margin exceeds 1e-9"""
    import torch
    om, lm = meshes(K, 2, 70, 37, "euler", bc=(1, 1, 1, 1))
    p = W.quadrant_params(7, split=(0.503, 0.497))
    s = solver(K, lm, k, "llf")
    s.crkdg_project(K.IC_QUADRANT, p)
    u = O.project(om, k, O.IC_QUADRANT, p)
    # smooth perturbation so that many cells sit near the thresholds
    rng = np.random.default_rng(k)
    u[:, 1:] += 5e-5 * rng.standard_normal(u[:, 1:].shape)  # around M h^2 = 1e-4
    s.crkdg_set_state(u)
    flags = torch.zeros(om.ncells, dtype=torch.uint8, device="cuda")
    n_gpu = s.crkdg_limit(0.5, flags)
    lim_o, fl_o, n_o = O.limit_tvb(om, k, 0.5, u)
    _, margin, _ = O.tvb_flags(om, k, 0.5, u)
    fg = flags.cpu().numpy()
    safe = margin > 1e-9
    assert safe.mean() > 0.9
    assert np.array_equal(fg[safe] != 0, fl_o[safe] != 0)
    agree = (fg == fl_o)
    got = s.crkdg_get_state()
    assert rel_err(got[:, :, agree], lim_o[:, :, agree]) < 1e-13
    assert np.array_equal(got[:, 0], u[:, 0])  # means untouched
    assert abs(n_gpu - n_o) <= (~safe).sum()


# --- FP32-bulk form (FP64 cell averages, FP32 higher modes and arithmetic) ----

def mixed_solver(K, cfg, k, stages, bc_state=None):
    x0, x1, y0, y1 = cfg["box"]
    bc = tuple(BC[b] for b in cfg["bc"])
    lm = K.make_mesh(2, cfg["nx"], cfg["ny"], x0=x0, x1=x1, y0=y0, y1=y1, bc=bc,
                     bc_state=bc_state, equation=K.EQ_EULER, precision=K.FP32_MIXED)
    om = O.Mesh(2, cfg["nx"], cfg["ny"], x0=x0, x1=x1, y0=y0, y1=y1, bc=bc, bc_state=bc_state,
                equation=O.EQ_EULER, flux=O.FLUX_LLF)
    return K.Solver(lm, k, K.FLUX_LLF, stages), om


def l2_rel(a, b):
    return float(np.sqrt(((a - b) ** 2).sum() / (b ** 2).sum()))


@pytest.mark.parametrize("sched", ["split", "fused"])
@pytest.mark.parametrize("k,tab,stages", [(2, "eq3", 3), (3, "rk4", 4), (1, "eq2", 2)])
def test_mixed_density_wave_run(K, k, tab, stages, sched):
    """density-wave workload (Section 4.1.2 example), 48 x 40 cells, 60 steps:
    the FP32-bulk form stays within 1e-5 relative L2 of the FP64 oracle, its
    cell averages stay FP64 and the sums are conserved to FP64 round-off; in
    both step schedules (RK4 has weights on every stage, so it always takes
    the split one)"""
    cfg = dict(W.config("c3"), nx=48, ny=40)
    s, om = mixed_solver(K, cfg, k, stages)
    if sched == "split":
        s.crkdg_set_schedule(K.SCHED_SPLIT)
    elif tab != "rk4":
        s.crkdg_set_schedule(K.SCHED_FUSED)
    assert s.crkdg_get_schedule() == (K.SCHED_FUSED if sched == "fused" and tab != "rk4"
                                      else K.SCHED_SPLIT)
    P = cfg["ic_params"]
    s.crkdg_project(K.IC_EULER_WAVE, P)
    u = O.project(om, k, O.IC_EULER_WAVE, P)
    got0 = s.crkdg_get_state()
    assert rel_err(got0[:, 0], u[:, 0]) < 1e-14          # FP64 averages
    assert rel_err(got0, u) < 1e-7                       # FP32 higher modes
    m0 = [s.crkdg_total(c) for c in range(4)]
    dt = cfg["cfl"] / O.max_wavespeed(om, k, u)
    A, b, c = (np.array(v, float) for v in W.TABLEAU[tab])
    for n in range(60):
        s.crkdg_step(dt)
        u = O.step_crkdg(om, k, (A, b, c), n * dt, dt, u)
    got = s.crkdg_get_state()
    assert l2_rel(got, u) < 1e-5, l2_rel(got, u)
    for cc in range(4):
        assert abs(s.crkdg_total(cc) - m0[cc]) < 1e-13 * max(1.0, abs(m0[cc]))


def test_fp32_inner_density_wave_run(K):
    """FP32 inner stages (stored as FP32 increments over u^n), FP64 final
    stage: Section 3.3's perturbation argument says the inner-stage error
    enters a step only at O(eps dt^2).  Same run as above (Q^2, scheme (eq:3),
    48 x 40, 60 steps): far closer to the FP64 oracle than the FP32-bulk form,
    and conservative to FP64 round-off."""
    cfg = dict(W.config("c3"), nx=48, ny=40)
    P = cfg["ic_params"]
    k, tab = 2, "eq3"
    errs = {}
    for prec in (K.FP32_INNER, K.FP32_MIXED):
        x0, x1, y0, y1 = cfg["box"]
        lm = K.make_mesh(2, cfg["nx"], cfg["ny"], x0=x0, x1=x1, y0=y0, y1=y1, bc=(0, 0, 0, 0),
                         equation=K.EQ_EULER, precision=prec)
        om = O.Mesh(2, cfg["nx"], cfg["ny"], x0=x0, x1=x1, y0=y0, y1=y1, bc=(0, 0, 0, 0),
                    equation=O.EQ_EULER, flux=O.FLUX_LLF)
        s = K.Solver(lm, k, K.FLUX_LLF, 3)
        s.crkdg_project(K.IC_EULER_WAVE, P)
        u = O.project(om, k, O.IC_EULER_WAVE, P)
        m0 = [s.crkdg_total(c) for c in range(4)]
        dt = cfg["cfl"] / O.max_wavespeed(om, k, u)
        A, b, c = (np.array(v, float) for v in W.TABLEAU[tab])
        for n in range(60):
            s.crkdg_step(dt)
            u = O.step_crkdg(om, k, (A, b, c), n * dt, dt, u)
        errs[prec] = l2_rel(s.crkdg_get_state(), u)
        if prec == K.FP32_INNER:
            for cc in range(4):
                assert abs(s.crkdg_total(cc) - m0[cc]) < 1e-13 * max(1.0, abs(m0[cc]))
    print(f"[fp32-inner] rel L2 vs FP64 oracle: inner {errs[K.FP32_INNER]:.2e}, "
          f"bulk {errs[K.FP32_MIXED]:.2e}", flush=True)
    assert errs[K.FP32_INNER] < 1e-7
    assert errs[K.FP32_INNER] < 0.1 * errs[K.FP32_MIXED]


def test_fp32_inner_shock_step_matches_oracle(K):
    """one step of the shock workload (128 x 32, Dirichlet inflow, limiter
    after) in the FP32-inner form against the FP64 oracle"""
    import torch
    cfg = W.config("c5", scale=32)
    params, xi = W.shock_problem(2000, cfg["nx"], cfg["ny"])
    ghost = W.post_shock_conserved(params[0])
    x0, x1, y0, y1 = cfg["box"]
    lm = K.make_mesh(2, cfg["nx"], cfg["ny"], x0=x0, x1=x1, y0=y0, y1=y1, bc=(2, 1, 1, 1),
                     bc_state=[ghost] * 4, equation=K.EQ_EULER, precision=K.FP32_INNER)
    om = O.Mesh(2, cfg["nx"], cfg["ny"], x0=x0, x1=x1, y0=y0, y1=y1, bc=(2, 1, 1, 1),
                bc_state=[ghost] * 4, equation=O.EQ_EULER, flux=O.FLUX_LLF)
    s = K.Solver(lm, 2, K.FLUX_LLF, 3)
    s.crkdg_project(K.IC_SHOCK, params, aux=torch.from_numpy(xi).cuda())
    s.crkdg_limit(50.0)
    u = s.crkdg_get_state()
    dt = cfg["cfl"] / O.max_wavespeed(om, 2, u)
    s.crkdg_step(dt)
    A, b, c = (np.array(v, float) for v in W.TABLEAU["eq3"])
    ref = O.step_crkdg(om, 2, (A, b, c), 0.0, dt, u)
    got = s.crkdg_get_state()
    assert l2_rel(got, ref) < 1e-8


def test_fp32_increments_density_wave_run(K):
    """FP32 arithmetic in the inner and the final stage, increments over the
    FP64 u^n added in FP64.  Same run as above (Q^2, scheme (eq:3), 48 x 40,
    60 steps).  On this smooth run it is as close to the FP64 oracle as the
    FP32-bulk form (measured 9.9e-8 and 1.0e-7): the FP32 evaluation of the
    final stage's DG operator already errs by O(eps CFL) per step (its face
    and volume fluxes cancel to a difference of size O(h)), so rounding the
    stored modes to FP32 was not the larger term.  Conservative to FP64
    round-off (FP64 cell averages and face sums)."""
    cfg = dict(W.config("c3"), nx=48, ny=40)
    P = cfg["ic_params"]
    k, tab = 2, "eq3"
    errs = {}
    for prec in (K.FP32_INCREMENTS, K.FP32_MIXED):
        x0, x1, y0, y1 = cfg["box"]
        lm = K.make_mesh(2, cfg["nx"], cfg["ny"], x0=x0, x1=x1, y0=y0, y1=y1, bc=(0, 0, 0, 0),
                         equation=K.EQ_EULER, precision=prec)
        om = O.Mesh(2, cfg["nx"], cfg["ny"], x0=x0, x1=x1, y0=y0, y1=y1, bc=(0, 0, 0, 0),
                    equation=O.EQ_EULER, flux=O.FLUX_LLF)
        s = K.Solver(lm, k, K.FLUX_LLF, 3)
        s.crkdg_project(K.IC_EULER_WAVE, P)
        u = O.project(om, k, O.IC_EULER_WAVE, P)
        m0 = [s.crkdg_total(c) for c in range(4)]
        dt = cfg["cfl"] / O.max_wavespeed(om, k, u)
        A, b, c = (np.array(v, float) for v in W.TABLEAU[tab])
        for n in range(60):
            s.crkdg_step(dt)
            u = O.step_crkdg(om, k, (A, b, c), n * dt, dt, u)
        errs[prec] = l2_rel(s.crkdg_get_state(), u)
        if prec == K.FP32_INCREMENTS:
            for cc in range(4):
                assert abs(s.crkdg_total(cc) - m0[cc]) < 1e-13 * max(1.0, abs(m0[cc]))
    print(f"[fp32-increments] rel L2 vs FP64 oracle: increments {errs[K.FP32_INCREMENTS]:.2e}, "
          f"bulk {errs[K.FP32_MIXED]:.2e}", flush=True)
    assert errs[K.FP32_INCREMENTS] < 2e-7 and errs[K.FP32_MIXED] < 2e-7


def test_fp32_increments_shock_step_and_limiter(K):
    """one step of the shock workload (128 x 32, Dirichlet inflow) in the
    FP32-increments form against the FP64 oracle, then the FP64 limiter"""
    import torch
    cfg = W.config("c5", scale=32)
    params, xi = W.shock_problem(2000, cfg["nx"], cfg["ny"])
    ghost = W.post_shock_conserved(params[0])
    x0, x1, y0, y1 = cfg["box"]
    lm = K.make_mesh(2, cfg["nx"], cfg["ny"], x0=x0, x1=x1, y0=y0, y1=y1, bc=(2, 1, 1, 1),
                     bc_state=[ghost] * 4, equation=K.EQ_EULER, precision=K.FP32_INCREMENTS)
    om = O.Mesh(2, cfg["nx"], cfg["ny"], x0=x0, x1=x1, y0=y0, y1=y1, bc=(2, 1, 1, 1),
                bc_state=[ghost] * 4, equation=O.EQ_EULER, flux=O.FLUX_LLF)
    s = K.Solver(lm, 2, K.FLUX_LLF, 3)
    s.crkdg_project(K.IC_SHOCK, params, aux=torch.from_numpy(xi).cuda())
    s.crkdg_limit(50.0)
    u = s.crkdg_get_state()
    dt = cfg["cfl"] / O.max_wavespeed(om, 2, u)
    s.crkdg_step(dt)
    A, b, c = (np.array(v, float) for v in W.TABLEAU["eq3"])
    ref = O.step_crkdg(om, 2, (A, b, c), 0.0, dt, u)
    got = s.crkdg_get_state()
    err = l2_rel(got, ref)
    print(f"[fp32-increments] shock step rel L2 {err:.2e}", flush=True)
    assert err < 1e-7
    flags = torch.zeros(om.ncells, dtype=torch.uint8, device="cuda")
    s.crkdg_limit(50.0, flags)
    lim_o, fl_o, _ = O.limit_tvb(om, 2, 50.0, got)
    _, margin, _ = O.tvb_flags(om, 2, 50.0, got)
    fg = flags.cpu().numpy()
    safe = margin > 1e-9
    assert np.array_equal(fg[safe], fl_o[safe])
    agree = fg == fl_o
    assert rel_err(s.crkdg_get_state()[:, :, agree], lim_o[:, :, agree]) < 1e-13


def test_mixed_shock_step_and_limiter(K):
    cfg = W.config("c5", scale=32)  # 128 x 32
    params, xi = W.shock_problem(2000, cfg["nx"], cfg["ny"])
    ghost = W.post_shock_conserved(params[0])
    import torch
    s, om = mixed_solver(K, cfg, 2, 3, bc_state=[ghost] * 4)
    s.crkdg_project(K.IC_SHOCK, params, aux=torch.from_numpy(xi).cuda())
    s.crkdg_limit(50.0)
    u = s.crkdg_get_state()        # the FP32-bulk state, as FP64
    dt = cfg["cfl"] / O.max_wavespeed(om, 2, u)
    s.crkdg_step(dt)
    A, b, c = (np.array(v, float) for v in W.TABLEAU["eq3"])
    ref = O.step_crkdg(om, 2, (A, b, c), 0.0, dt, u)
    got = s.crkdg_get_state()
    assert l2_rel(got, ref) < 1e-6
    # limiter: FP64 test on the FP32-bulk state; compare where decisions are safe
    flags = torch.zeros(om.ncells, dtype=torch.uint8, device="cuda")
    s.crkdg_limit(50.0, flags)
    lim_o, fl_o, _ = O.limit_tvb(om, 2, 50.0, got)
    _, margin, _ = O.tvb_flags(om, 2, 50.0, got)
    fg = flags.cpu().numpy()
    safe = margin > 1e-7
    assert np.array_equal(fg[safe] != 0, fl_o[safe] != 0)
    after = s.crkdg_get_state()
    agree = fg == fl_o
    assert l2_rel(after[:, :, agree], lim_o[:, :, agree]) < 1e-6


# --- errors against a restricted finer reference ------------------------------

@pytest.mark.parametrize("r,ry,kc,kf", [(2, 2, 2, 2), (3, 2, 2, 1), (1, 1, 3, 0)])
def test_error_against_restricted_reference(K, r, ry, kc, kf):
    """L1/L2/Linf of the cell averages against the r x ry block means of a
    finer state equal the oracle's averaged-error routine on the same data
    (diagnostic of the error tables of Section 4)"""
    nx, ny = 37, 13
    box = (0.0, 2.0, -1.0, 0.5)
    omc, lmc = meshes(K, 2, nx, ny, "euler", box=box)
    omf, lmf = meshes(K, 2, r * nx, ry * ny, "euler", box=box)
    sc, sf = solver(K, lmc, kc, "llf"), solver(K, lmf, kf, "llf")
    uc = random_state("euler", omc.shape(kc), 5)
    uf = random_state("euler", omf.shape(kf), 6)
    sc.crkdg_set_state(uc)
    sf.crkdg_set_state(uf)
    for comp in (0, 3):
        fine = uf[comp, 0].reshape(ry * ny, r * nx)
        ref = fine.reshape(ny, ry, nx, r).mean(axis=(1, 3)).reshape(-1)
        want = O.errors_vs_avg(omc, kc, uc, ref, comp=comp)
        got = sc.crkdg_error_ref(sf, comp)
        assert np.allclose(got, want, rtol=1e-12, atol=0.0), (got, want)
    # mismatched meshes are rejected
    omb, lmb = meshes(K, 2, 2 * nx + 1, ny, "euler", box=box)
    sb = solver(K, lmb, 1, "llf")
    with pytest.raises(K.CrkdgError):
        sc.crkdg_error_ref(sb, 0)


def test_limit_dt_equals_limit_then_compute_dt(K):
    """the fused limiter + next-step dt gives bitwise the state, flags and dt
    of crkdg_limit followed by crkdg_compute_dt (TVB and learned modes)"""
    import torch
    cfg = W.config("c5", scale=32)  # 128 x 32, boundary tiles and a ragged last block
    params, xi = W.shock_problem(2001, cfg["nx"], cfg["ny"])
    ghost = W.post_shock_conserved(params[0])
    rng = np.random.default_rng(4)
    P = torch.from_numpy((0.4 * rng.standard_normal(O.N_MLP_PARAMS)).astype(np.float32)).cuda()
    for precision in (K.FP64, K.FP32_MIXED):
        for mlp in (False, True):
            out = []
            for fused in (False, True):
                x0, x1, y0, y1 = cfg["box"]
                lm = K.make_mesh(2, cfg["nx"] - 3, cfg["ny"], x0=x0, x1=x1, y0=y0, y1=y1,
                                 bc=(2, 1, 1, 1), bc_state=[ghost] * 4, equation=K.EQ_EULER,
                                 precision=precision)
                s = K.Solver(lm, 2, K.FLUX_LLF, 3)
                p2, xi2 = W.shock_problem(2001, cfg["nx"] - 3, cfg["ny"])
                s.crkdg_project(K.IC_SHOCK, p2, aux=torch.from_numpy(xi2).cuda())
                s.crkdg_limit(50.0)
                s.crkdg_step(0.1 / s.crkdg_max_wavespeed())
                flags = torch.zeros(s.ncells, dtype=torch.uint8, device="cuda")
                dt = torch.zeros(1, dtype=torch.float64, device="cuda")
                if fused:
                    s.crkdg_limit_dt(50.0, 0.1, dt, flags, params=P if mlp else None,
                                     tau_lo=0.3, tau_hi=0.7)
                else:
                    if mlp:
                        s.crkdg_limit_mlp(50.0, P, 0.3, 0.7, flags, count=False)
                    else:
                        s.crkdg_limit(50.0, flags, count=False)
                    s.crkdg_compute_dt(0.1, dt)
                out.append((s.crkdg_get_state(), flags.cpu().numpy(), dt.item()))
            assert np.array_equal(out[0][0], out[1][0])
            assert np.array_equal(out[0][1], out[1][1])
            assert out[0][2] == out[1][2] and out[0][2] > 0.0
