"""Pins of the oracle against numbers the paper prints.

- Table 'tab:CFL' (Section 1): maximum CFL of cRKDG and RKDG, upwind flux,
  reproduced by von Neumann analysis of the oracle's own operators.
- Table 'table:boundary_treatment' (Section 4.1.1, Example 'ex:1derror'):
  1D P^2 advection errors, periodic and inflow boundaries.
- Table 'table:euler accuracy' and Table 'table:ssprk2-wrong_scheme'
  (Section 4.1.1, Example 'ex:1dremark'): 1D Euler accuracy and the
  Shu--Osher-substitution negative test.
- Table 'table:2deuler-periodic-rectangle' (Section 4.1.2): convergence order.
- Example 'ex:shuosher' (Section 4.2.1): the printed left state is the
  Mach-3 Rankine--Hugoniot post-shock state.

Readings: fixed dt stepped while it fits (last time level t_n <= T, errors
against the exact solution at t_n); unnormalised L2 over the domain with a
(k+3)-point Gauss rule; Linf at the same points.
"""
import json
import math
import os

import numpy as np
import pytest

import oracle as O
from tests import fourier as F
from tests.tableaus import EQ2, EQ3, FE, RK4, RK38, SSP2, SSP3

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def gold(name):
    with open(os.path.join(GOLD, name)) as f:
        return json.load(f)


# --- von Neumann: the oracle's operators are the analysed ones ----------

@pytest.mark.parametrize("k", [0, 1, 2, 3])
def test_oracle_1d_operators_are_the_fourier_blocks(k):
    N, h = 8, 0.25
    mesh = O.Mesh(1, N, x0=0, x1=N * h, equation=O.EQ_ADVECTION, flux=O.FLUX_UPWIND, adv=(1.0, 0))
    B0, B1, Bloc = F.blocks(k)
    nb = k + 1
    for op, blocks in ((O.OP_DG, (B0, B1)), (O.OP_LOC, (Bloc, 0 * Bloc))):
        M = np.zeros((nb * N, nb * N))
        for col in range(nb * N):
            e = np.zeros((1, nb, N))
            e[0, col % nb, col // nb] = 1.0
            M[:, col] = (h * O.apply(mesh, k, op, e))[0].T.ravel()
        for j in range(N):
            assert np.allclose(M[j * nb:(j + 1) * nb, j * nb:(j + 1) * nb], blocks[0], atol=1e-12)
            jm = (j - 1) % N
            assert np.allclose(M[j * nb:(j + 1) * nb, jm * nb:(jm + 1) * nb], blocks[1], atol=1e-12)


@pytest.mark.slow
def test_max_cfl_table():
    """Three of the four printed entries reproduce to the printed digits.
    The third-order cRKDG entry (0.178) does not: the scheme (eq:3) with the
    upwind flux and P^2 has its limit at 0.1708, set by the theta = pi mode
    (confirmed by direct time stepping in test_third_order_limit_by_time_stepping).
    The paper's own P^2 experiments use CFL 0.16, inside both values."""
    g = gold("tab_cfl.json")
    got = {
        ("crkdg", "2"): F.max_cfl(1, EQ2, "crkdg"),
        ("crkdg", "3"): F.max_cfl(2, EQ3, "crkdg"),
        ("rkdg", "2"): F.max_cfl(1, SSP2, "rkdg"),
        ("rkdg", "3"): F.max_cfl(2, SSP3, "rkdg"),
    }
    # a stability limit is printed rounded down (0.20975 appears as 0.209)
    for key in (("crkdg", "2"), ("rkdg", "2"), ("rkdg", "3")):
        assert math.floor(got[key] * 1000) / 1000 == pytest.approx(g[key[0]][key[1]], abs=1e-9), \
            (key, got[key])
    c3 = got[("crkdg", "3")]
    assert 0.16 < c3 < g["crkdg"]["3"] and math.floor(c3 * 1000) == 170
    # tableau independence of the cRKDG limit among p-stage p-th order methods
    assert abs(F.max_cfl(2, SSP3, "crkdg") - c3) < 1e-4


@pytest.mark.parametrize("nu,stable", [(0.170, True), (0.172, False)])
def test_third_order_limit_by_time_stepping(nu, stable):
    N, k = 32, 2
    mesh = O.Mesh(1, N, x0=0, x1=1, equation=O.EQ_ADVECTION, flux=O.FLUX_UPWIND, adv=(1.0, 0))
    u = np.random.default_rng(0).standard_normal(mesh.shape(k))
    n0 = np.abs(u).max()
    for _ in range(3000):
        u = O.step_crkdg(mesh, k, EQ3, 0.0, nu / N, u)
    growth = np.abs(u).max() / n0
    assert (growth < 1.0) if stable else (growth > 1e3)


def test_c1_exact_discrete_answer():
    """64 cells on [0, 2pi], P^2, SSP-RK3 Butcher cRKDG, dt = 0.1 h, 640 steps:
    the oracle equals the block-circulant closed form (DFT + G^n)"""
    N, k = 64, 2
    h = 2 * np.pi / N
    mesh = O.Mesh(1, N, x0=0, x1=2 * np.pi, equation=O.EQ_ADVECTION, flux=O.FLUX_UPWIND,
                  adv=(1.0, 0))
    u0 = O.project(mesh, k, O.IC_ADV_SIN)
    u = u0.copy()
    dt = 0.1 * h
    for n in range(640):
        u = O.step_crkdg(mesh, k, SSP3, n * dt, dt, u)
    ref = F.evolve_periodic(k, u0[0], 0.1, SSP3, 640)
    assert np.abs(u[0] - ref).max() < 1e-12
    # and it is close to the exact solution sin(x - 2 pi) = sin(x)
    e = O.errors(mesh, k, u, O.IC_ADV_SIN, t=640 * dt)
    assert e[2] < 1e-4


# --- Table 'table:boundary_treatment' -------------------------------------

def _run_adv1d(N, scheme, inflow):
    k, L, T = 2, 4 * np.pi, 20.0
    h = L / N
    dt = 0.16 * h
    bc = (O.BC_DIRICHLET, O.BC_TRANSMISSIVE, 0, 0) if inflow else (0, 0, 0, 0)
    mesh = O.Mesh(1, N, x0=0, x1=L, bc=bc, bc_exact=O.IC_ADV_SIN if inflow else 0,
                  equation=O.EQ_ADVECTION, flux=O.FLUX_UPWIND, adv=(1.0, 0))
    u = O.project(mesh, k, O.IC_ADV_SIN)
    n = math.floor(T / dt)
    for i in range(n):
        if scheme == "crkdg":
            u = O.step_crkdg(mesh, k, EQ3, i * dt, dt, u)
        else:
            u = O.step_rkdg_ssp(mesh, k, 3, i * dt, dt, u)
    return O.errors(mesh, k, u, O.IC_ADV_SIN, t=n * dt)


@pytest.mark.parametrize("inflow", [False, True])
def test_boundary_treatment_crkdg(inflow):
    g = gold("boundary_treatment.json")
    tag = "inflow" if inflow else "periodic"
    l2s = []
    for idx, N in enumerate(g["N"][:4]):
        e = _run_adv1d(N, "crkdg", inflow)
        l2s.append(e[1])
        assert e[1] == pytest.approx(g[f"crkdg_{tag}_L2"][idx], rel=1e-2), (N, e)
        assert e[2] == pytest.approx(g[f"crkdg_{tag}_Linf"][idx], rel=1e-2), (N, e)
    orders = np.log2(np.array(l2s[:-1]) / np.array(l2s[1:]))
    assert np.all(np.abs(orders - 3.0) < 0.03)


def test_boundary_treatment_rkdg_orders():
    """comparison scheme: optimal order with periodic data, reduced Linf order
    with exact inflow data at the inner stages (Section 3.4)"""
    per = [_run_adv1d(N, "rkdg", False) for N in (80, 160, 320)]
    inf = [_run_adv1d(N, "rkdg", True) for N in (80, 160, 320)]
    op = np.log2(per[0][1] / per[1][1]), np.log2(per[1][1] / per[2][1])
    oi = np.log2(inf[1][2] / inf[2][2])
    assert all(abs(o - 3.0) < 0.05 for o in op)
    assert oi < 2.5  # degenerate inflow Linf order
    g = gold("boundary_treatment.json")
    assert per[0][1] == pytest.approx(g["rkdg_periodic_L2"][1], rel=0.06)


# --- 1D Euler tables -------------------------------------------------------

def _run_euler1d(N, k, cfl, step):
    mesh = O.Mesh(1, N, x0=0, x1=2, equation=O.EQ_EULER, flux=O.FLUX_LLF)
    P = [1.0, 0.0, 1.0]
    u = O.project(mesh, k, O.IC_EULER_WAVE, P)
    h, T, t = 2.0 / N, 2.0, 0.0
    while t < T - 1e-13:
        dt = min(cfl / O.max_wavespeed(mesh, k, u), T - t)
        u = step(mesh, k, t, dt, u)
        t += dt
    return O.errors(mesh, k, u, O.IC_EULER_WAVE, P, t=T)


def test_euler1d_accuracy_table():
    g = gold("euler1d_accuracy.json")
    e1 = [_run_euler1d(N, 1, 0.3, lambda m, k, t, dt, u: O.step_crkdg(m, k, EQ2, t, dt, u))
          for N in g["N"][:3]]
    e2 = [_run_euler1d(N, 2, 0.16, lambda m, k, t, dt, u: O.step_crkdg(m, k, EQ3, t, dt, u))
          for N in g["N"][:3]]
    for i in range(3):
        assert e1[i][1] == pytest.approx(g["k1_L2"][i], rel=0.05)
        assert e2[i][1] == pytest.approx(g["k2_L2"][i], rel=0.05)
    assert abs(np.log2(e1[1][1] / e1[2][1]) - 2.0) < 0.1
    assert abs(np.log2(e2[1][1] / e2[2][1]) - 3.0) < 0.1


def test_shu_osher_substitution_is_first_order():
    g = gold("ssprk2_wrong.json")
    wr = [_run_euler1d(N, 1, 0.1, lambda m, k, t, dt, u: O.step_wrong_ssp(m, k, 2, t, dt, u))
          for N in g["N"]]
    ok = [_run_euler1d(N, 1, 0.1, lambda m, k, t, dt, u: O.step_crkdg(m, k, SSP2, t, dt, u))
          for N in g["N"]]
    for i in range(3):
        assert wr[i][1] == pytest.approx(g["wrong_k1_L2"][i], rel=0.02)
        assert ok[i][1] == pytest.approx(g["correct_k1_L2"][i], rel=0.06)
    assert abs(np.log2(wr[1][1] / wr[2][1]) - 1.0) < 0.1
    assert abs(np.log2(ok[1][1] / ok[2][1]) - 2.0) < 0.1
    wr3 = [_run_euler1d(N, 2, 0.1, lambda m, k, t, dt, u: O.step_wrong_ssp(m, k, 3, t, dt, u))
           for N in g["N"]]
    ok3 = [_run_euler1d(N, 2, 0.1, lambda m, k, t, dt, u: O.step_crkdg(m, k, SSP3, t, dt, u))
           for N in g["N"]]
    for i in range(3):
        assert wr3[i][1] == pytest.approx(g["wrong_k2_L2"][i], rel=0.15)
        assert ok3[i][1] == pytest.approx(g["correct_k2_L2"][i], rel=0.06)
    assert np.log2(wr3[1][1] / wr3[2][1]) < 2.2          # sub-optimal
    assert abs(np.log2(ok3[1][1] / ok3[2][1]) - 3.0) < 0.1  # optimal


# --- 2D Euler order (rectangular meshes, Q^k) -------------------------------

def _run_euler2d_wave(N, k, cfl, tab, T=0.5):
    mesh = O.Mesh(2, N, N, x0=0, x1=2, y0=0, y1=2, equation=O.EQ_EULER, flux=O.FLUX_LLF)
    P = [0.7, 0.3, 1.0]
    u = O.project(mesh, k, O.IC_EULER_WAVE, P)
    t = 0.0
    while t < T - 1e-13:
        dt = min(cfl / O.max_wavespeed(mesh, k, u), T - t)
        u = O.step_crkdg(mesh, k, tab, t, dt, u)
        t += dt
    return O.errors(mesh, k, u, O.IC_EULER_WAVE, P, t=T)


@pytest.mark.slow
def test_euler2d_density_wave_order():
    # orders measured: 2.65 (10->20), 2.81 (20->40), 2.92 (40->80): approaching 3
    e = [_run_euler2d_wave(N, 2, 0.12, EQ3)[1] for N in (10, 20, 40)]
    o1, o2 = np.log2(e[0] / e[1]), np.log2(e[1] / e[2])
    assert 2.6 < o1 < o2 < 3.1, e
    g = gold("euler2d_rect.json")
    # Q^2 versus the paper's P^2: same order, magnitude within a small factor
    assert g["crkdg_k2_L2"][0] / 4 < e[1] < 4 * g["crkdg_k2_L2"][0]


@pytest.mark.slow
def test_euler2d_q3_rk4_order():
    e = [_run_euler2d_wave(N, 3, 0.05, RK4, T=0.2)[1] for N in (6, 12, 24)]
    assert abs(np.log2(e[1] / e[2]) - 4.0) < 0.3, e


# --- the printed Shu--Osher left state is the Mach-3 RH state ---------------

def test_rankine_hugoniot_state():
    g = gold("shu_osher_state.json")
    M, gam = g["mach"], g["gamma"]
    rho2 = (gam + 1) * M**2 / ((gam - 1) * M**2 + 2)
    p2 = (2 * gam * M**2 - (gam - 1)) / (gam + 1)
    S = M * math.sqrt(gam)
    u2 = S * (1 - 1 / rho2)
    assert [round(rho2, 6), round(u2, 6), round(p2, 6)] == g["left_state"]


# --- Example 'ex:2dadv' (Table 'table:2dlinear-dirichlet') on rectangles ----

def _run_adv2d(N, scheme, inflow):
    """u_t + u_x + u_y = 0 on [-1, 1]^2, u0 = sin(pi x) sin(pi y), upwind
    flux, k = 3 with classical RK4 (Section 4), to t = 0.4 with
    dt = h/30 (cRKDG) or h/20 (RKDG) as in the table; inflow: the exact
    solution on the left and bottom sides at the stage times, outflow
    (transmissive) on the right and top.  The paper uses P^3 on triangles;
    this is the Q^3 analogue on N x N rectangles."""
    from tests.tableaus import RK4
    bc = (2, 1, 2, 1) if inflow else (0, 0, 0, 0)
    m = O.Mesh(2, N, N, x0=-1, x1=1, y0=-1, y1=1, bc=bc,
               bc_exact=O.IC_ADV_SIN if inflow else 0, equation=O.EQ_ADVECTION,
               adv=(1.0, 1.0), flux=O.FLUX_UPWIND)
    u = O.project(m, 3, O.IC_ADV_SIN)
    n = round(0.4 / ((2.0 / N) / (30 if scheme == "crkdg" else 20)))
    dt = 0.4 / n
    step = O.step_crkdg if scheme == "crkdg" else O.step_rkdg
    for i in range(n):
        u = step(m, 3, RK4, i * dt, dt, u)
    return O.errors(m, 3, u, O.IC_ADV_SIN, t=0.4)


def test_2d_inflow_keeps_the_order_of_crkdg_only():
    """with inflow data cRKDG stays fourth order in L2 and Linf; RKDG, whose
    inner stages see the exact boundary data, drops in Linf (the paper's
    table: about 2; here 2.9 already from N = 16 to 32, 2.2 from 32 to 64)"""
    c = [_run_adv2d(N, "crkdg", True) for N in (16, 32)]
    r = [_run_adv2d(N, "rkdg", True) for N in (16, 32)]
    oc2, oci = np.log2(c[0][1] / c[1][1]), np.log2(c[0][2] / c[1][2])
    ori = np.log2(r[0][2] / r[1][2])
    assert abs(oc2 - 4.0) < 0.15 and abs(oci - 4.0) < 0.15, (oc2, oci)
    assert ori < 3.3, ori
    assert c[1][2] < 0.5 * r[1][2]
    # periodic data: both optimal
    p = [_run_adv2d(N, "rkdg", False) for N in (16, 32)]
    assert abs(np.log2(p[0][1] / p[1][1]) - 4.0) < 0.15
