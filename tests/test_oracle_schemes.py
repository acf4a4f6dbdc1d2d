"""Pins of the oracle's time stepping against invariants and closed forms.

- conservation of the summed cell averages (Section 3.2.2, equations (avg)
  and (g)); the inner stages alone do not conserve (Section 3.2.2);
- P^0: the local operator vanishes (Section 3.3), so cRKDG is the
  forward-Euler finite-volume scheme for any tableau with sum(b) = 1;
- s = 1: cRKDG and RKDG coincide (equations (rkdg) and (crkdg));
- linear constant-coefficient problems: every p-stage p-th order tableau
  gives the closed form (linear) of Section 3.5.1, theorem 'equivalence'.
"""
import numpy as np
import pytest

import oracle as O
from tests.tableaus import EQ2, EQ3, FE, RK4, RK38, SSP2, SSP3


def vortex_mesh(n, k):
    mesh = O.Mesh(2, n, n, x0=0, x1=10, y0=0, y1=10, equation=O.EQ_EULER, flux=O.FLUX_LLF)
    u = O.project(mesh, k, O.IC_VORTEX, [5.0, 5.0, 5.0, 10.0, 10.0])
    return mesh, u


@pytest.mark.parametrize("tab,k", [(EQ3, 2), (RK4, 3), (EQ2, 1), (SSP3, 2)])
def test_conservation_periodic_euler(tab, k):
    mesh, u = vortex_mesh(8, k)
    m0 = [O.total_mass(mesh, k, u, c) for c in range(4)]
    for n in range(10):
        u = O.step_crkdg(mesh, k, tab, n * 0.01, 0.01, u)
    for c in range(4):
        m1 = O.total_mass(mesh, k, u, c)
        assert abs(m1 - m0[c]) <= 1e-13 * max(1.0, abs(m0[c])), (c, m1 - m0[c])


def test_inner_stage_alone_is_not_conservative():
    mesh, u = vortex_mesh(8, 2)
    st = O.crkdg_stages(mesh, 2, EQ3, 0.0, 0.05, u)
    drift = max(abs(O.total_mass(mesh, 2, st[2], c) - O.total_mass(mesh, 2, u, c))
                for c in range(4))
    assert drift > 1e-8


@pytest.mark.parametrize("tab", [EQ2, EQ3, RK4, SSP3])
def test_k0_is_forward_euler_finite_volume(tab):
    mesh = O.Mesh(2, 6, 5, x0=0, x1=1, y0=0, y1=1, bc=(1, 1, 0, 0), equation=O.EQ_EULER,
                  flux=O.FLUX_LLF)
    u = O.project(mesh, 0, O.IC_QUADRANT,
                  [0.5, 0.5, 1.0, 0.1, 0.0, 1.0, 0.5, -0.2, 0.3, 0.4, 0.125, 0.0, 0.0, 0.1,
                   0.7, 0.3, -0.3, 0.9])
    a = O.step_crkdg(mesh, 0, tab, 0.0, 0.01, u)
    b = O.step_rkdg(mesh, 0, FE, 0.0, 0.01, u)
    assert np.abs(a - b).max() <= 1e-15 * np.abs(b).max()


@pytest.mark.parametrize("k", [1, 2, 3])
def test_one_stage_crkdg_is_rkdg(k):
    mesh, u = vortex_mesh(6, k)
    a = O.step_crkdg(mesh, k, FE, 0.0, 0.01, u)
    b = O.step_rkdg(mesh, k, FE, 0.0, 0.01, u)
    assert np.array_equal(a, b)


def _closed_form(mesh, k, p, dt, u):
    """u - dt DG( sum_{i<p} dt^i/(i+1)! L^i u ),  L = -loc"""
    acc = u.copy()
    term = u.copy()
    fact = 1.0
    for i in range(1, p):
        term = -dt * O.apply(mesh, k, O.OP_LOC, term)
        fact *= (i + 1)
        acc = acc + term / fact
    return u - dt * O.apply(mesh, k, O.OP_DG, acc)


@pytest.mark.parametrize("dim", [1, 2])
@pytest.mark.parametrize("tabs,k", [((EQ3, SSP3), 2), ((RK4, RK38), 3), ((EQ2, SSP2), 1)])
def test_linear_tableau_independence_and_closed_form(dim, tabs, k):
    rng = np.random.default_rng(7)
    mesh = O.Mesh(dim, 7, 5, x0=0, x1=1, y0=0, y1=1, equation=O.EQ_ADVECTION,
                  flux=O.FLUX_UPWIND, adv=(0.9, -0.6))
    u = rng.standard_normal(mesh.shape(k))
    dt = 0.01
    a = O.step_crkdg(mesh, k, tabs[0], 0.0, dt, u)
    b = O.step_crkdg(mesh, k, tabs[1], 0.0, dt, u)
    c = _closed_form(mesh, k, len(tabs[0][1]), dt, u)
    scale = np.abs(u).max()
    assert np.abs(a - b).max() < 1e-13 * scale
    assert np.abs(a - c).max() < 1e-13 * scale


def test_c1_ssp3_and_eq3_agree_over_a_run():
    """64 cells, P^2, 640 steps: the two 3-stage tableaus agree (linear case)"""
    N, k = 64, 2
    h = 2 * np.pi / N
    mesh = O.Mesh(1, N, x0=0, x1=2 * np.pi, equation=O.EQ_ADVECTION, flux=O.FLUX_UPWIND,
                  adv=(1.0, 0))
    u = O.project(mesh, k, O.IC_ADV_SIN)
    a, b = u.copy(), u.copy()
    for n in range(640):
        a = O.step_crkdg(mesh, k, SSP3, n * 0.1 * h, 0.1 * h, a)
        b = O.step_crkdg(mesh, k, EQ3, n * 0.1 * h, 0.1 * h, b)
    assert np.abs(a - b).max() < 1e-12


def test_vortex_error_small():
    """the vortex translates with unit velocity; after t=0.5 the FP64 cRKDG
    solution on 32^2 cells is close to the exact translated vortex"""
    mesh, u = vortex_mesh(32, 2)
    dt = 0.1 / O.max_wavespeed(mesh, 2, u)
    t = 0.0
    while t < 0.5 - 1e-12:
        d = min(dt, 0.5 - t)
        u = O.step_crkdg(mesh, 2, EQ3, t, d, u)
        t += d
    e = O.errors(mesh, 2, u, O.IC_VORTEX, [5.0, 5.0, 5.0, 10.0, 10.0], t=0.5)
    assert e[2] < 5e-3
