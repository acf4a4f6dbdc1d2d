"""Pins of the oracle's double Mach reflection (Section 4, example "Double
Mach reflection": a Mach 10 shock at 60 degrees to a reflecting wall that
starts at x = 1/6; the paper leaves the states to the classical test).

- the post-shock state satisfies the Rankine--Hugoniot conditions across the
  moving shock (mass, normal and tangential momentum, energy);
- the exact solution puts the shock where a line through (1/6, 0) at 60
  degrees, moved with the shock speed along its normal, lies at time t;
- the reflecting wall is a symmetry plane: the DG operator and the TVB
  decisions next to it equal those of the mirrored problem on a mesh twice
  as tall, where the wall is an interior face.
"""
import math

import numpy as np
import pytest

import oracle as O
from paper_2307_06471_amd import workloads as W

G = 1.4


def prim(q, g=G):
    r = q[0]
    u, v = q[1] / r, q[2] / r
    return r, u, v, (g - 1.0) * (q[3] - 0.5 * r * (u * u + v * v))


def test_rankine_hugoniot_across_the_moving_shock():
    pre, post, S = O.dmr_states(G)
    r1, u1, v1, p1 = prim(pre)
    r2, u2, v2, p2 = prim(post)
    assert (r1, u1, v1, p1) == pytest.approx((1.4, 0.0, 0.0, 1.0), abs=1e-14)
    assert S == pytest.approx(10.0 * math.sqrt(G * p1 / r1), rel=1e-15)  # Mach 10
    n = np.array([math.sin(math.pi / 3), -math.cos(math.pi / 3)])  # into the gas at rest
    tang = np.array([-n[1], n[0]])
    un1, un2 = 0.0, u2 * n[0] + v2 * n[1]
    E1, E2 = pre[3], post[3]
    scale = r2 * S * S
    # fluxes through the moving shock: F(q) - S q along the normal
    assert r1 * (un1 - S) == pytest.approx(r2 * (un2 - S), rel=1e-13)
    assert r1 * un1 * (un1 - S) + p1 == pytest.approx(r2 * un2 * (un2 - S) + p2, rel=1e-13)
    assert E1 * (un1 - S) + p1 * un1 == pytest.approx(E2 * (un2 - S) + p2 * un2,
                                                      abs=1e-13 * scale * S)
    assert abs(u2 * tang[0] + v2 * tang[1]) < 1e-13 * S  # no tangential jump
    assert r2 > r1 and p2 > p1 and un2 > 0  # compressive, gas pushed along the normal
    # it is a shock of the right strength: entropy rises
    assert math.log(p2 / r2 ** G) > math.log(p1 / r1 ** G)


@pytest.mark.parametrize("t", [0.0, 0.01, 0.03])
def test_exact_shock_position(t):
    """project the exact solution on a fine strip along the top side and find
    the column where the density switches from post- to pre-shock"""
    nx = 800
    m = O.Mesh(2, nx, 1, x0=0.0, x1=4.0, y0=1.0 - 1e-3, y1=1.0, equation=O.EQ_EULER, gamma=G,
               flux=O.FLUX_LLF)
    u = O.project(m, 0, O.IC_DMR, t=t)
    rho = u[0, 0]
    _, post, S = O.dmr_states(G)
    behind = np.nonzero(np.abs(rho - post[0]) < 1e-12)[0]
    x_switch = 4.0 * (behind.max() + 1) / nx
    y = 1.0 - 0.5e-3
    x_line = 1.0 / 6.0 + (y + 2.0 * S * t) / math.sqrt(3.0)  # normal speed S, horizontal 2S/sqrt3
    assert abs(x_switch - x_line) <= 4.0 / nx


def wall_and_mirror(nx, ny, k, seed):
    """a state over [0.5, 1.5] x [0, 1] (reflecting wall below, since x >= 1/6
    everywhere) and the same state mirrored into [0.5, 1.5] x [-1, 0]"""
    nb = (k + 1) ** 2
    u = W.random_euler_modes(np.random.default_rng(seed), nb, nx * ny)
    wall = O.Mesh(2, nx, ny, x0=0.5, x1=1.5, y0=0.0, y1=1.0, bc=(0, 0, 2, 1),
                  bc_exact=O.IC_DMR, equation=O.EQ_EULER, gamma=G, flux=O.FLUX_LLF)
    twice = O.Mesh(2, nx, 2 * ny, x0=0.5, x1=1.5, y0=-1.0, y1=1.0, bc=(0, 0, 1, 1),
                   equation=O.EQ_EULER, gamma=G, flux=O.FLUX_LLF)
    q = u.reshape(4, nb, ny, nx)
    n_of = np.array([b // (k + 1) for b in range(nb)])
    sign = (-1.0) ** n_of  # P_n(-eta) = (-1)^n P_n(eta)
    mir = q[:, :, ::-1, :] * sign[None, :, None, None]
    mir[2] *= -1.0  # the mirrored momentum normal to the wall
    big = np.concatenate([mir, q], axis=2).reshape(4, nb, 2 * ny * nx)
    return wall, twice, u, big


@pytest.mark.parametrize("k", [1, 2])
def test_reflecting_wall_is_a_symmetry_plane(k):
    nx, ny = 12, 7
    wall, twice, u, big = wall_and_mirror(nx, ny, k, 3 + k)
    a = O.apply(wall, k, O.OP_DG, u)
    b = O.apply(twice, k, O.OP_DG, big)[:, :, ny * nx:]
    assert np.abs(a - b).max() < 1e-12 * np.abs(b).max()


def test_limiter_ghost_at_the_wall_is_the_mirror_cell():
    k, nx, ny = 2, 12, 7
    wall, twice, u, big = wall_and_mirror(nx, ny, k, 11)
    for M in (0.0, 20.0):
        fa, ma, _ = O.tvb_flags(wall, k, M, u, t=0.01)
        fb, mb, _ = O.tvb_flags(twice, k, M, big)
        assert np.array_equal(fa, fb[ny * nx:])
        assert np.allclose(ma, mb[ny * nx:], rtol=1e-12, atol=1e-300)


def test_inflow_and_top_ghosts_follow_the_exact_shock():
    """one DG operator application on a small mesh over the whole problem
    (piecewise constants: the projected Mach 10 jump at higher degree
    undershoots to negative pressure and needs the limiter first): the left
    column's operator equals that of a mesh whose left ghost is the
    post-shock state"""
    k, nx, ny = 0, 16, 4
    t = 0.0
    m = O.Mesh(2, nx, ny, x0=0.0, x1=4.0, y0=0.0, y1=1.0, bc=(2, 1, 2, 2), bc_exact=O.IC_DMR,
               equation=O.EQ_EULER, gamma=G, flux=O.FLUX_LLF)
    _, post, _ = O.dmr_states(G)
    m2 = O.Mesh(2, nx, ny, x0=0.0, x1=4.0, y0=0.0, y1=1.0, bc=(2, 1, 2, 2),
                bc_state=[list(post)] * 4, equation=O.EQ_EULER, gamma=G, flux=O.FLUX_LLF)
    u = O.project(m, k, O.IC_DMR, t=t)
    a = O.apply(m, k, O.OP_DG, u, t_bc=t)
    b = O.apply(m2, k, O.OP_DG, u, t_bc=t)
    assert np.isfinite(a).all() and np.isfinite(b).all()
    left = np.arange(ny) * nx  # the left column: its left ghost is post-shock in both
    rows = left[1:-1]  # not touching the bottom (wall) or top (moving shock) sides
    assert np.abs(a[:, :, rows] - b[:, :, rows]).max() < 1e-12 * np.abs(b).max()
    # along the top, ahead of the shock the exact solution is the pre-shock state:
    # the top-right cell's operator equals that with a pre-shock top ghost
    pre, _, _ = O.dmr_states(G)
    m3 = O.Mesh(2, nx, ny, x0=0.0, x1=4.0, y0=0.0, y1=1.0, bc=(2, 1, 2, 2),
                bc_state=[list(post), list(pre), list(post), list(pre)], equation=O.EQ_EULER,
                gamma=G, flux=O.FLUX_LLF)
    c = O.apply(m3, k, O.OP_DG, u, t_bc=t)
    tr = ny * nx - 1
    assert np.abs(a[:, :, tr] - c[:, :, tr]).max() < 1e-12 * np.abs(c).max()
