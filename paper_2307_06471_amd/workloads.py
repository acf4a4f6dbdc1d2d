"""Seeded synthetic workloads (input generators only).

This module holds no arithmetic of the method: it defines mesh sizes,
boundary conditions, tableau choices, CFL numbers and final times, draws the
seeded random parameters of the shock problems and the smoothed noise field,
and nothing else.  Initial conditions are projected by the library (product
path) or by the oracle (tests), each with its own code.

Workloads (all inputs are synthetic; the paper's examples are analytic PDE
problems, so no dataset is involved):
  c1  1D u_t + u_x = 0 on [0, 2 pi], periodic, 64 cells, P^2, SSP-RK3 in Butcher
      form, upwind flux, u0 = sin x, dt = 0.1 h, 640 steps to T = 2 pi
      (shape of the paper's 1D advection example, Section 4.1.1);
  c2  2D Euler isentropic vortex on [0, 10]^2, periodic, 256^2 Q^2, scheme (eq:3),
      Lax--Friedrichs, CFL 0.1, T = 1;
  c3  2D Euler density wave rho = 1 + 0.2 sin(pi(x+y)), (u, v, p) = (0.7, 0.3, 1)
      on [0, 2]^2, periodic, 1024^2 Q^3, RK4, CFL 0.05, T = 0.5 (the paper's
      2D Euler accuracy example, Section 4.1.2, scaled up);
  c4  2D Euler four-quadrant Riemann problems on [0, 1]^2, 1024^2 Q^2, (eq:3),
      transmissive, quadrant states drawn from the seed, TVB M = 50;
  c5  2D Euler on [0, 4] x [0, 1], 4096 x 1024 Q^2, (eq:3): a Mach-3 planar shock
      (post-shock state of the paper's Shu--Osher example, Section 4.2.1) at a
      seeded angle in [20, 40] degrees running into a density field
      1 + 0.1 xi, xi a smoothed unit-variance noise field; left boundary holds
      the post-shock state, the others are transmissive; TVB M = 50 (the
      paper's 2D shock examples use M = 50, Section 4.2.2).
"""
import math

import numpy as np

GAMMA = 1.4
POST_SHOCK = (3.857143, 2.629369, 10.333333)  # (rho, normal velocity, p), Mach 3 into (1, 0, 1)

# tableaus as (A, b, c); the paper's schemes (eq:2), (eq:3), classical RK4, and
# the Butcher form of SSP-RK3 named for the 1D advection workload
TABLEAU = {
    "fe": ([[0.0]], [1.0], [0.0]),
    "eq2": ([[0, 0], [0.5, 0]], [0, 1], [0, 0.5]),
    "eq3": ([[0, 0, 0], [1 / 3, 0, 0], [0, 2 / 3, 0]], [0.25, 0, 0.75], [0, 1 / 3, 2 / 3]),
    "ssp3": ([[0, 0, 0], [1, 0, 0], [0.25, 0.25, 0]], [1 / 6, 1 / 6, 2 / 3], [0, 1, 0.5]),
    "rk4": ([[0, 0, 0, 0], [0.5, 0, 0, 0], [0, 0.5, 0, 0], [0, 0, 1, 0]],
            [1 / 6, 1 / 3, 1 / 3, 1 / 6], [0, 0.5, 0.5, 1]),
}
RK_STAGES = {"fe": 1, "eq2": 2, "eq3": 3, "rk4": 4}


def config(name, scale=1):
    """Workload description; `scale` divides the cell counts (for small
    parity versions of the same problem)."""
    if name == "c1":
        return dict(name="c1", dim=1, nx=64 // scale, ny=1, box=(0.0, 2 * math.pi, 0.0, 1.0),
                    k=2, equation="advection", flux="upwind", tableau="ssp3", adv=(1.0, 0.0),
                    bc=("periodic",) * 4, ic="adv_sin", dt_over_h=0.1, steps=640, limiter=None)
    if name == "c2":
        return dict(name="c2", dim=2, nx=256 // scale, ny=256 // scale, box=(0.0, 10.0, 0.0, 10.0),
                    k=2, equation="euler", flux="llf", tableau="eq3", bc=("periodic",) * 4,
                    ic="vortex", ic_params=[5.0, 5.0, 5.0, 10.0, 10.0], cfl=0.1, T=1.0,
                    limiter=None)
    if name == "c3":
        return dict(name="c3", dim=2, nx=1024 // scale, ny=1024 // scale, box=(0.0, 2.0, 0.0, 2.0),
                    k=3, equation="euler", flux="llf", tableau="rk4", bc=("periodic",) * 4,
                    ic="euler_wave", ic_params=[0.7, 0.3, 1.0], cfl=0.05, T=0.5, limiter=None)
    if name == "c4":
        return dict(name="c4", dim=2, nx=1024 // scale, ny=1024 // scale, box=(0.0, 1.0, 0.0, 1.0),
                    k=2, equation="euler", flux="llf", tableau="eq3", bc=("transmissive",) * 4,
                    ic="quadrant", cfl=0.1, T_over_smax=0.25, limiter=("tvb", 50.0))
    if name == "c5":
        return dict(name="c5", dim=2, nx=4096 // scale, ny=1024 // scale, box=(0.0, 4.0, 0.0, 1.0),
                    k=2, equation="euler", flux="llf", tableau="eq3",
                    bc=("dirichlet", "transmissive", "transmissive", "transmissive"),
                    ic="shock", cfl=0.1, T=0.25, limiter=("tvb", 50.0))
    raise KeyError(name)


def quadrant_states(seed):
    """(rho, u, v, p) for the NE, NW, SW, SE quadrants, in that draw order"""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(4):
        rho = rng.uniform(0.1, 1.5)
        u = rng.uniform(-1.0, 1.0)
        v = rng.uniform(-1.0, 1.0)
        p = rng.uniform(0.1, 1.5)
        out.append((rho, u, v, p))
    return out


def quadrant_params(seed, split=(0.5, 0.5)):
    p = [split[0], split[1]]
    for s in quadrant_states(seed):
        p.extend(s)
    return p


def shock_angle(seed):
    rng = np.random.default_rng(seed)
    return math.radians(rng.uniform(20.0, 40.0)), rng


def smoothed_noise(rng, nx, ny, sigma_cells=8.0):
    """white noise on the cell-centre grid, Gaussian-filtered (periodic FFT,
    sigma in cells) and renormalised to zero mean and unit variance"""
    w = rng.standard_normal((ny, nx))
    kx = np.fft.fftfreq(nx)
    ky = np.fft.fftfreq(ny)
    G = np.exp(-2.0 * (math.pi * sigma_cells) ** 2 * (kx[None, :] ** 2 + ky[:, None] ** 2))
    f = np.real(np.fft.ifft2(np.fft.fft2(w) * G))
    f -= f.mean()
    f /= f.std()
    return np.ascontiguousarray(f)


def shock_problem(seed, nx, ny, field_grid=None):
    """parameters of the shock workload and its noise field xi on the nx x ny
    cell-centre grid, or on the field_grid = (na, ma) grid over the same
    domain (so that meshes of different resolution see the same initial
    density function; the grid size then travels in params[8:10])"""
    theta, rng = shock_angle(seed)
    na, ma = field_grid if field_grid is not None else (nx, ny)
    xi = smoothed_noise(rng, na, ma)
    rho_s, un_s, p_s = POST_SHOCK
    params = [theta, rho_s, un_s, p_s, 0.5, 0.5, 0.5, 0.1]
    if field_grid is not None:
        params += [float(na), float(ma)]
    return params, xi


def post_shock_conserved(theta):
    rho, un, p = POST_SHOCK
    u, v = un * math.cos(theta), un * math.sin(theta)
    return [rho, rho * u, rho * v, p / (GAMMA - 1) + 0.5 * rho * (u * u + v * v)]


def random_euler_modes(rng, nmodes, ncells, amp=0.05):
    """random but physical 2D Euler modal data (for operator parity tests)"""
    u = amp * rng.standard_normal((4, nmodes, ncells))
    u[0, 0] = 1.0 + 0.3 * rng.random(ncells)
    u[1, 0] = 0.4 * rng.standard_normal(ncells)
    u[2, 0] = 0.4 * rng.standard_normal(ncells)
    u[3, 0] = 2.5 + rng.random(ncells)
    return u
