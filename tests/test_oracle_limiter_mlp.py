"""Pins of the oracle's final-stage limiter and of the learned indicator.

The paper applies a TVB minmod limiter once per cRKDG step after the final
stage (Section 2.2 remark on limiters; Section 4.2) and defers the limiter's
details to its reference [rkdg5].  Parity unpinned against the paper: these
tests pin generic properties only (means kept exactly, linear data never
troubled, jumps always troubled, eigen-decomposition exact, threshold).
The MLP indicator is not in the paper: its gradient is pinned by finite
differences and its optimiser by the closed form of the first Adam step.
"""
import numpy as np
import pytest

import oracle as O
from tests import bruteforce as BF


def quad_mesh(n, bc=1):
    return O.Mesh(2, n, n, x0=0, x1=1, y0=0, y1=1, bc=(bc,) * 4, equation=O.EQ_EULER,
                  flux=O.FLUX_LLF)


QUAD = [0.5, 0.5, 1.0, 0.75, -0.5, 1.0, 2.0, 0.0, 0.3, 1.0, 1.0, 0.0, 0.0, 0.4,
        0.5, 0.2, 0.1, 0.6]


@pytest.mark.parametrize("d", [0, 1])
def test_euler_eigenvectors(d):
    mesh = quad_mesh(4)
    q = np.array([1.3, 0.4, -0.5, 3.7])
    L, R = O.euler_eig(mesh, q, d)
    assert np.allclose(L @ R, np.eye(4), atol=1e-13)
    # columns of R are eigenvectors of the Jacobian (central differences of
    # an independently written flux) with eigenvalues u_n - c, u_n, u_n, u_n + c
    J = np.zeros((4, 4))
    eps = 1e-6
    for j in range(4):
        e = np.zeros(4)
        e[j] = eps
        J[:, j] = (BF.euler_flux(q + e, d, 2) - BF.euler_flux(q - e, d, 2)) / (2 * eps)
    un = q[1 + d] / q[0]
    p = 0.4 * (q[3] - 0.5 * (q[1] ** 2 + q[2] ** 2) / q[0])
    c = np.sqrt(1.4 * p / q[0])
    for col, lam in enumerate([un - c, un, un, un + c]):
        assert np.allclose(J @ R[:, col], lam * R[:, col], atol=1e-7)


def test_limiter_keeps_means_exactly():
    mesh = quad_mesh(12)
    k = 2
    # jumps cut through cells; uniform cells have zero slopes and stay untouched
    u = O.project(mesh, k, O.IC_QUADRANT, [0.53, 0.47] + QUAD[2:])
    v, flags, n = O.limit_tvb(mesh, k, 1e-3, u)  # M h^2 above round-off
    assert 0 < n < mesh.ncells
    assert np.array_equal(v[:, 0], u[:, 0])
    # untouched cells are bit-identical; troubled ones keep only P1 modes
    keep = flags == 0
    assert np.array_equal(v[:, :, keep], u[:, :, keep])
    hi = [b for b in range(9) if b not in (0, 1, 3)]
    assert np.all(v[:, hi][:, :, ~keep] == 0.0)


@pytest.mark.parametrize("k", [1, 2, 3])
def test_linear_data_is_never_troubled(k):
    mesh = quad_mesh(10)
    nb = (k + 1) ** 2
    u = np.zeros((4, nb, 100))
    xc = (np.arange(10) + 0.5) / 10
    X, Y = np.meshgrid(xc, xc)
    lin = [(1.0, 0.2, 0.1), (0.1, 0.05, -0.02), (0.05, 0.0, 0.03), (2.5, 0.1, 0.2)]
    for c, (a0, ax, ay) in enumerate(lin):
        u[c, 0] = (a0 + ax * X + ay * Y).ravel()
        u[c, 1] = ax * 0.05
        u[c, k + 1] = ay * 0.05
    flags, margin, n = O.tvb_flags(mesh, k, 0.0, u)
    # boundary cells see a zero one-sided difference (transmissive ghosts)
    assert not flags.reshape(10, 10)[1:-1, 1:-1].any()
    assert n == 36


def test_jump_is_troubled_and_threshold_switches_it_off():
    mesh = quad_mesh(16)
    k = 2
    u = O.project(mesh, k, O.IC_QUADRANT, [0.53, 0.47] + QUAD[2:])  # jumps inside cells
    flags, _, n = O.tvb_flags(mesh, k, 1e-3, u)
    F = flags.reshape(16, 16)
    assert n > 0
    assert F[:, 8].all() and F[7, :].all()  # the cut columns / rows
    # a huge TVB constant accepts every jump
    _, _, n_big = O.tvb_flags(mesh, k, 1e12, u)
    assert n_big == 0


def test_scalar_minmod_truth_table_through_1d_limiter():
    """1D scalar data, three cells; the middle cell's slope against the
    neighbour differences decides (minmod of equal signs keeps the smallest
    magnitude; mixed signs give zero)"""
    mesh = O.Mesh(1, 3, x0=0, x1=3, bc=(1, 1, 0, 0), equation=O.EQ_ADVECTION,
                  flux=O.FLUX_UPWIND, adv=(1.0, 0))
    cases = [
        # (averages, middle slope mode, expected limited slope, troubled)
        ((0.0, 1.0, 2.0), 0.4, 0.4, False),   # |a| smallest, same signs
        ((0.0, 1.0, 2.0), 1.5, 1.0, True),    # limited to the differences
        ((0.0, 1.0, 0.0), 0.3, 0.0, True),    # extremum: mixed signs -> 0
        ((0.0, 1.0, 2.0), -0.2, 0.0, True),   # slope against the trend
    ]
    for avgs, slope, expect, troubled in cases:
        u = np.zeros((1, 2, 3))
        u[0, 0] = avgs
        u[0, 1, 1] = slope
        v, flags, _ = O.limit_tvb(mesh, 1, 0.0, u)
        assert bool(flags[1]) == troubled
        assert v[0, 1, 1] == expect
        assert np.array_equal(v[0, 0], u[0, 0])


def test_positivity_safeguard_demotes_and_keeps_mean():
    mesh = quad_mesh(4, bc=1)
    k = 2
    u = O.project(mesh, k, O.IC_CONST, [1.0, 0.0, 0.0, 2.5])
    u[0, 4, 5] = 1.5  # (1,1) mode of density: rho < 0 at face points
    v, flags, n = O.limit_tvb(mesh, k, 1e12, u)
    assert flags[5] & 2  # positivity demotion bit
    assert np.array_equal(v[:, 0], u[:, 0])
    assert n == 1


def test_nonphysical_mean_is_reported():
    mesh = quad_mesh(4, bc=1)
    u = O.project(mesh, 1, O.IC_CONST, [1.0, 0.0, 0.0, 2.5])
    u[3, 0, 2] = -1.0
    _, _, n = O.limit_tvb(mesh, 1, 50.0, u)
    assert n == -1


# --- learned indicator -----------------------------------------------------

def test_features_of_linear_data():
    mesh = O.Mesh(2, 8, 8, x0=0, x1=1, y0=0, y1=1, bc=(0,) * 4, equation=O.EQ_EULER)
    k, M = 2, 50.0
    u = np.zeros((4, 9, 64))
    xc = (np.arange(8) + 0.5) / 8
    X, Y = np.meshgrid(xc, xc)
    ax, ay = 0.4, -0.3
    u[0, 0] = (1.0 + ax * X + ay * Y).ravel()
    u[0, 1] = ax / 16
    u[0, 3] = ay / 16
    u[3, 0] = 2.5
    Xf = O.mlp_features(mesh, k, M, u)
    h = 1 / 8
    i, j = 3, 4  # interior cell
    x = Xf[j * 8 + i]
    sx = 2 * abs(ax) * h + M * h * h
    assert x[0] == pytest.approx(ax * h / 2 / sx, rel=1e-12)
    assert x[1] == pytest.approx(ax * h / 2 / sx, rel=1e-12)
    assert abs(x[2]) < 1e-12
    sy = 2 * abs(ay) * h + M * h * h
    assert x[3] == pytest.approx(ay * h / 2 / sy, rel=1e-12)
    assert np.all(x[6:] == 0.0)  # energy is constant


def test_mlp_gradient_matches_finite_differences():
    rng = np.random.default_rng(1)
    P = 0.3 * rng.standard_normal(O.N_MLP_PARAMS)
    X = rng.standard_normal((64, 12))
    y = (rng.random(64) < 0.3).astype(np.uint8)
    loss, g = O.mlp_loss_grad(P, X, y, pos_weight=3.0)
    idx = rng.choice(O.N_MLP_PARAMS, 50, replace=False)
    h = 1e-6
    for i in idx:
        Pp, Pm = P.copy(), P.copy()
        Pp[i] += h
        Pm[i] -= h
        fd = (O.mlp_loss_grad(Pp, X, y, 3.0)[0] - O.mlp_loss_grad(Pm, X, y, 3.0)[0]) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(g[i])), (i, fd, g[i])


def test_mlp_zero_params_and_loss_value():
    P = np.zeros(O.N_MLP_PARAMS)
    P[-1] = 0.7
    X = np.random.default_rng(2).standard_normal((5, 12))
    assert np.allclose(O.mlp_forward(P, X), 0.7)
    y = np.array([1, 0, 1, 0, 0], dtype=np.uint8)
    loss, _ = O.mlp_loss_grad(P, X, y, pos_weight=2.0)
    sp = lambda z: np.log1p(np.exp(z))
    ref = (2 * (2.0 * sp(-0.7)) + 3 * sp(0.7)) / 5
    assert loss == pytest.approx(ref, rel=1e-14)


def test_adam_first_step_closed_form():
    g = np.array([0.5, -2.0, 1e-3])
    p = np.zeros(3)
    m1, m2 = np.zeros(3), np.zeros(3)
    O.adam(p, m1, m2, g, 1, lr=0.01, eps=1e-8)
    assert np.allclose(p, -0.01 * g / (np.abs(g) + 1e-8), rtol=1e-12)


def hand_network():
    """W1: h1_0 = x0, h1_1 = x1 - 0.5; W2: h2_0 = 3 h1_0 + 5 h1_1, h2_1 = -h1_0;
    output z = 2 h2_0 + 4 h2_1 - 1 (all other weights zero)"""
    P = np.zeros(O.N_MLP_PARAMS)
    OW1, OB1 = 0, 12 * 32
    OW2, OB2 = OB1 + 32, OB1 + 32 + 32 * 32
    OW3, OB3 = OB2 + 32, OB2 + 64
    P[OW1 + 0 * 12 + 0] = 1.0
    P[OW1 + 1 * 12 + 1] = 1.0
    P[OB1 + 1] = -0.5
    P[OW2 + 0 * 32 + 0] = 3.0
    P[OW2 + 0 * 32 + 1] = 5.0
    P[OW2 + 1 * 32 + 0] = -1.0
    P[OW3 + 0] = 2.0
    P[OW3 + 1] = 4.0
    P[OB3] = -1.0
    return P


def test_mlp_relu_network_by_hand():
    P = hand_network()
    X = np.zeros((3, 12))
    X[0, :2] = [1.0, 2.0]     # h1 = (1, 1.5): h2 = (10.5, 0): z = 20
    X[1, :2] = [-1.0, 0.25]   # h1 = (0, 0): h2 = (0, 0): z = -1
    X[2, :2] = [-2.0, 1.0]    # h1 = (0, 0.5): h2 = (2.5, 0): z = 4
    assert np.array_equal(O.mlp_forward(P, X), [20.0, -1.0, 4.0])


def test_forced_reconstruction_returns_the_p1_slopes():
    """positivity forces the limited P1 reconstruction on a cell whose slopes
    no field limits (huge M): mapping the characteristic slopes back must
    give the conserved slopes unchanged (R L s = s for any s), and every
    other mode, including (1,1), is zeroed; the mean is kept"""
    mesh = quad_mesh(4, bc=1)
    k = 2
    u = O.project(mesh, k, O.IC_CONST, [1.0, 0.3, -0.2, 2.5])
    cell = 5
    sx = np.array([0.1, 0.05, -0.03, 0.2])    # mode (1,0) of the four components
    sy = np.array([-0.08, 0.02, 0.04, -0.1])  # mode (0,1)
    u[:, 1, cell] = sx
    u[:, 3, cell] = sy
    u[0, 4, cell] = 1.5                       # density mode (1,1): rho < 0 at corners
    u[3, 8, cell] = 0.05                      # energy mode (2,2)
    v, flags, _ = O.limit_tvb(mesh, k, 1e12, u)
    assert flags[cell] == 2                   # forced by the point test, not by TVB
    assert np.abs(v[:, 1, cell] - sx).max() <= 1e-14
    assert np.abs(v[:, 3, cell] - sy).max() <= 1e-14
    assert np.all(v[:, [2, 4, 5, 6, 7, 8], cell] == 0.0)
    assert np.array_equal(v[:, 0], u[:, 0])


def _fd_jacobian(q, d):
    J = np.zeros((4, 4))
    eps = 1e-6
    for j in range(4):
        e = np.zeros(4)
        e[j] = eps
        J[:, j] = (BF.euler_flux(q + e, d, 2) - BF.euler_flux(q - e, d, 2)) / (2 * eps)
    return J


@pytest.mark.parametrize("d", [0, 1])
def test_one_limited_characteristic_field_matches_numpy_eigenvectors(d):
    """the middle cell of a 3-cell row (column for d = 1), P1 slope s and
    neighbour differences D+ and D- built in the eigenvector basis of the
    flux Jacobian (numpy's eig of central differences of an independently
    written flux, not the oracle's eigenvectors): the u - c field has
    coefficients (1, 0.2, 0.5), so minmod limits it to 0.2; the u + c field
    (0.3, 1, 0.8) keeps 0.3; in the double eigenvalue u's eigenspace D+ and
    D- are 2 s, so that part of s is kept in every basis of the eigenspace.
    With M = 0 the limited slope is independent of how the eigenvectors
    are scaled: it must be s - 0.8 (0.02 r_{u-c})."""
    qb = np.array([1.3, 0.4, -0.5, 3.7])
    J = _fd_jacobian(qb, d)
    lam, V = np.linalg.eig(J)
    assert np.abs(lam.imag).max() < 1e-9
    lam, V = lam.real, V.real
    order = np.argsort(lam)
    lam, V = lam[order], V[:, order]
    un = qb[1 + d] / qb[0]
    p = 0.4 * (qb[3] - 0.5 * (qb[1] ** 2 + qb[2] ** 2) / qb[0])
    c = np.sqrt(1.4 * p / qb[0])
    assert np.allclose(lam, [un - c, un, un, un + c], atol=1e-8)
    r1, r2, r3, r4 = (V[:, i] for i in range(4))
    a = 0.02
    su = a * (0.1 * r2 - 0.05 * r3)          # the part of s in u's eigenspace
    s = a * 1.0 * r1 + su + a * 0.3 * r4
    dp = a * 0.2 * r1 + 2 * su + a * 1.0 * r4
    dm = a * 0.5 * r1 + 2 * su + a * 0.8 * r4
    expect = s - a * 0.8 * r1
    k = 2
    n = 3
    mesh = O.Mesh(2, n if d == 0 else 1, 1 if d == 0 else n, x0=0, x1=n if d == 0 else 1,
                  y0=0, y1=1 if d == 0 else n, bc=(1, 1, 1, 1), equation=O.EQ_EULER,
                  flux=O.FLUX_LLF)
    u = np.zeros((4, 9, 3))
    u[:, 0, 0] = qb - dm
    u[:, 0, 1] = qb
    u[:, 0, 2] = qb + dp
    slope = 1 if d == 0 else 3               # mode (1,0) or (0,1)
    u[:, slope, 1] = s
    u[:, 4, 1] = 0.01                         # mode (1,1): zeroed in a limited cell
    v, flags, _ = O.limit_tvb(mesh, k, 0.0, u)
    assert flags[1] == 1
    assert np.abs(v[:, slope, 1] - expect).max() <= 1e-7 * np.abs(expect).max()
    other = [b for b in range(1, 9) if b != slope]
    assert np.all(v[:, other, 1] == 0.0)
    assert np.array_equal(v[:, 0, 1], qb)
    # the limited field really moved: the unlimited slope is far from it
    assert np.abs(s - expect).max() > 1e-3


@pytest.mark.parametrize("k", [2, 3])
def test_features_of_polynomial_data_in_closed_form(k):
    """a density varying as x^2 (k = 2) or x^3 (k = 3) along x and an energy
    varying as y^2 / y^3 along y, each represented exactly on every cell:
    the trace jumps, neighbour differences and the 12 features follow from
    point values and cell averages of the polynomials (written out here),
    not from the modal coefficients"""
    n, M = 6, 50.0
    h = 1.0 / n
    mesh = O.Mesh(2, n, n, x0=0, x1=1, y0=0, y1=1, bc=(1, 1, 1, 1), equation=O.EQ_EULER,
                  flux=O.FLUX_LLF)
    Q = k + 1
    # Legendre coefficients on a cell of centre xc, width h of q(x) = x^k:
    # substitute x = xc + (h/2) xi and expand xi^2 = (P0 + 2 P2)/3,
    # xi^3 = (3 P1 + 2 P3)/5
    def coeffs(xc):
        g = h / 2
        if k == 2:
            return [xc * xc + g * g / 3, 2 * xc * g, 2 * g * g / 3]
        return [xc ** 3 + xc * g * g, 3 * xc * xc * g + 3 * g ** 3 / 5, 2 * xc * g * g, 2 * g ** 3 / 5]

    def avg(xc):  # exact cell average of x^k
        a, b = xc - h / 2, xc + h / 2
        return (b ** (k + 1) - a ** (k + 1)) / ((k + 1) * h)

    u = np.zeros((4, Q * Q, n * n))
    for j in range(n):
        for i in range(n):
            cell = j * n + i
            xc, yc = (i + 0.5) * h, (j + 0.5) * h
            cx, cy = coeffs(xc), coeffs(yc)
            u[0, 0, cell] = 2.0 + cx[0]
            u[3, 0, cell] = 3.0 + cy[0]
            for m in range(1, Q):
                u[0, m, cell] = cx[m]          # density modes (m, 0)
                u[3, m * Q, cell] = cy[m]      # energy modes (0, m)
    assert np.allclose(u[0, 0], 2.0 + np.tile([avg((i + 0.5) * h) for i in range(n)], n),
                       rtol=0, atol=1e-15)
    X = O.mlp_features(mesh, k, M, u)
    f = lambda x: x ** k
    for j in range(1, n - 1):
        for i in range(1, n - 1):
            cell = j * n + i
            want = np.zeros(12)
            for qi, (coord, along) in enumerate((((i + 0.5) * h, 0), ((j + 0.5) * h, 1))):
                c = coord
                fwd = f(c + h / 2) - avg(c)     # forward face value minus the average
                bwd = avg(c) - f(c - h / 2)     # the average minus the backward face value
                dp = avg(c + h) - avg(c)
                dm = avg(c) - avg(c - h)
                s = abs(dp) + abs(dm) + M * h * h + 1e-300
                # direction `along` varies; the other direction sees constants
                want[(qi * 2 + along) * 3:(qi * 2 + along) * 3 + 3] = [fwd / s, bwd / s,
                                                                       (dp - dm) / s]
            assert np.allclose(X[cell], want, rtol=1e-12, atol=1e-14), (i, j, X[cell], want)
    # the backward and forward jumps really differ here (an even-degree term)
    assert np.abs(X[:, 0] - X[:, 1]).max() > 1e-4
