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


def test_bf16_rounding_ties_to_even():
    """bfloat16 keeps 8 significand bits: spacing 2^-7 just above 1"""
    assert O.bf16(1.0 + 2.0 ** -8) == 1.0                      # tie, even neighbour below
    assert O.bf16(1.0 + 3 * 2.0 ** -8) == 1.0 + 2.0 ** -6      # tie, even neighbour above
    assert O.bf16(1.0 + 2.0 ** -8 + 2.0 ** -20) == 1.0 + 2.0 ** -7
    assert O.bf16(-(1.0 + 2.0 ** -8)) == -1.0
    assert O.bf16(0.15625) == 0.15625                          # already representable


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
    assert np.array_equal(O.mlp_infer(P, X), [20.0, -1.0, 4.0])   # all values bf16-exact


def test_mlp_infer_matches_forward_within_bf16():
    rng = np.random.default_rng(3)
    P = 0.3 * rng.standard_normal(O.N_MLP_PARAMS)
    X = rng.standard_normal((200, 12))
    z64 = O.mlp_forward(P, X)
    zin = O.mlp_infer(P, X)
    # bfloat16 carries 2^-9 relative error per rounded value; a few percent of
    # the logit scale at most
    assert np.abs(zin - z64).max() < 0.05 * max(1.0, np.abs(z64).max())
    assert np.abs(zin - z64).max() > 0.0  # the rounding is really applied
