"""Pins of the oracle's tables and spatial operators against things other
than the oracle itself: numpy's Legendre/Gauss routines, exact derivatives
of polynomials, flux consistency, and an independent dense brute force.

Paper references: DG operator (Section 2.1, equation (DG operator)); local
operator and its projection property (Section 2.2, equation (dxl));
P^0 local operator vanishes (Section 3.3); flux consistency (Section 3.2.2,
theorem 'thm:lwthm' assumption 2(a)).
"""
import numpy as np
import pytest
from numpy.polynomial import legendre as npleg

import oracle as O
from tests import bruteforce as BF


# --- tables --------------------------------------------------------------

@pytest.mark.parametrize("n", range(1, 9))
def test_gauss_matches_numpy_and_integrates_monomials(n):
    x, w = O.gauss(n)
    xr, wr = npleg.leggauss(n)
    assert np.allclose(x, xr, atol=1e-15, rtol=0)
    assert np.allclose(w, wr, atol=1e-15, rtol=0)
    assert abs(w.sum() - 2.0) < 1e-14
    for p in range(2 * n):  # exact up to degree 2n-1
        exact = 0.0 if p % 2 else 2.0 / (p + 1)
        assert abs((w * x**p).sum() - exact) < 1e-14


@pytest.mark.parametrize("m", range(0, 7))
def test_legendre_values_and_derivatives(m):
    xs = np.linspace(-1, 1, 17)
    c = np.eye(m + 1)[m]
    for x in xs:
        assert abs(O.legendre(m, x) - npleg.legval(x, c)) < 1e-14
        assert abs(O.dlegendre(m, x) - npleg.legval(x, npleg.legder(c))) < 1e-13
    assert O.legendre(m, 1.0) == 1.0 and O.legendre(m, -1.0) == (-1.0) ** m
    xg, wg = npleg.leggauss(m + 1)
    norm = sum(wg[i] * O.legendre(m, xg[i]) ** 2 for i in range(m + 1))
    assert abs(norm - 2.0 / (2 * m + 1)) < 1e-14


# --- local operator = projected derivative for linear flux ---------------

@pytest.mark.parametrize("k", [0, 1, 2, 3])
def test_loc_linear_flux_is_exact_derivative_1d(k):
    rng = np.random.default_rng(k)
    nx, L, a = 7, 2.0, 1.7
    mesh = O.Mesh(1, nx, x0=0, x1=L, equation=O.EQ_ADVECTION, flux=O.FLUX_UPWIND, adv=(a, 0))
    u = rng.standard_normal(mesh.shape(k))
    out = O.apply(mesh, k, O.OP_LOC, u)
    h = L / nx
    for cell in range(nx):
        der = npleg.legder(u[0, :, cell]) * (2.0 / h) * a
        der = np.concatenate([der, np.zeros(k + 1 - der.size)])
        assert np.allclose(out[0, :, cell], der, atol=1e-12 * (1 + abs(der).max()))


@pytest.mark.parametrize("k", [0, 1, 2, 3])
def test_loc_linear_flux_is_exact_derivative_2d(k):
    rng = np.random.default_rng(10 + k)
    nx, ny, a, b = 3, 4, 0.7, -1.3
    mesh = O.Mesh(2, nx, ny, x0=0, x1=1.5, y0=-1, y1=1, equation=O.EQ_ADVECTION,
                  flux=O.FLUX_UPWIND, adv=(a, b))
    u = rng.standard_normal(mesh.shape(k))
    out = O.apply(mesh, k, O.OP_LOC, u)
    hx, hy = 1.5 / nx, 2.0 / ny
    for cell in range(nx * ny):
        C = u[0, :, cell].reshape(k + 1, k + 1)  # C[n, m]: mode m + (k+1) n
        dx = np.zeros_like(C)
        dy = np.zeros_like(C)
        if k > 0:
            dx[:, :k] = npleg.legder(C, axis=1) * (2 / hx)
            dy[:k, :] = npleg.legder(C, axis=0) * (2 / hy)
        ref = (a * dx + b * dy).ravel()
        assert np.allclose(out[0, :, cell], ref, atol=1e-12 * (1 + abs(ref).max()))


@pytest.mark.parametrize("dim", [1, 2])
def test_loc_vanishes_for_p0(dim):
    rng = np.random.default_rng(3)
    mesh = O.Mesh(dim, 5, 4, x0=0, x1=1, y0=0, y1=1, equation=O.EQ_EULER, flux=O.FLUX_LLF)
    nc = mesh.ncomp()
    u = np.zeros(mesh.shape(0))
    u[0, 0] = 1 + 0.3 * rng.random(mesh.ncells)
    u[1, 0] = 0.2 * rng.standard_normal(mesh.ncells)
    if dim == 2:
        u[2, 0] = 0.2 * rng.standard_normal(mesh.ncells)
    u[nc - 1, 0] = 2.5 + rng.random(mesh.ncells)
    assert np.all(O.apply(mesh, 0, O.OP_LOC, u) == 0.0)


@pytest.mark.parametrize("k", [0, 1, 2, 3])
@pytest.mark.parametrize("dim", [1, 2])
def test_free_stream(dim, k):
    mesh = O.Mesh(dim, 4, 3, x0=0, x1=1, y0=0, y1=2, equation=O.EQ_EULER, flux=O.FLUX_LLF)
    q = [1.3, 0.4, -0.2, 3.1] if dim == 2 else [1.3, 0.4, 3.1]
    u = O.project(mesh, k, O.IC_CONST, q)
    for op in (O.OP_LOC, O.OP_DG):
        out = O.apply(mesh, k, op, u)
        assert np.abs(out).max() < 1e-13


@pytest.mark.parametrize("k", [1, 2, 3])
@pytest.mark.parametrize("dim", [1, 2])
def test_dg_equals_loc_for_continuous_polynomial_state(dim, k):
    """u_int = u_ext on every face, so the consistent numerical flux equals
    f(u).nu and the two operators coincide"""
    mesh = O.Mesh(dim, 4, 3, x0=0, x1=1, y0=0, y1=1, bc=(1, 1, 1, 1),
                  equation=O.EQ_EULER, flux=O.FLUX_LLF)
    nc = mesh.ncomp()
    u = np.zeros(mesh.shape(k))
    # global polynomial of degree 1 in x (and y): exactly representable
    xc = (np.arange(4) + 0.5) / 4
    yc = (np.arange(3) + 0.5) / 3
    X = np.tile(xc, mesh.ny if dim == 2 else 1)
    Y = np.repeat(yc, 4) if dim == 2 else 0 * X
    coef = [(1.0, 0.3, 0.2), (0.2, 0.1, -0.1), (-0.1, 0.05, 0.1), (3.0, 0.2, 0.3)]
    comps = coef if dim == 2 else [coef[0], coef[1], coef[3]]
    for c, (c0, cx, cy) in enumerate(comps[:nc]):
        u[c, 0] = c0 + cx * X + (cy * Y if dim == 2 else 0)
        u[c, 1] = cx * 0.5 / 4
        if dim == 2:
            u[c, k + 1] = cy * 0.5 / 3
    lo = O.apply(mesh, k, O.OP_LOC, u)
    dg = O.apply(mesh, k, O.OP_DG, u)
    assert np.allclose(lo, dg, atol=1e-12, rtol=1e-12)


# --- dense brute force ----------------------------------------------------

def _random_euler_state(rng, shape, dim):
    nc, nb, n = shape
    u = 0.05 * rng.standard_normal(shape)
    u[0, 0] = 1.0 + 0.2 * rng.random(n)
    u[1, 0] = 0.3 * rng.standard_normal(n)
    if dim == 2:
        u[2, 0] = 0.3 * rng.standard_normal(n)
    u[nc - 1, 0] = 2.5 + rng.random(n)
    return u


@pytest.mark.parametrize("k", [0, 1, 2, 3, 4])
@pytest.mark.parametrize("dim", [1, 2])
@pytest.mark.parametrize("equation", ["advection", "euler"])
@pytest.mark.parametrize("bc", ["periodic", "transmissive"])
def test_operators_match_dense_brute_force(k, dim, equation, bc):
    rng = np.random.default_rng(100 * k + 10 * dim + (equation == "euler"))
    nx, ny, lx, ly = 3, 3, 1.2, 0.9
    eq = O.EQ_EULER if equation == "euler" else O.EQ_ADVECTION
    adv = (0.8, -1.1)
    bcc = O.BC_PERIODIC if bc == "periodic" else O.BC_TRANSMISSIVE
    mesh = O.Mesh(dim, nx, ny, x0=0, x1=lx, y0=0, y1=ly, bc=(bcc,) * 4, equation=eq,
                  flux=O.FLUX_LLF, adv=adv)
    prob = BF.Problem(dim, nx, ny, k, lx, ly, equation, adv=adv, bc=bc)
    if equation == "euler":
        u = _random_euler_state(rng, mesh.shape(k), dim)
    else:
        u = rng.standard_normal(mesh.shape(k))
    for op, name in ((O.OP_LOC, "loc"), (O.OP_DG, "dg")):
        a = O.apply(mesh, k, op, u)
        b = BF.apply(prob, u, name)
        scale = 1 + np.abs(b).max()
        assert np.abs(a - b).max() <= 1e-12 * scale, (name, np.abs(a - b).max())
