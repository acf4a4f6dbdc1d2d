"""Brute-force dense-matrix evaluation of the paper's two spatial operators.

Independent of the oracle: basis functions from numpy.polynomial.legendre,
quadrature from numpy's leggauss, a full mass matrix assembled by
quadrature and solved with numpy.linalg (no diagonal-mass shortcut), each
face flux computed once in canonical orientation and scattered with +/- to
the two cells.  Vectorised over cells with numpy; used only on tiny meshes.

Definitions: DG operator, Section 2.1, equation (DG operator); local
operator, Section 2.2, equation (dxl).  Quadrature: (k+1) Gauss points per
direction in the volume and on each face.
"""
import numpy as np
from numpy.polynomial import legendre as npleg

GAMMA = 1.4


def _P(k, x):
    return np.array([npleg.legval(x, np.eye(k + 1)[m]) for m in range(k + 1)])


def _dP(k, x):
    return np.array([npleg.legval(x, npleg.legder(np.eye(k + 1)[m])) if m > 0 else 0 * x
                     for m in range(k + 1)])


def euler_flux(q, d, dim):
    """physical Euler flux in direction d; q has the component axis first"""
    rho = q[0]
    if dim == 1:
        w = q[1] / rho
        p = (GAMMA - 1) * (q[2] - 0.5 * rho * w * w)
        return np.stack([q[1], q[1] * w + p, w * (q[2] + p)])
    u, v = q[1] / rho, q[2] / rho
    p = (GAMMA - 1) * (q[3] - 0.5 * rho * (u * u + v * v))
    vn = u if d == 0 else v
    mom = [q[1] * vn, q[2] * vn]
    mom[d] = mom[d] + p
    return np.stack([rho * vn, mom[0], mom[1], vn * (q[3] + p)])


def euler_speed(q, d, dim):
    rho = q[0]
    if dim == 1:
        w = q[1] / rho
        p = (GAMMA - 1) * (q[2] - 0.5 * rho * w * w)
        vn = w
    else:
        u, v = q[1] / rho, q[2] / rho
        p = (GAMMA - 1) * (q[3] - 0.5 * rho * (u * u + v * v))
        vn = u if d == 0 else v
    return np.abs(vn) + np.sqrt(GAMMA * p / rho)


class Problem:
    def __init__(self, dim, nx, ny, k, lx, ly, equation, adv=(1.0, 0.0), bc="periodic"):
        self.dim, self.nx, self.ny, self.k = dim, nx, (ny if dim == 2 else 1), k
        self.hx, self.hy = lx / nx, (ly / ny if dim == 2 else 1.0)
        self.equation, self.adv, self.bc = equation, adv, bc

    def flux(self, q, d):
        if self.equation == "advection":
            return self.adv[d] * q
        if self.equation == "burgers":
            return 0.5 * q * q
        return euler_flux(q, d, self.dim)

    def speed(self, q, d):
        if self.equation == "advection":
            return np.full(q.shape[1:], abs(self.adv[d]))
        return euler_speed(q, d, self.dim)

    def lf(self, qL, qR, d):
        """flux across a face in the +e_d direction, left/right traces:
        Lax--Friedrichs, or for Burgers the flux of the exact Riemann
        solution sampled at the face (a shock moving at (qL + qR)/2 when
        qL > qR, else a rarefaction fan u = x/t clipped to [qL, qR])"""
        if self.equation == "burgers":
            shock = qL > qR
            u0 = np.where(shock, np.where(qL + qR > 0, qL, qR), np.clip(0.0, qL, qR))
            return 0.5 * u0 * u0
        a = np.maximum(self.speed(qL, d), self.speed(qR, d))
        return 0.5 * (self.flux(qL, d) + self.flux(qR, d) - a * (qR - qL))


def apply(prob, u, op):
    """u: (nc, nb, ncell) modal coefficients, mode m + (k+1) n.  Returns
    nabla.f in the same layout.  op: 'loc' or 'dg'."""
    k, dim = prob.k, prob.dim
    nx, ny = prob.nx, prob.ny
    nc = u.shape[0]
    Q = k + 1
    xg, wg = npleg.leggauss(Q)
    Pg, dPg = _P(k, xg), _dP(k, xg)
    P1, Pm1 = _P(k, np.array([1.0]))[:, 0], _P(k, np.array([-1.0]))[:, 0]
    if dim == 1:
        modes = [(m, 0) for m in range(k + 1)]
    else:
        modes = [(m, n) for n in range(k + 1) for m in range(k + 1)]
    nb = len(modes)
    U = u.reshape(nc, nb, ny, nx)
    # full mass matrix of the reference element by a (k+2)-point rule, then scaled
    xm, wm = npleg.leggauss(k + 2)
    Pm = _P(k, xm)
    if dim == 1:
        Mref = np.einsum("a,ia,ja->ij", wm, Pm, Pm) * prob.hx / 2
    else:
        Mref = np.zeros((nb, nb))
        for I, (m, n) in enumerate(modes):
            for J, (mm, nn) in enumerate(modes):
                Mref[I, J] = (wm * Pm[m] * Pm[mm]).sum() * (wm * Pm[n] * Pm[nn]).sum()
        Mref *= prob.hx * prob.hy / 4
    R = np.zeros((nc, nb, ny, nx))
    if dim == 1:
        V = np.array([Pg[m] for (m, _) in modes])       # (nb, Q)
        DV = np.array([dPg[m] for (m, _) in modes])
        q = np.einsum("cbji,ba->caji", U, V)             # (nc, Q, ny, nx)
        f = prob.flux(q, 0)
        R -= np.einsum("a,caji,ba->cbji", wg, f, DV)     # (h/2)(2/h) = 1
        tR = np.einsum("cbji,b->cji", U, np.array([P1[m] for m, _ in modes]))
        tL = np.einsum("cbji,b->cji", U, np.array([Pm1[m] for m, _ in modes]))
        phR = np.array([P1[m] for m, _ in modes])
        phL = np.array([Pm1[m] for m, _ in modes])
        if op == "loc":
            FR, FL = prob.flux(tR, 0), prob.flux(tL, 0)
            R += np.einsum("cji,b->cbji", FR, phR) - np.einsum("cji,b->cbji", FL, phL)
        else:
            left_of_face = np.roll(tR, 1, axis=2)   # trace of cell i-1 at its right end
            if prob.bc == "transmissive":
                left_of_face[:, :, 0] = tL[:, :, 0]
            G = prob.lf(left_of_face, tL, 0)         # flux through the left face of cell i
            Gr = np.roll(G, -1, axis=2)
            if prob.bc == "transmissive":
                Gr[:, :, -1] = prob.lf(tR[:, :, -1], tR[:, :, -1], 0)
            R += np.einsum("cji,b->cbji", Gr, phR) - np.einsum("cji,b->cbji", G, phL)
        D = np.linalg.solve(Mref, R.reshape(nc, nb, -1).transpose(1, 0, 2).reshape(nb, -1))
        return D.reshape(nb, nc, -1).transpose(1, 0, 2)
    # 2D
    V = np.zeros((nb, Q, Q))
    DX = np.zeros((nb, Q, Q))
    DY = np.zeros((nb, Q, Q))
    for I, (m, n) in enumerate(modes):
        V[I] = np.outer(Pg[m], Pg[n])
        DX[I] = np.outer(dPg[m], Pg[n]) * (2 / prob.hx)
        DY[I] = np.outer(Pg[m], dPg[n]) * (2 / prob.hy)
    W2 = np.outer(wg, wg) * prob.hx * prob.hy / 4
    q = np.einsum("cbji,bxy->cxyji", U, V)
    fx, fy = prob.flux(q, 0), prob.flux(q, 1)
    R -= np.einsum("xy,cxyji,bxy->cbji", W2, fx, DX) + np.einsum("xy,cxyji,bxy->cbji", W2, fy, DY)
    # face traces: x-faces at xi=+-1 (points along eta), y-faces at eta=+-1
    TXR = np.array([np.outer([P1[m]], Pg[n])[0] for (m, n) in modes])   # (nb, Q)
    TXL = np.array([np.outer([Pm1[m]], Pg[n])[0] for (m, n) in modes])
    TYT = np.array([Pg[m] * P1[n] for (m, n) in modes])
    TYB = np.array([Pg[m] * Pm1[n] for (m, n) in modes])
    tR = np.einsum("cbji,bp->cpji", U, TXR)
    tL = np.einsum("cbji,bp->cpji", U, TXL)
    tT = np.einsum("cbji,bp->cpji", U, TYT)
    tB = np.einsum("cbji,bp->cpji", U, TYB)
    wx = wg * prob.hy / 2
    wy = wg * prob.hx / 2
    if op == "loc":
        FR, FL = prob.flux(tR, 0), prob.flux(tL, 0)
        GT, GB = prob.flux(tT, 1), prob.flux(tB, 1)
    else:
        lft = np.roll(tR, 1, axis=3)
        bot = np.roll(tT, 1, axis=2)
        if prob.bc == "transmissive":
            lft[..., 0] = tL[..., 0]
            bot[:, :, 0, :] = tB[:, :, 0, :]
        FL = prob.lf(lft, tL, 0)
        GB = prob.lf(bot, tB, 1)
        FR = np.roll(FL, -1, axis=3)
        GT = np.roll(GB, -1, axis=2)
        if prob.bc == "transmissive":
            FR[..., -1] = prob.lf(tR[..., -1], tR[..., -1], 0)
            GT[:, :, -1, :] = prob.lf(tT[:, :, -1, :], tT[:, :, -1, :], 1)
    R += np.einsum("p,cpji,bp->cbji", wx, FR, TXR) - np.einsum("p,cpji,bp->cbji", wx, FL, TXL)
    R += np.einsum("p,cpji,bp->cbji", wy, GT, TYT) - np.einsum("p,cpji,bp->cbji", wy, GB, TYB)
    D = np.linalg.solve(Mref, R.reshape(nc, nb, -1).transpose(1, 0, 2).reshape(nb, -1))
    return D.reshape(nb, nc, -1).transpose(1, 0, 2)
