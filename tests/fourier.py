"""von Neumann analysis of the 1D DG operators for u_t + u_x = 0 with the
upwind flux on a uniform periodic mesh (Section 1, Table 'tab:CFL';
the method of analysis is the one the paper names there).

The dimensionless cell blocks are built from exact Legendre integrals with
numpy (independent of the oracle):
  h D_DG u_j  = diag(2m+1) [ (-S + 1 1^T) u_j - e_L 1^T u_{j-1} ]
  h D_loc u_j = diag(2m+1) [ (-S + 1 1^T - e_L e_L^T) u_j ]
with S_ml = int_{-1}^{1} P_l P_m' and (e_L)_m = P_m(-1) = (-1)^m.
"""
import numpy as np
from numpy.polynomial import legendre as npleg


def blocks(k):
    xg, wg = npleg.leggauss(k + 4)
    P = np.array([npleg.legval(xg, np.eye(k + 1)[m]) for m in range(k + 1)])
    dP = np.array([npleg.legval(xg, npleg.legder(np.eye(k + 1)[m])) if m else 0 * xg
                   for m in range(k + 1)])
    S = np.einsum("a,ma,la->ml", wg, dP, P)
    one = np.ones(k + 1)
    eL = (-1.0) ** np.arange(k + 1)
    scale = np.diag(2 * np.arange(k + 1) + 1.0)
    B0 = scale @ (-S + np.outer(one, one))
    B1 = scale @ (-np.outer(eL, one))
    Bloc = scale @ (-S + np.outer(one, one) - np.outer(eL, eL))
    return B0, B1, Bloc


def symbols(k, theta):
    B0, B1, Bloc = blocks(k)
    return B0 + np.exp(-1j * theta) * B1, Bloc.astype(complex)


def amplification(k, theta, nu, tableau, scheme="crkdg"):
    """G(theta) of one step for a Butcher tableau (A, b, c); nu = dt/h"""
    A, b, _ = tableau
    Adg, Aloc = symbols(k, theta)
    inner = Aloc if scheme == "crkdg" else Adg
    s = len(b)
    I = np.eye(k + 1, dtype=complex)
    U = []
    for i in range(s):
        Ui = I.copy()
        for j in range(i):
            if A[i][j] != 0.0:
                Ui = Ui - nu * A[i][j] * (inner @ U[j])
        U.append(Ui)
    G = I.copy()
    for i in range(s):
        if b[i] != 0.0:
            G = G - nu * b[i] * (Adg @ U[i])
    return G


def spectral_radius_max(k, nu, tableau, scheme, nth=721):
    r = 0.0
    for th in np.linspace(0, 2 * np.pi, nth):
        r = max(r, np.abs(np.linalg.eigvals(amplification(k, th, nu, tableau, scheme))).max())
    return r


def max_cfl(k, tableau, scheme, lo=0.01, hi=1.0, tol=1e-5):
    while hi - lo > tol:
        mid = 0.5 * (lo + hi)
        if spectral_radius_max(k, mid, tableau, scheme) <= 1.0 + 1e-10:
            lo = mid
        else:
            hi = mid
    return lo


def evolve_periodic(k, u0, nu, tableau, nsteps, scheme="crkdg"):
    """exact discrete evolution of modal data u0[(k+1), N] by block-circulant
    diagonalisation: DFT over cells, G(theta)^n per wavenumber, inverse DFT"""
    N = u0.shape[1]
    c = np.fft.fft(u0, axis=1)
    out = np.zeros_like(c)
    for kap in range(N):
        th = 2 * np.pi * kap / N
        G = amplification(k, th, nu, tableau, scheme)
        out[:, kap] = np.linalg.matrix_power(G, nsteps) @ c[:, kap]
    return np.real(np.fft.ifft(out, axis=1))
