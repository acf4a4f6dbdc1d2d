"""Build the oracle's and the library's description of the same workload."""
import numpy as np

import oracle as O
from paper_2307_06471_amd import workloads as W

BC = {"periodic": 0, "transmissive": 1, "dirichlet": 2}


def tableau(name):
    A, b, c = W.TABLEAU[name]
    return (np.array(A, float), np.array(b, float), np.array(c, float))


def oracle_mesh(cfg, bc_state=None, bc_exact=0, ic_params=None):
    x0, x1, y0, y1 = cfg["box"]
    eq = O.EQ_EULER if cfg["equation"] == "euler" else O.EQ_ADVECTION
    flux = O.FLUX_LLF if cfg["flux"] == "llf" else O.FLUX_UPWIND
    return O.Mesh(cfg["dim"], cfg["nx"], cfg["ny"], x0=x0, x1=x1, y0=y0, y1=y1,
                  bc=tuple(BC[b] for b in cfg["bc"]), bc_state=bc_state, bc_exact=bc_exact,
                  ic_params=ic_params, equation=eq, adv=cfg.get("adv", (1.0, 0.0)),
                  gamma=W.GAMMA, flux=flux)


def lib_mesh(cfg, bc_state=None, bc_exact=0, precision=0):
    from paper_2307_06471_amd import crkdg as K
    x0, x1, y0, y1 = cfg["box"]
    eq = K.EQ_EULER if cfg["equation"] == "euler" else K.EQ_ADVECTION
    return K.make_mesh(cfg["dim"], cfg["nx"], cfg["ny"], x0=x0, x1=x1, y0=y0, y1=y1,
                       bc=tuple(BC[b] for b in cfg["bc"]), bc_state=bc_state, bc_exact=bc_exact,
                       equation=eq, adv=cfg.get("adv", (1.0, 0.0)), gamma=W.GAMMA,
                       precision=precision)


def lib_flux(cfg):
    from paper_2307_06471_amd import crkdg as K
    return K.FLUX_LLF if cfg["flux"] == "llf" else K.FLUX_UPWIND


def rel_err(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    return float(np.abs(a - b).max() / max(1e-300, np.abs(b).max()))


U32 = 2.0 ** -24  # unit roundoff of binary32


def _gamma(n):
    return n * U32 / (1.0 - n * U32)


def mlp_fp32_bound(P, X, safety=2.0):
    """per-sample bound on |z_fp32 - z_fp64| for the 12 -> 32 -> 32 -> 1 ReLU
    network evaluated in binary32 (any summation order, fused or not) on
    features rounded to binary32, against the binary64 network on the
    unrounded features.  Standard forward error analysis: a sum of n terms
    carries at most gamma_n = n u / (1 - n u) times the sum of the terms'
    magnitudes; ReLU is 1-Lipschitz; rounding the features costs u |x| per
    feature (2 u allowed: the two sides also compute the features in a
    different FP64 order).  Returns safety x the bound, from the absolute
    weights and the binary64 activations."""
    P = np.asarray(P, dtype=np.float64)
    X = np.atleast_2d(np.asarray(X, dtype=np.float64))
    W1 = P[:384].reshape(32, 12)
    b1 = P[384:416]
    W2 = P[416:1440].reshape(32, 32)
    b2 = P[1440:1472]
    w3 = P[1472:1504]
    b3 = P[1504]
    A1 = np.abs(X) @ np.abs(W1).T                      # sum |W1| |x|
    h1 = np.maximum(X @ W1.T + b1, 0.0)
    e1 = _gamma(13) * (A1 * (1 + 2 * U32) + np.abs(b1)) + 2 * U32 * A1
    e2 = e1 @ np.abs(W2).T + _gamma(33) * ((h1 + e1) @ np.abs(W2).T + np.abs(b2))
    h2 = np.maximum(h1 @ W2.T + b2, 0.0)
    ez = e2 @ np.abs(w3) + _gamma(34) * ((h2 + e2) @ np.abs(w3) + abs(b3))
    return safety * ez
