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
