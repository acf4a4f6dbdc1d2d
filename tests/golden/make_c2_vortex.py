"""Write tests/golden/c2_vortex_256.json: the oracle's full run of the 2D
Euler isentropic vortex on 256 x 256 Q^2 cells to T = 1.

Calls only the oracle (oracle/) and the seeded input definitions
(paper_2307_06471_amd/workloads.py).  Scheme (eq:3) of Section 2.2, the
Lax--Friedrichs flux of Section 2.1, periodic boundaries, CFL 0.1 with a
fixed dt from the initial cell averages and the last step clipped to land on
T (the paper fixes dt from a CFL number, Section 4.1.2).  Stored:
  - dt, the number of steps and the last step;
  - the state of a seeded sample of cells (all 36 modal values each);
  - per (component, mode): the sum over cells and the sum of squares;
  - the conserved totals sum_K |K| ubar at t = 0 and at T;
  - L1 / L2 / Linf density errors against the exact translated vortex.
Takes about half an hour on one core:
    python tests/golden/make_c2_vortex.py
"""
import json
import math
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle as O  # noqa: E402
from paper_2307_06471_amd import workloads as W  # noqa: E402

OUT = os.path.join(HERE, "c2_vortex_256.json")
N_SAMPLE = 256


def sample_cells(nx, ny):
    rng = np.random.default_rng(256)
    fixed = [0, nx - 1, (ny - 1) * nx, nx * ny - 1, (ny // 2) * nx + nx // 2,
             (ny // 2) * nx + nx // 2 + 1, (ny // 2 + 1) * nx + nx // 2]
    rnd = rng.choice(nx * ny, N_SAMPLE - len(fixed), replace=False)
    return sorted(set(int(c) for c in fixed) | set(int(c) for c in rnd))


def main():
    cfg = W.config("c2")
    nx, ny, k = cfg["nx"], cfg["ny"], cfg["k"]
    x0, x1, y0, y1 = cfg["box"]
    om = O.Mesh(2, nx, ny, x0=x0, x1=x1, y0=y0, y1=y1, equation=O.EQ_EULER, gamma=W.GAMMA,
                flux=O.FLUX_LLF)
    A, b, c = (np.array(v, float) for v in W.TABLEAU[cfg["tableau"]])
    u = O.project(om, k, O.IC_VORTEX, cfg["ic_params"])
    tot0 = [O.total_mass(om, k, u, comp) for comp in range(4)]
    dt = cfg["cfl"] / O.max_wavespeed(om, k, u)
    T = cfg["T"]
    nsteps = int(math.ceil(T / dt - 1e-12))
    t = 0.0
    t0 = time.time()
    for n in range(nsteps):
        h = dt if n < nsteps - 1 else T - t
        u = O.step_crkdg(om, k, (A, b, c), t, h, u)
        t = t + h if n < nsteps - 1 else T
        if n % 50 == 0:
            print(f"step {n + 1}/{nsteps}, {time.time() - t0:.0f} s", flush=True)
    cells = sample_cells(nx, ny)
    err = O.errors(om, k, u, O.IC_VORTEX, cfg["ic_params"], t=T)
    out = {
        "source": "oracle run of the 2D Euler isentropic vortex (scheme eq:3, Section 2.2; "
                  "Lax-Friedrichs flux, Section 2.1), written by tests/golden/make_c2_vortex.py",
        "nx": nx, "ny": ny, "k": k, "T": T, "cfl": cfg["cfl"],
        "dt": dt, "steps": nsteps, "last_dt": T - (nsteps - 1) * dt,
        "cells": cells,
        "state": u[:, :, cells].transpose(2, 0, 1).tolist(),
        "sum": u.sum(axis=2).tolist(),
        "sumsq": (u * u).sum(axis=2).tolist(),
        "total_t0": tot0,
        "total_T": [O.total_mass(om, k, u, comp) for comp in range(4)],
        "errors_density": [float(e) for e in err],
        "oracle_seconds": round(time.time() - t0, 1),
    }
    with open(OUT + ".tmp", "w") as f:
        json.dump(out, f)
    os.replace(OUT + ".tmp", OUT)
    print(f"wrote {OUT}: {nsteps} steps, errors {err}")


if __name__ == "__main__":
    main()
