"""Writes tests/golden/adjoint_channel_1024x512.json: the oracle's outlet mass flux J of
the 1024 x 512 porous channel (velocity inlet, pressure outlet) after 4000 steps and
central differences of J with respect to the porosity at 32 seeded random nodes of the
whole channel, each with two step sizes (h and 2h) so that the differences' own
uncertainty (rounding noise ~ 1/h, truncation ~ h^2) can be read off, all in FP64.
Calls only the oracle; inputs come from paper_1406_6438_amd.workloads.

    python tests/golden/make_adjoint_golden.py [threads]
"""
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_1406_6438_amd import workloads as W  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "adjoint_channel_1024x512.json")
NCELLS = 32
H = 1e-4


def params(w):
    U = W.ADJOINT_U_IN
    return oracle.Params(Lx=w.Lx, Ly=w.Ly, tau=w.tau, bc_x=oracle.INOUT, bc_y=oracle.WALL,
                         d_p=w.d_p, rho0=w.rho0, u0x=U, u_in=U, rho_out=W.ADJOINT_RHO_OUT)


def cells_of(w, eps):
    """32 nodes drawn uniformly over the channel (PCG64 seed 20260); a node whose porosity
    lies within 2h of 1 is skipped (the Ergun drag vanishes at eps = 1 and is not smooth
    there)."""
    rng = np.random.Generator(np.random.PCG64(20260))
    out = []
    while len(out) < NCELLS:
        y, x = int(rng.integers(0, w.Ly)), int(rng.integers(0, w.Lx))
        if eps[y, x] + 2 * H < 1.0 and (y, x) not in out:
            out.append((y, x))
    return out


def main():
    threads = int(sys.argv[1]) if len(sys.argv) > 1 else oracle.default_threads()
    w = W.ADJOINT_CHANNEL
    eps = w.porosity().astype(np.float32).astype(np.float64)
    p = params(w)
    cells = cells_of(w, eps)

    def J(e):
        t = time.time()
        v = oracle.outlet_flux(p, e, oracle.run(p, e, w.steps, threads))
        print(f"  J = {v:.15e} ({time.time() - t:.0f} s)", flush=True)
        return v

    J0 = J(eps)
    fd = {H: [], 2 * H: []}
    for (y, x) in cells:
        for h in (H, 2 * H):
            e = eps.copy()
            e[y, x] += h
            jp = J(e)
            e[y, x] -= 2 * h
            jm = J(e)
            fd[h].append((jp - jm) / (2 * h))
        print(f"cell (y={y}, x={x}): dJ/deps ~ {fd[H][-1]:.12e} (2h: {fd[2 * H][-1]:.12e})",
              flush=True)
    json.dump({"workload": w.name, "boundaries": "velocity inlet u_in=0.02, pressure outlet "
                                                  "rho_out=1, bounce-back walls in y",
               "steps": w.steps, "J": J0, "h": H, "cells_yx": cells,
               "dJdeps_central_difference": fd[H], "dJdeps_central_difference_2h": fd[2 * H],
               "note": "oracle FP64; porosity rounded to FP32 as the GPU receives it"},
              open(OUT, "w"), indent=1)
    print("wrote", OUT)


if __name__ == "__main__":
    main()
