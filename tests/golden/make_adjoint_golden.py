"""Writes tests/golden/adjoint_channel_1024x512.json: the oracle's outlet mass flux J of
the 1024 x 512 open porous channel after 4000 steps and central differences of J with
respect to the porosity at six seeded nodes (h = 1e-5), all in FP64.  Calls only the
oracle; inputs come from paper_1406_6438_amd.workloads.

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


def params(w):
    U = W.ADJOINT_U_IN
    return oracle.Params(Lx=w.Lx, Ly=w.Ly, tau=w.tau, bc_x=oracle.OPEN, bc_y=oracle.WALL,
                         d_p=w.d_p, rho0=w.rho0, u0x=U, rho_in=1.0, u_in=U, rho_out=1.0,
                         u_out=U)


def main():
    threads = int(sys.argv[1]) if len(sys.argv) > 1 else oracle.default_threads()
    w = W.ADJOINT_CHANNEL
    eps = w.porosity().astype(np.float32).astype(np.float64)
    p = params(w)
    rng = np.random.Generator(np.random.PCG64(20260))
    cells = [(int(rng.integers(0, w.Ly)), int(rng.integers(w.Lx - 40, w.Lx))) for _ in range(4)]
    cells += [(int(rng.integers(0, w.Ly)), int(rng.integers(0, w.Lx))) for _ in range(2)]
    h = 1e-5

    def J(e):
        t = time.time()
        v = oracle.outlet_flux(p, e, oracle.run(p, e, w.steps, threads))
        print(f"  J = {v:.15e} ({time.time() - t:.0f} s)", flush=True)
        return v

    J0 = J(eps)
    fd = []
    for (y, x) in cells:
        e = eps.copy()
        e[y, x] += h
        jp = J(e)
        e[y, x] -= 2 * h
        jm = J(e)
        fd.append((jp - jm) / (2 * h))
        print(f"cell (y={y}, x={x}): dJ/deps ~ {fd[-1]:.9e}", flush=True)
    json.dump({"workload": w.name, "steps": w.steps, "J": J0, "h": h,
               "cells_yx": cells, "dJdeps_central_difference": fd,
               "note": "oracle FP64; porosity rounded to FP32 as the GPU receives it"},
              open(OUT, "w"), indent=1)
    print("wrote", OUT)


if __name__ == "__main__":
    main()
