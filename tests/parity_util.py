"""Helpers shared by the GPU parity tests: one problem spec turned into the
oracle's parameters and the library's parameters, and paired runs."""
from __future__ import annotations

import dataclasses
import math
import sys

import numpy as np

import oracle


@dataclasses.dataclass
class Spec:
    Lx: int
    Ly: int
    tau: float = 0.8
    walls_x: bool = False
    walls_y: bool = False
    drag_const: bool = False
    d_p: float = math.inf
    K: float = math.inf
    F_eps: float = 0.0
    G: tuple = (0.0, 0.0)
    rho0: float = 1.0
    u0: tuple = (0.0, 0.0)
    storage: str = "f64"
    fp16_scale_log2: int = 10
    diag_every: int = 0
    open_x: bool = False
    inout: bool = False             # open x ends as velocity inlet / pressure outlet
    rho_in: float = 1.0
    u_in: float = 0.0
    rho_out: float = 1.0
    u_out: float = 0.0
    u_wall: tuple = (0.0, 0.0)      # sliding y-walls: x-velocity below, above
    sweep_vec: int = 0              # one-step sweep width (0 = automatic)
    steps_per_pass: int = 0         # most steps per pass: 0 = automatic (3), 1, 2, 3
    pass_rows: int = 0              # rows per chunk of the three-step pass: 0 = automatic

    def oracle(self) -> oracle.Params:
        return oracle.Params(Lx=self.Lx, Ly=self.Ly, tau=self.tau,
                             bc_x=(oracle.INOUT if self.inout else
                                   oracle.OPEN if self.open_x else
                                   oracle.WALL if self.walls_x else oracle.PERIODIC),
                             bc_y=oracle.WALL if self.walls_y else oracle.PERIODIC,
                             drag=oracle.DRAG_CONST if self.drag_const else oracle.DRAG_ERGUN,
                             d_p=self.d_p, K=self.K, F_eps=self.F_eps, Gx=self.G[0],
                             Gy=self.G[1], rho0=self.rho0, u0x=self.u0[0], u0y=self.u0[1],
                             rho_in=self.rho_in, u_in=self.u_in, rho_out=self.rho_out,
                             u_out=self.u_out, uw_bot=self.u_wall[0], uw_top=self.u_wall[1])

    def gpu(self):
        from paper_1406_6438_amd import lbm
        return lbm.Params(Lx=self.Lx, Ly=self.Ly, tau=self.tau,
                          bc_x=(lbm.BC_INOUT if self.inout else
                                lbm.BC_OPEN if self.open_x else
                                lbm.BC_BOUNCEBACK if self.walls_x else lbm.BC_PERIODIC),
                          bc_y=lbm.BC_BOUNCEBACK if self.walls_y else lbm.BC_PERIODIC,
                          storage=lbm.STORAGE[self.storage],
                          drag=lbm.DRAG_CONST if self.drag_const else lbm.DRAG_ERGUN,
                          d_p=self.d_p, K=self.K, F_eps=self.F_eps, G=tuple(self.G),
                          rho0=self.rho0, u0=tuple(self.u0),
                          fp16_scale_log2=self.fp16_scale_log2, diag_every=self.diag_every,
                          rho_in=self.rho_in, u_in=self.u_in, rho_out=self.rho_out,
                          u_out=self.u_out, u_wall=tuple(self.u_wall),
                          sweep_vec=self.sweep_vec, steps_per_pass=self.steps_per_pass,
                          pass_rows=self.pass_rows)

    def input_eps(self, eps: np.ndarray) -> np.ndarray:
        """The porosity both sides receive: rounded once to the GPU's compute precision."""
        if self.storage == "f64":
            return np.ascontiguousarray(eps, dtype=np.float64)
        return np.ascontiguousarray(eps, dtype=np.float32).astype(np.float64)


# Execution paths of lbm_vans_step: "auto" (the library's choice: on the small test
# grids the one-step sweep with one node per lane, as their widest sweep would have
# fewer tiles than the GPU has compute units), "triples" (three steps per pass in the
# default 24-row chunks), "short" and "tiny" (three steps per pass in 12-row and
# 6-row chunks: FP32 storage), "tall" (three steps per pass in 28-row chunks: FP32 storage; the FP16 pass
# has one height), "quads" (four steps per pass: FP32 storage), "pairs" (at most two
# steps per pass), "wide" (one step per pass,
# widest vector width) and "narrow" (one step per pass, one node per lane), so that
# the test grids cover every sweep kernel.
def exec_mode(mode: str, storage: str) -> dict:
    if mode == "auto":
        return {}
    if mode == "triples":
        return {"steps_per_pass": 3, "pass_rows": 24 if storage in ("f32", "f16") else 0}
    if mode == "short":
        return {"steps_per_pass": 3, "pass_rows": 12 if storage == "f32" else 0}
    if mode == "tiny":
        return {"steps_per_pass": 3, "pass_rows": 6 if storage == "f32" else 0}
    if mode == "tall":
        return {"steps_per_pass": 3, "pass_rows": 28 if storage == "f32" else 0}
    if mode == "quads":
        return {"steps_per_pass": 4}
    if mode == "pairs":
        return {"steps_per_pass": 2}
    if mode == "wide":
        return {"sweep_vec": 2 if storage == "f64" else 4, "steps_per_pass": 1}
    return {"sweep_vec": 1, "steps_per_pass": 1}


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def rel_l2(a, b) -> float:
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def gpu_run(spec: Spec, eps: np.ndarray, nsteps: int, f0: np.ndarray | None = None,
            keep: bool = False):
    """Run the GPU library; returns (moments dict as numpy, state f as numpy[, solver])."""
    from paper_1406_6438_amd import lbm
    s = lbm.Solver(spec.gpu(), spec.input_eps(eps))
    if f0 is not None:
        s.set_state(f0)
    s.step(nsteps)
    m = s.moments()
    out = {k: m[k].double().cpu().numpy() for k in ("eps_rho", "rho", "ux", "uy")}
    out["diag"] = m["diag"]
    out["rc"] = m["rc"]
    f = s.get_state().cpu().numpy()
    if keep:
        return out, f, s
    s.close()
    return out, f


def oracle_run(spec: Spec, eps: np.ndarray, nsteps: int, f0: np.ndarray | None = None):
    p = spec.oracle()
    e = spec.input_eps(eps)
    f = oracle.init(p, e) if f0 is None else np.array(f0, dtype=np.float64)
    f = oracle.steps(p, e, f, nsteps)
    return oracle.moments(p, e, f), f
