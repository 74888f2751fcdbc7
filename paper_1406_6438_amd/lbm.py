"""ctypes binding of liblbm_vans.so (declared in include/lbm_vans.h).

Argument marshalling only: every step of the method runs in the HIP kernels of
the library.  Device memory comes from torch tensors (the work buffer, the
porosity, output fields) and the HIP stream is torch's current stream.  The
module functions carry the C names; ``Solver`` is a small owner of one handle
and its work tensor.

The library is loaded from this package directory.  If it is missing the
import of the first entry point raises -- there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import dataclasses
import math
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liblbm_vans.so")

OK, EINVAL, EHIP, ENONFINITE, ENOTIMPL = 0, -1, -2, -3, -4
WMACH = 1                # warning: max |u| / c_s above MACH_WARN (the call completed)
MACH_WARN = 0.3
BC_PERIODIC, BC_BOUNCEBACK, BC_OPEN, BC_INOUT = 0, 1, 2, 3
F64, F32_SHIFTED, F16_SHIFTED = 0, 1, 2
DRAG_ERGUN, DRAG_CONST = 0, 1
NDIAG = 8
DIAG_RING = 4096
ABI_VERSION = 9

# Every symbol include/lbm_vans.h declares.
SYMBOLS = ("lbm_vans_work_bytes", "lbm_vans_init", "lbm_vans_step", "lbm_vans_step_count",
           "lbm_vans_pass_plan", "lbm_vans_batch_pass_plan", "lbm_vans_moments", "lbm_vans_get_state", "lbm_vans_set_state",
           "lbm_vans_diag_read", "lbm_vans_grad_work_bytes", "lbm_vans_grad",
           "lbm_vans_grad_static", "lbm_vans_objective",
           "lbm_vans_destroy", "lbm_vans_batch_work_bytes", "lbm_vans_batch_create",
           "lbm_vans_batch_configure", "lbm_vans_batch_get_config", "lbm_vans_batch_tune",
           "lbm_vans_batch_step", "lbm_vans_batch_grad_work_bytes", "lbm_vans_batch_grad",
           "lbm_vans_batch_destroy", "lbm_vans_last_error", "lbm_vans_abi_version")
OBJ_OUTLET_FLUX = 0

STORAGE = {"f64": F64, "f32": F32_SHIFTED, "f16": F16_SHIFTED}


class LbmVansParams(ctypes.Structure):
    _fields_ = [
        ("Lx", ctypes.c_int32), ("Ly", ctypes.c_int32),
        ("bc_x", ctypes.c_int32), ("bc_y", ctypes.c_int32),
        ("storage", ctypes.c_int32), ("drag", ctypes.c_int32),
        ("tau", ctypes.c_double), ("d_p", ctypes.c_double),
        ("K", ctypes.c_double), ("F_eps", ctypes.c_double),
        ("G", ctypes.c_double * 2), ("rho0", ctypes.c_double), ("u0", ctypes.c_double * 2),
        ("fp16_scale_log2", ctypes.c_int32), ("diag_every", ctypes.c_int32),
        ("rho_in", ctypes.c_double), ("u_in", ctypes.c_double),
        ("rho_out", ctypes.c_double), ("u_out", ctypes.c_double),
        ("u_wall", ctypes.c_double * 2),
        ("sweep_vec", ctypes.c_int32), ("steps_per_pass", ctypes.c_int32),
        ("pass_rows", ctypes.c_int32),
    ]


class LbmVansBatchConfig(ctypes.Structure):
    _fields_ = [("vec", ctypes.c_int32), ("grid", ctypes.c_int32),
                ("graph_steps", ctypes.c_int32), ("steps_per_pass", ctypes.c_int32),
                ("pass_rows", ctypes.c_int32), ("us_per_step", ctypes.c_double)]

    def as_dict(self) -> dict:
        return {"vec": self.vec, "grid": self.grid, "graph_steps": self.graph_steps,
                "steps_per_pass": self.steps_per_pass, "pass_rows": self.pass_rows,
                "us_per_step": self.us_per_step}


@dataclasses.dataclass
class Params:
    """Mirror of lbm_vans_params (see include/lbm_vans.h for every field)."""
    Lx: int
    Ly: int
    tau: float
    bc_x: int = BC_PERIODIC
    bc_y: int = BC_PERIODIC
    storage: int = F32_SHIFTED
    drag: int = DRAG_ERGUN
    d_p: float = math.inf
    K: float = math.inf
    F_eps: float = 0.0
    G: tuple = (0.0, 0.0)
    rho0: float = 1.0
    u0: tuple = (0.0, 0.0)
    fp16_scale_log2: int = 10
    diag_every: int = 0
    rho_in: float = 1.0
    u_in: float = 0.0
    rho_out: float = 1.0
    u_out: float = 0.0
    u_wall: tuple = (0.0, 0.0)
    sweep_vec: int = 0      # nodes per lane of the one-step sweep, 0 = automatic
    steps_per_pass: int = 0  # most steps per pass: 0 = automatic (3), 1, 2 or 3
    pass_rows: int = 0       # rows per chunk of the three-step pass: 0 = automatic, 6, 12, 24, 28

    def c(self) -> LbmVansParams:
        return LbmVansParams(self.Lx, self.Ly, self.bc_x, self.bc_y, self.storage, self.drag,
                             self.tau, self.d_p, self.K, self.F_eps,
                             (ctypes.c_double * 2)(*self.G), self.rho0,
                             (ctypes.c_double * 2)(*self.u0), self.fp16_scale_log2,
                             self.diag_every, self.rho_in, self.u_in, self.rho_out, self.u_out,
                             (ctypes.c_double * 2)(*self.u_wall), self.sweep_vec,
                             self.steps_per_pass, self.pass_rows)


class LbmVansError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"liblbm_vans error {code}: {msg}")
        self.code = code


_lib = None


def load(path: str = LIB_PATH):
    """Load the HIP library (raises if it is not built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} is not built; run __graft_entry__.build() "
                          "(python paper_1406_6438_amd/build.py)")
    L = ctypes.CDLL(path)
    P = ctypes.POINTER(LbmVansParams)
    vp, i32, i64, dp = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.POINTER(ctypes.c_double)
    L.lbm_vans_work_bytes.argtypes = [P]
    L.lbm_vans_work_bytes.restype = ctypes.c_size_t
    L.lbm_vans_init.argtypes = [P, vp, vp, ctypes.c_size_t, vp, ctypes.POINTER(vp)]
    L.lbm_vans_step.argtypes = [vp, i64]
    L.lbm_vans_step_count.argtypes = [vp]
    L.lbm_vans_step_count.restype = i64
    i32p = ctypes.POINTER(i32)
    L.lbm_vans_pass_plan.argtypes = [vp, i32p, i32p]
    L.lbm_vans_batch_pass_plan.argtypes = [vp, i32p, i32p]
    L.lbm_vans_moments.argtypes = [vp, vp, vp, vp, vp, dp]
    L.lbm_vans_get_state.argtypes = [vp, vp]
    L.lbm_vans_set_state.argtypes = [vp, vp]
    L.lbm_vans_diag_read.argtypes = [vp, dp, i32, ctypes.POINTER(i32)]
    L.lbm_vans_grad_work_bytes.argtypes = [P, i32, i64, i32]
    L.lbm_vans_grad_work_bytes.restype = ctypes.c_size_t
    L.lbm_vans_grad.argtypes = [vp, i32, i64, i32, vp, ctypes.c_size_t, vp, dp]
    L.lbm_vans_grad_static.argtypes = [vp, i32, i64, i32, vp, dp]
    L.lbm_vans_objective.argtypes = [vp, i32, dp]
    L.lbm_vans_destroy.argtypes = [vp]
    L.lbm_vans_destroy.restype = None
    C = ctypes.POINTER(LbmVansBatchConfig)
    L.lbm_vans_batch_work_bytes.argtypes = [ctypes.POINTER(vp), i32]
    L.lbm_vans_batch_work_bytes.restype = ctypes.c_size_t
    L.lbm_vans_batch_create.argtypes = [ctypes.POINTER(vp), i32, vp, ctypes.c_size_t, vp,
                                        ctypes.POINTER(vp)]
    L.lbm_vans_batch_configure.argtypes = [vp, C]
    L.lbm_vans_batch_get_config.argtypes = [vp, C]
    L.lbm_vans_batch_tune.argtypes = [vp, i32, C, C, i32, ctypes.POINTER(i32)]
    L.lbm_vans_batch_step.argtypes = [vp, i64]
    L.lbm_vans_batch_grad_work_bytes.argtypes = [vp, i32, i64, i32]
    L.lbm_vans_batch_grad_work_bytes.restype = ctypes.c_size_t
    L.lbm_vans_batch_grad.argtypes = [vp, i32, i64, i32, vp, ctypes.c_size_t,
                                      ctypes.POINTER(vp), dp]
    L.lbm_vans_batch_destroy.argtypes = [vp]
    L.lbm_vans_batch_destroy.restype = None
    L.lbm_vans_last_error.argtypes = []
    L.lbm_vans_last_error.restype = ctypes.c_char_p
    L.lbm_vans_abi_version.argtypes = []
    for n in ("lbm_vans_init", "lbm_vans_step", "lbm_vans_moments", "lbm_vans_get_state",
              "lbm_vans_set_state", "lbm_vans_diag_read", "lbm_vans_grad",
              "lbm_vans_grad_static", "lbm_vans_objective",
              "lbm_vans_batch_create", "lbm_vans_batch_configure", "lbm_vans_batch_get_config",
              "lbm_vans_batch_tune", "lbm_vans_batch_step", "lbm_vans_batch_grad",
              "lbm_vans_abi_version"):
        getattr(L, n).restype = ctypes.c_int
    if L.lbm_vans_abi_version() != ABI_VERSION:
        raise ImportError("liblbm_vans ABI version mismatch")
    _lib = L
    return L


def _check(rc: int):
    if rc != OK:
        raise LbmVansError(rc, load().lbm_vans_last_error().decode())
    return rc


def _dev_ptr(t) -> int | None:
    return None if t is None else t.data_ptr()


def lbm_vans_work_bytes(p: Params) -> int:
    n = load().lbm_vans_work_bytes(ctypes.byref(p.c()))
    if n == 0:
        raise LbmVansError(EINVAL, load().lbm_vans_last_error().decode())
    return n


def lbm_vans_init(p: Params, eps, work, stream) -> ctypes.c_void_p:
    h = ctypes.c_void_p()
    _check(load().lbm_vans_init(ctypes.byref(p.c()), eps.data_ptr(), work.data_ptr(),
                                work.numel() * work.element_size(), stream, ctypes.byref(h)))
    return h


def lbm_vans_step(h, nsteps: int):
    _check(load().lbm_vans_step(h, int(nsteps)))


def lbm_vans_step_count(h) -> int:
    return load().lbm_vans_step_count(h)


def lbm_vans_moments(h, eps_rho=None, rho=None, ux=None, uy=None, want_diag: bool = True):
    diag = (ctypes.c_double * NDIAG)() if want_diag else None
    rc = load().lbm_vans_moments(h, _dev_ptr(eps_rho), _dev_ptr(rho), _dev_ptr(ux),
                                 _dev_ptr(uy), diag)
    if rc in (ENONFINITE, WMACH):
        return np.array(diag[:]), rc
    _check(rc)
    return (np.array(diag[:]) if want_diag else None), rc


def lbm_vans_get_state(h, f):
    _check(load().lbm_vans_get_state(h, f.data_ptr()))


def lbm_vans_set_state(h, f):
    _check(load().lbm_vans_set_state(h, f.data_ptr()))


def lbm_vans_diag_read(h, max_records: int = DIAG_RING):
    buf = (ctypes.c_double * (NDIAG * max_records))()
    n = ctypes.c_int32()
    rc = load().lbm_vans_diag_read(h, buf, max_records, ctypes.byref(n))
    arr = np.array(buf[: n.value * NDIAG]).reshape(n.value, NDIAG)
    if rc not in (OK, ENONFINITE, WMACH):
        _check(rc)
    return arr, rc


def lbm_vans_grad_work_bytes(p: Params, objective: int, nsteps: int, ckpt_every: int) -> int:
    n = load().lbm_vans_grad_work_bytes(ctypes.byref(p.c()), objective, int(nsteps),
                                        int(ckpt_every))
    if n == 0:
        raise LbmVansError(EINVAL, load().lbm_vans_last_error().decode())
    return n


def lbm_vans_grad(h, objective: int, nsteps: int, ckpt_every: int, grad_work, dJdeps) -> float:
    J = ctypes.c_double()
    _check(load().lbm_vans_grad(h, objective, int(nsteps), int(ckpt_every), grad_work.data_ptr(),
                                grad_work.numel() * grad_work.element_size(), dJdeps.data_ptr(),
                                ctypes.byref(J)))
    return J.value


def lbm_vans_objective(h, objective: int = 0) -> float:
    """J of the current state (the outlet mass flux), on the device, no reverse sweep."""
    J = ctypes.c_double()
    _check(load().lbm_vans_objective(h, objective, ctypes.byref(J)))
    return J.value


def lbm_vans_grad_static(h, objective: int, nsteps: int, ckpt_every: int, dJdeps) -> float:
    """lbm_vans_grad in the library-held workspace (no caller buffer)."""
    J = ctypes.c_double()
    _check(load().lbm_vans_grad_static(h, objective, int(nsteps), int(ckpt_every),
                                       dJdeps.data_ptr(), ctypes.byref(J)))
    return J.value


GRAD_STATIC_BYTES = 64 << 20


def lbm_vans_destroy(h):
    if h:
        load().lbm_vans_destroy(h)


def _handles(members):
    arr = (ctypes.c_void_p * len(members))(*[m.h.value for m in members])
    return arr


def lbm_vans_batch_work_bytes(members) -> int:
    n = load().lbm_vans_batch_work_bytes(_handles(members), len(members))
    if n == 0:
        raise LbmVansError(EINVAL, "invalid batch members")
    return n


def lbm_vans_batch_create(members, work, stream) -> ctypes.c_void_p:
    b = ctypes.c_void_p()
    _check(load().lbm_vans_batch_create(_handles(members), len(members), work.data_ptr(),
                                        work.numel() * work.element_size(), stream,
                                        ctypes.byref(b)))
    return b


def lbm_vans_batch_configure(b, vec: int, grid: int, graph_steps: int, steps_per_pass: int = 0,
                             pass_rows: int = 0):
    c = LbmVansBatchConfig(vec, grid, graph_steps, steps_per_pass, pass_rows, 0.0)
    _check(load().lbm_vans_batch_configure(b, ctypes.byref(c)))


def lbm_vans_pass_plan(h) -> tuple:
    """(most steps per pass, rows per chunk of the three-step pass or 0) of a handle."""
    spp, rows = ctypes.c_int32(), ctypes.c_int32()
    _check(load().lbm_vans_pass_plan(h, ctypes.byref(spp), ctypes.byref(rows)))
    return spp.value, rows.value


def lbm_vans_batch_pass_plan(b) -> tuple:
    """lbm_vans_pass_plan for batched launches under the current configuration."""
    spp, rows = ctypes.c_int32(), ctypes.c_int32()
    _check(load().lbm_vans_batch_pass_plan(b, ctypes.byref(spp), ctypes.byref(rows)))
    return spp.value, rows.value


def lbm_vans_batch_get_config(b) -> dict:
    c = LbmVansBatchConfig()
    _check(load().lbm_vans_batch_get_config(b, ctypes.byref(c)))
    return c.as_dict()


def lbm_vans_batch_tune(b, reps: int = 5, max_trials: int = 64):
    best = LbmVansBatchConfig()
    trials = (LbmVansBatchConfig * max_trials)()
    n = ctypes.c_int32()
    _check(load().lbm_vans_batch_tune(b, int(reps), ctypes.byref(best), trials, max_trials,
                                      ctypes.byref(n)))
    return best.as_dict(), [trials[k].as_dict() for k in range(min(n.value, max_trials))]


def lbm_vans_batch_step(b, nsteps: int):
    _check(load().lbm_vans_batch_step(b, int(nsteps)))


def lbm_vans_batch_grad_work_bytes(b, objective: int, nsteps: int, ckpt_every: int) -> int:
    n = load().lbm_vans_batch_grad_work_bytes(b, objective, int(nsteps), int(ckpt_every))
    if n == 0:
        raise LbmVansError(EINVAL, load().lbm_vans_last_error().decode())
    return n


def lbm_vans_batch_grad(b, objective: int, nsteps: int, ckpt_every: int, grad_work, dJdeps):
    ptrs = (ctypes.c_void_p * len(dJdeps))(*[g.data_ptr() for g in dJdeps])
    J = (ctypes.c_double * len(dJdeps))()
    _check(load().lbm_vans_batch_grad(b, objective, int(nsteps), int(ckpt_every),
                                      grad_work.data_ptr(),
                                      grad_work.numel() * grad_work.element_size(), ptrs, J))
    return list(J)


def lbm_vans_batch_destroy(b):
    if b:
        load().lbm_vans_batch_destroy(b)


class Solver:
    """One solver handle with torch-owned device memory on ``device``.

    ``eps`` is the porosity [Ly, Lx] (numpy or torch); it is cast once to the
    compute type of the storage (float64 for f64, float32 otherwise) and
    uploaded.  All calls run on torch's current stream of ``device``.
    """

    def __init__(self, p: Params, eps, device="cuda:0"):
        import torch

        load()
        self.torch = torch
        self.p = p
        self.device = torch.device(device)
        self.real = torch.float64 if p.storage == F64 else torch.float32
        eps_t = torch.as_tensor(np.asarray(eps) if not isinstance(eps, torch.Tensor) else eps)
        if tuple(eps_t.shape) != (p.Ly, p.Lx):
            raise ValueError(f"eps has shape {tuple(eps_t.shape)}, expected {(p.Ly, p.Lx)}")
        with torch.cuda.device(self.device):
            self.eps = eps_t.to(dtype=self.real).contiguous().to(self.device)
            nbytes = lbm_vans_work_bytes(p)
            # 256-byte aligned: torch's caching allocator returns >= 512-byte aligned blocks.
            self.work = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
            assert self.work.data_ptr() % 256 == 0
            self.stream = torch.cuda.current_stream(self.device)
            self.h = lbm_vans_init(p, self.eps, self.work, self.stream.cuda_stream)

    def step(self, nsteps: int):
        lbm_vans_step(self.h, nsteps)

    @property
    def n(self) -> int:
        return lbm_vans_step_count(self.h)

    @property
    def pass_plan(self) -> tuple:
        """(most steps per pass, rows per chunk of the three-step pass or 0)."""
        return lbm_vans_pass_plan(self.h)

    def moments(self, want_diag: bool = True):
        """dict of eps_rho, rho, ux, uy tensors [Ly, Lx] and the diagnostics record."""
        t = self.torch
        out = {k: t.empty((self.p.Ly, self.p.Lx), dtype=self.real, device=self.device)
               for k in ("eps_rho", "rho", "ux", "uy")}
        diag, rc = lbm_vans_moments(self.h, out["eps_rho"], out["rho"], out["ux"], out["uy"],
                                    want_diag)
        out["diag"] = diag
        out["rc"] = rc
        return out

    def get_state(self):
        f = self.torch.empty((9, self.p.Ly, self.p.Lx), dtype=self.torch.float64,
                             device=self.device)
        lbm_vans_get_state(self.h, f)
        return f

    def set_state(self, f):
        f = self.torch.as_tensor(f, dtype=self.torch.float64).contiguous().to(self.device)
        if tuple(f.shape) != (9, self.p.Ly, self.p.Lx):
            raise ValueError("state must be [9, Ly, Lx]")
        lbm_vans_set_state(self.h, f)
        self.stream.synchronize()

    def diag_records(self):
        return lbm_vans_diag_read(self.h)

    def grad(self, nsteps: int, ckpt_every: int = 200, objective: int = OBJ_OUTLET_FLUX):
        """(J, dJ/deps as a float64 tensor [Ly, Lx]) of the objective after nsteps steps
        from the initial state (reverse sweep with a checkpoint every ckpt_every steps).
        The solver's state is f(., nsteps) afterwards."""
        t = self.torch
        nbytes = lbm_vans_grad_work_bytes(self.p, objective, nsteps, ckpt_every)
        with t.cuda.device(self.device):
            gw = t.empty(nbytes, dtype=t.uint8, device=self.device)
            g = t.empty((self.p.Ly, self.p.Lx), dtype=t.float64, device=self.device)
            J = lbm_vans_grad(self.h, objective, nsteps, ckpt_every, gw, g)
            del gw
        return J, g

    def close(self):
        if getattr(self, "h", None):
            lbm_vans_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch:
    """Many Solvers advanced together by batched launches (one per vector width
    present, per step; captured into graphs).  The members stay usable as
    Solvers (moments, get_state) between batch calls; all calls run on torch's
    current stream of the members' device."""

    def __init__(self, members):
        import torch

        self.torch = torch
        self.members = list(members)
        if not self.members:
            raise ValueError("no members")
        self.device = self.members[0].device
        with torch.cuda.device(self.device):
            nbytes = lbm_vans_batch_work_bytes(self.members)
            self.work = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
            self.stream = torch.cuda.current_stream(self.device)
            self.b = lbm_vans_batch_create(self.members, self.work, self.stream.cuda_stream)

    def configure(self, vec: int, grid: int = 0, graph_steps: int = 24, steps_per_pass: int = 0,
                  pass_rows: int = 0):
        """steps_per_pass: most steps per launch (0 = automatic: 4 or 3 with FP32
        storage, 3 with FP16; 1, 2, 3, or 4 with FP32); pass_rows: rows per chunk of the
        three-step pass (0 = automatic; 24 or 28 with FP32 storage)."""
        lbm_vans_batch_configure(self.b, vec, grid, graph_steps, steps_per_pass, pass_rows)

    @property
    def config(self) -> dict:
        return lbm_vans_batch_get_config(self.b)

    @property
    def pass_plan(self) -> tuple:
        """(most steps per launch, rows per chunk of the three-step pass or 0)."""
        return lbm_vans_batch_pass_plan(self.b)

    def tune(self, reps: int = 5):
        """Autotune the launch shape; returns (best, all trials) as dicts."""
        return lbm_vans_batch_tune(self.b, reps)

    def step(self, nsteps: int):
        lbm_vans_batch_step(self.b, nsteps)

    def grad(self, nsteps: int, ckpt_every: int, objective: int = OBJ_OUTLET_FLUX):
        """(list of J, list of float64 dJ/deps tensors) for every member."""
        t = self.torch
        nbytes = lbm_vans_batch_grad_work_bytes(self.b, objective, nsteps, ckpt_every)
        with t.cuda.device(self.device):
            gw = t.empty(nbytes, dtype=t.uint8, device=self.device)
            gs = [t.empty((m.p.Ly, m.p.Lx), dtype=t.float64, device=self.device)
                  for m in self.members]
            J = lbm_vans_batch_grad(self.b, objective, nsteps, ckpt_every, gw, gs)
            del gw
        return J, gs

    def close(self):
        if getattr(self, "b", None):
            lbm_vans_batch_destroy(self.b)
            self.b = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def outlet_flux_function():
    """A torch.autograd.Function: J = OutletFlux.apply(eps, params, nsteps, ckpt_every)
    gives the outlet mass flux after nsteps steps and backpropagates dJ/deps computed by
    the library's reverse sweep."""
    import torch

    class OutletFlux(torch.autograd.Function):
        @staticmethod
        def forward(ctx, eps, params, nsteps, ckpt_every):
            s = Solver(params, eps.detach(), device=eps.device if eps.is_cuda else "cuda:0")
            if not ctx.needs_input_grad[0]:
                # no gradient wanted: the forward steps and J only, no reverse sweep
                s.step(nsteps)
                J = lbm_vans_objective(s.h, OBJ_OUTLET_FLUX)
                s.close()
                return torch.tensor(J, dtype=torch.float64, device=eps.device)
            J, g = s.grad(nsteps, ckpt_every, OBJ_OUTLET_FLUX)
            s.close()
            ctx.save_for_backward(g)
            ctx.eps_dtype, ctx.eps_device = eps.dtype, eps.device
            return torch.tensor(J, dtype=torch.float64, device=eps.device)

        @staticmethod
        def backward(ctx, gJ):
            (g,) = ctx.saved_tensors
            grad = (g * gJ.to(g.device, torch.float64)).to(ctx.eps_device, ctx.eps_dtype)
            return grad, None, None, None

    return OutletFlux
