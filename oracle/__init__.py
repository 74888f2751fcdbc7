"""FP64 CPU oracle of the volume-averaged lattice Boltzmann model (arXiv:1406.6438).

TEST INFRASTRUCTURE ONLY.  Only the test suite, ``__graft_entry__.smoke()`` and
the CPU-baseline leg of ``bench.py`` may import this package.  It shares no code
with the GPU library; the two meet only through the seeded input generators of
``paper_1406_6438_amd.workloads``, which hold none of the method's arithmetic.

The arithmetic lives in ``lbm_vans_oracle.c`` (plain loops, IEEE binary64, no
FMA contraction).  This module is argument marshalling around it:

* ``feq``            -- equilibrium, eq. (d2q9eq)
* ``guo_source``     -- P_i / F_i form, eqs. (pi) and (Fi)
* ``drag_coeffs``    -- Darcy-Forchheimer drag with the Ergun closure
                        (Section "Examples and discussions")
* ``velocity``       -- implicit velocity of eq. (1moment), solved exactly
* ``grad_eps``       -- lattice gradient of the porosity
* ``init``           -- f(x, 0) = f^eq(eps(x) rho0, u0)
* ``collide`` / ``stream`` / ``steps`` -- one or more time steps of the final
                        lattice Boltzmann equation (collide, then push)
* ``open_ends``      -- the boundary state a velocity inlet / pressure outlet
                        builds the next entering populations from
* ``moments``        -- eps rho, rho, u, m = sum e_i f_i and T per cell
* ``outlet_flux`` / ``grad_outlet_flux`` -- J = sum of eps rho u_x over the last
                        column, and dJ/deps by the reverse (adjoint) of the steps
"""
from __future__ import annotations

import ctypes
import dataclasses
import math
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "lbm_vans_oracle.c")
_LIB = os.path.join(_HERE, "liblbm_vans_oracle.so")
# The mutation tests point this at a deliberately broken build of the oracle.
_LIB_OVERRIDE = os.environ.get("LBM_VANS_ORACLE_LIB")

PERIODIC = 0
WALL = 1
OPEN = 2
INOUT = 3           # velocity inlet at x = 0, pressure outlet at x = Lx-1
DRAG_ERGUN = 0
DRAG_CONST = 1

# Build flags of the oracle: no FMA contraction and no fast-math, so every
# operation is one correctly rounded binary64 operation.
CFLAGS = ["-O3", "-std=c11", "-fPIC", "-shared", "-ffp-contract=off", "-fno-fast-math",
          "-fopenmp", "-Wall", "-Wextra"]


def build(force: bool = True) -> str:
    """Compile the oracle with gcc into ``oracle/liblbm_vans_oracle.so``."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", *CFLAGS, "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class _Params(ctypes.Structure):
    _fields_ = [
        ("Lx", ctypes.c_int32), ("Ly", ctypes.c_int32),
        ("bc_x", ctypes.c_int32), ("bc_y", ctypes.c_int32),
        ("drag", ctypes.c_int32), ("pad_", ctypes.c_int32),
        ("tau", ctypes.c_double), ("d_p", ctypes.c_double),
        ("K", ctypes.c_double), ("F_eps", ctypes.c_double),
        ("Gx", ctypes.c_double), ("Gy", ctypes.c_double),
        ("rho0", ctypes.c_double), ("u0x", ctypes.c_double), ("u0y", ctypes.c_double),
        ("rho_in", ctypes.c_double), ("u_in", ctypes.c_double),
        ("rho_out", ctypes.c_double), ("u_out", ctypes.c_double),
        ("uw_bot", ctypes.c_double), ("uw_top", ctypes.c_double),
    ]


@dataclasses.dataclass
class Params:
    """Problem description: lattice size, boundaries, tau, drag law, body force, initial state."""
    Lx: int
    Ly: int
    tau: float
    bc_x: int = PERIODIC
    bc_y: int = PERIODIC
    drag: int = DRAG_ERGUN
    d_p: float = math.inf
    K: float = math.inf
    F_eps: float = 0.0
    Gx: float = 0.0
    Gy: float = 0.0
    rho0: float = 1.0
    u0x: float = 0.0
    u0y: float = 0.0
    rho_in: float = 1.0
    u_in: float = 0.0
    rho_out: float = 1.0
    u_out: float = 0.0
    uw_bot: float = 0.0     # WALL in y: x-velocity of the lower plate (sliding wall)
    uw_top: float = 0.0     # WALL in y: x-velocity of the upper plate

    def c(self) -> _Params:
        return _Params(self.Lx, self.Ly, self.bc_x, self.bc_y, self.drag, 0, self.tau,
                       self.d_p, self.K, self.F_eps, self.Gx, self.Gy, self.rho0,
                       self.u0x, self.u0y, self.rho_in, self.u_in, self.rho_out, self.u_out,
                       self.uw_bot, self.uw_top)


_lib = None
_D = ctypes.POINTER(ctypes.c_double)
_I = ctypes.POINTER(ctypes.c_int32)


def lib():
    global _lib
    if _lib is None:
        if _LIB_OVERRIDE:
            L = ctypes.CDLL(_LIB_OVERRIDE)
        else:
            if not os.path.exists(_LIB):
                build(force=True)
            L = ctypes.CDLL(_LIB)
        P = ctypes.POINTER(_Params)
        L.orc_lattice.argtypes = [_I, _I, _D, _I, _D]
        L.orc_feq.argtypes = [ctypes.c_double] * 3 + [_D]
        L.orc_guo_source.argtypes = [ctypes.c_double] * 5 + [_D]
        L.orc_drag_coeffs.argtypes = [P, ctypes.c_double, _D, _D]
        L.orc_velocity.argtypes = [P] + [ctypes.c_double] * 6 + [_D, _D, _D]
        L.orc_grad_eps.argtypes = [P, _D, _D, _D]
        L.orc_init.argtypes = [P, _D, _D]
        L.orc_collide.argtypes = [P, _D, _D, _D, _D, _D, ctypes.c_int]
        L.orc_open_ends.argtypes = [P, _D, _D, _D, _D, _D]
        L.orc_stream.argtypes = [P, _D, _D, _D, _D, ctypes.c_int]
        L.orc_steps.argtypes = [P, _D, _D, _D, _D, _D, ctypes.c_int64, ctypes.c_int]
        L.orc_steps.restype = ctypes.c_int
        L.orc_moments.argtypes = [P, _D, _D, _D, _D] + [_D] * 8
        L.orc_drag_derivs.argtypes = [P, ctypes.c_double, _D, _D]
        L.orc_node_collide.argtypes = [P, _D] + [ctypes.c_double] * 3 + [_D]
        L.orc_node_collide.restype = None
        L.orc_node_vjp.argtypes = ([P, _D] + [ctypes.c_double] * 3 + [_D] +
                                   [ctypes.c_double] * 3 + [_D, _D, _D, _D])
        L.orc_outlet_flux.argtypes = [P, _D, _D, _D, _D]
        L.orc_outlet_flux.restype = ctypes.c_double
        L.orc_grad_outlet_flux.argtypes = [P, _D, ctypes.c_int64, _D, _D, ctypes.c_int]
        L.orc_grad_outlet_flux.restype = ctypes.c_int
        for name in ("orc_drag_derivs", "orc_node_vjp"):
            getattr(L, name).restype = None
        for name in ("orc_lattice", "orc_feq", "orc_guo_source", "orc_drag_coeffs",
                     "orc_velocity", "orc_grad_eps", "orc_init", "orc_collide",
                     "orc_open_ends", "orc_stream", "orc_moments"):
            getattr(L, name).restype = None
        _lib = L
    return _lib


def _ptr(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(_D)


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


def default_threads() -> int:
    env = os.environ.get("OMP_NUM_THREADS")
    if env and env.isdigit() and int(env) > 0:
        return int(env)
    return max(1, min(16, os.cpu_count() or 1))


def lattice():
    """D2Q9 tables used by the oracle: (ex, ey, w, opp, cs2)."""
    ex = (ctypes.c_int32 * 9)()
    ey = (ctypes.c_int32 * 9)()
    w = (ctypes.c_double * 9)()
    opp = (ctypes.c_int32 * 9)()
    cs2 = ctypes.c_double()
    lib().orc_lattice(ex, ey, w, opp, ctypes.byref(cs2))
    return (np.array(ex[:]), np.array(ey[:]), np.array(w[:]), np.array(opp[:]), cs2.value)


def feq(eps_rho: float, ux: float, uy: float) -> np.ndarray:
    out = np.zeros(9)
    lib().orc_feq(eps_rho, ux, uy, _ptr(out))
    return out


def guo_source(tau: float, ux: float, uy: float, Tx: float, Ty: float) -> np.ndarray:
    out = np.zeros(9)
    lib().orc_guo_source(tau, ux, uy, Tx, Ty, _ptr(out))
    return out


def drag_coeffs(p: Params, eps: float):
    a = ctypes.c_double()
    b = ctypes.c_double()
    lib().orc_drag_coeffs(ctypes.byref(p.c()), eps, ctypes.byref(a), ctypes.byref(b))
    return a.value, b.value


def velocity(p: Params, S: float, mx: float, my: float, eps: float, gex: float, gey: float):
    """(ux, uy, rho) from eq. (1moment) for one cell."""
    ux = ctypes.c_double()
    uy = ctypes.c_double()
    rho = ctypes.c_double()
    lib().orc_velocity(ctypes.byref(p.c()), S, mx, my, eps, gex, gey, ctypes.byref(ux),
                       ctypes.byref(uy), ctypes.byref(rho))
    return ux.value, uy.value, rho.value


def grad_eps(p: Params, eps: np.ndarray):
    eps = _f64(eps)
    assert eps.shape == (p.Ly, p.Lx)
    gx = np.empty_like(eps)
    gy = np.empty_like(eps)
    lib().orc_grad_eps(ctypes.byref(p.c()), _ptr(eps), _ptr(gx), _ptr(gy))
    return gx, gy


def init(p: Params, eps: np.ndarray) -> np.ndarray:
    """f(x, 0) as an array [9, Ly, Lx]."""
    eps = _f64(eps)
    assert eps.shape == (p.Ly, p.Lx)
    f = np.empty((9, p.Ly, p.Lx))
    lib().orc_init(ctypes.byref(p.c()), _ptr(eps), _ptr(f))
    return f


def collide(p: Params, eps: np.ndarray, f: np.ndarray, threads: int | None = None):
    eps = _f64(eps)
    f = _f64(f)
    gx, gy = grad_eps(p, eps)
    out = np.empty_like(f)
    lib().orc_collide(ctypes.byref(p.c()), _ptr(eps), _ptr(gx), _ptr(gy), _ptr(f),
                      _ptr(out), threads or default_threads())
    return out


def open_ends(p: Params, eps: np.ndarray, f: np.ndarray) -> np.ndarray:
    """Velocity inlet / pressure outlet: per row, eps rho of the inlet node and the
    velocity of the outlet node of the state f, as an array [Ly, 3]."""
    eps = _f64(eps)
    f = _f64(f)
    gx, gy = grad_eps(p, eps)
    ends = np.empty((p.Ly, 3))
    lib().orc_open_ends(ctypes.byref(p.c()), _ptr(eps), _ptr(gx), _ptr(gy), _ptr(f),
                        _ptr(ends))
    return ends


def stream(p: Params, eps: np.ndarray, fpost: np.ndarray, f_prev: np.ndarray | None = None,
           threads: int | None = None):
    """Push streaming of the post-collision fpost; with a velocity inlet / pressure
    outlet the entering populations need f_prev, the state fpost was collided from."""
    eps = _f64(eps)
    fpost = _f64(fpost)
    ends = None
    if p.bc_x == INOUT:
        if f_prev is None:
            raise ValueError("a velocity inlet / pressure outlet needs the previous state")
        ends = open_ends(p, eps, f_prev)
    out = np.empty_like(fpost)
    lib().orc_stream(ctypes.byref(p.c()), _ptr(eps), _ptr(fpost),
                     _ptr(ends) if ends is not None else None, _ptr(out),
                     threads or default_threads())
    return out


def steps(p: Params, eps: np.ndarray, f: np.ndarray, nsteps: int,
          threads: int | None = None) -> np.ndarray:
    """f after nsteps time steps (a new array; f is not modified)."""
    eps = _f64(eps)
    assert eps.shape == (p.Ly, p.Lx)
    f = np.array(f, dtype=np.float64, order="C", copy=True)
    assert f.shape == (9, p.Ly, p.Lx)
    gx, gy = grad_eps(p, eps)
    scratch = np.empty_like(f)
    rc = lib().orc_steps(ctypes.byref(p.c()), _ptr(eps), _ptr(gx), _ptr(gy), _ptr(f),
                         _ptr(scratch), int(nsteps), threads or default_threads())
    if rc != 0:
        raise MemoryError("oracle steps: out of memory")
    return f


def run(p: Params, eps: np.ndarray, nsteps: int, threads: int | None = None) -> np.ndarray:
    """Initial state, then nsteps steps."""
    return steps(p, eps, init(p, eps), nsteps, threads)


def moments(p: Params, eps: np.ndarray, f: np.ndarray) -> dict:
    """Per-cell eps*rho, rho, ux, uy, mx, my, Tx, Ty of the state f."""
    eps = _f64(eps)
    f = _f64(f)
    gx, gy = grad_eps(p, eps)
    out = {k: np.empty_like(eps) for k in ("eps_rho", "rho", "ux", "uy", "mx", "my", "Tx", "Ty")}
    lib().orc_moments(ctypes.byref(p.c()), _ptr(eps), _ptr(gx), _ptr(gy), _ptr(f),
                      *(_ptr(out[k]) for k in ("eps_rho", "rho", "ux", "uy", "mx", "my",
                                               "Tx", "Ty")))
    return out


def drag_derivs(p: Params, eps: float):
    da = ctypes.c_double()
    db = ctypes.c_double()
    lib().orc_drag_derivs(ctypes.byref(p.c()), eps, ctypes.byref(da), ctypes.byref(db))
    return da.value, db.value


def node_collide(p: Params, f, eps: float, gex: float, gey: float) -> np.ndarray:
    """Post-collision populations of one node."""
    f = _f64(f)
    out = np.zeros(9)
    lib().orc_node_collide(ctypes.byref(p.c()), _ptr(f), eps, gex, gey, _ptr(out))
    return out


def node_vjp(p: Params, f, eps: float, gex: float, gey: float, fpost_bar, S_bar=0.0,
             ux_bar=0.0, uy_bar=0.0):
    """Adjoints (f_bar[9], eps_bar, gex_bar, gey_bar) of one node's inputs."""
    f = _f64(f)
    pb = _f64(fpost_bar)
    fb = np.zeros(9)
    eb, gxb, gyb = ctypes.c_double(0.0), ctypes.c_double(0.0), ctypes.c_double(0.0)
    lib().orc_node_vjp(ctypes.byref(p.c()), _ptr(f), eps, gex, gey, _ptr(pb), S_bar, ux_bar,
                       uy_bar, _ptr(fb), ctypes.byref(eb), ctypes.byref(gxb), ctypes.byref(gyb))
    return fb, eb.value, gxb.value, gyb.value


def outlet_flux(p: Params, eps: np.ndarray, f: np.ndarray) -> float:
    """J = sum over the column x = Lx-1 of eps rho u_x of the state f."""
    eps = _f64(eps)
    f = _f64(f)
    gx, gy = grad_eps(p, eps)
    return lib().orc_outlet_flux(ctypes.byref(p.c()), _ptr(eps), _ptr(gx), _ptr(gy), _ptr(f))


def grad_outlet_flux(p: Params, eps: np.ndarray, nsteps: int, threads: int | None = None):
    """(J, dJ/deps) for J = outlet_flux after nsteps steps from the initial state."""
    eps = _f64(eps)
    assert eps.shape == (p.Ly, p.Lx)
    g = np.zeros_like(eps)
    J = ctypes.c_double()
    rc = lib().orc_grad_outlet_flux(ctypes.byref(p.c()), _ptr(eps), int(nsteps), _ptr(g),
                                    ctypes.byref(J), threads or default_threads())
    if rc != 0:
        raise MemoryError("oracle adjoint: out of memory")
    return J.value, g
