"""GPU parity of the sliding y-walls and the paper's Couette experiment
(Section "Examples and discussions": 80 x 80 lattice, porosity 0.1, upper
plate sliding, lower plate at rest, periodic x) against the FP64 oracle and
against the solution of eq. (velocity).

Tolerances:
* short runs with sliding walls: the single-problem bounds (FP64 1e-13 on
  populations after 40 steps; FP32 / FP16 scaled by their unit roundoff and the
  largest stored magnitude);
* steady Couette profiles: FP64 within 1e-10 U of the oracle's steady profile
  (a fixed point of the same discrete map, reached from the same start; measured
  up to 5e-11 U at the smallest U); FP32 within 8 * 2^-24 rho0 + 2e-4 U absolute:
  the rounding floor of the FP32 momentum (u = m / (eps rho) with m a sum of
  populations of total size eps rho, so its rounding is a few units of 2^-24
  relative to rho) plus a relative part (measured: at most 5.5e-7 absolute at
  Re 50); against eq. (velocity) within the oracle's own discretisation error
  plus that bound;
* gradient with sliding walls: FP64 within 1e-10 of the largest |dJ/deps| of
  the oracle's reverse pass.
"""
import dataclasses
import functools
import math

import numpy as np
import pytest

import oracle
import refsol
from parity_util import Spec, gpu_run, oracle_run, rel_l2, say
from paper_1406_6438_amd import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1406_6438_amd import lbm
    lbm.load()


def _bound(spec, eps, fo, nsteps):
    if spec.storage == "f64":
        return 1e-13
    rest = oracle.init(dataclasses.replace(spec, u0=(0.0, 0.0)).oracle(), spec.input_eps(eps))
    de = max(np.abs(eps - np.roll(eps, s, axis=a)).max() for a in (0, 1) for s in (1, -1))
    D = np.abs(fo - rest).max() + de / 18.0
    if spec.storage == "f32":
        return 4 * (nsteps + 1) * 2.0 ** -24 * D
    return 2 * (nsteps + 1) * 2.0 ** -11 * D


# (Lx, Ly, x boundary): ragged and aligned widths, periodic / walls / open x ends
GEOMS = [(12, 7, "periodic"), (13, 9, "walls"), (130, 6, "open"), (260, 5, "periodic"),
         (5, 3, "open"), (64, 4, "walls")]


@pytest.mark.parametrize("storage", ["f64", "f32", "f16"])
@pytest.mark.parametrize("geom", GEOMS, ids=lambda g: "%dx%d_%s" % g)
def test_sliding_walls_parity(geom, storage):
    Lx, Ly, bx = geom
    say(f"[sliding walls {storage}] {Lx}x{Ly} x={bx}")
    spec = Spec(Lx=Lx, Ly=Ly, tau=0.7, walls_y=True, walls_x=bx == "walls", open_x=bx == "open",
                d_p=6.0, u0=(0.01, 0.0), rho_in=1.01, u_in=0.02, rho_out=0.99, u_out=0.02,
                u_wall=(-0.03, 0.05), storage=storage)
    eps = W.grf_porosity(Lx, Ly, seed=700 + Lx, ell=3.0, lo=0.4, hi=1.0)
    for nsteps in (0, 1, 40):
        mg, fg = gpu_run(spec, eps, nsteps)
        mo, fo = oracle_run(spec, eps, nsteps)
        err = np.abs(fg - fo).max()
        assert err <= _bound(spec, eps, fo, nsteps), (nsteps, err)
    if storage != "f16":
        assert rel_l2(mg["ux"], mo["ux"]) <= (1e-12 if storage == "f64" else 1e-5)


def test_sliding_walls_set_get_roundtrip():
    """A plain state written with set_state reads back exactly, also in the slots
    returned by the sliding walls (stored without the gain the reader adds)."""
    from paper_1406_6438_amd import lbm
    spec = Spec(Lx=20, Ly=8, walls_y=True, d_p=5.0, u_wall=(0.02, -0.04), storage="f64")
    eps = W.grf_porosity(20, 8, seed=71, ell=2.0, lo=0.4, hi=1.0)
    f0 = oracle.init(spec.oracle(), eps) * (1.0 + W.noise((9, 8, 20), 5, 1e-3))
    s = lbm.Solver(spec.gpu(), eps)
    s.set_state(f0)
    # a few FP64 roundings of numbers below 0.5 (storage shift and wall gain out and back)
    assert np.abs(s.get_state().cpu().numpy() - f0).max() <= 3e-16
    s.step(7)
    mo, fo = oracle_run(spec, eps, 7, f0)
    assert np.abs(s.get_state().cpu().numpy() - fo).max() <= 1e-13
    s.close()


@pytest.mark.parametrize("geom", [(24, 10, True), (13, 6, False)], ids=["open", "periodic"])
def test_gradient_with_sliding_walls(geom):
    from paper_1406_6438_amd import lbm
    Lx, Ly, is_open = geom
    spec = Spec(Lx=Lx, Ly=Ly, tau=0.75, walls_y=True, open_x=is_open, d_p=6.0, u0=(0.01, 0.0),
                rho_in=1.0, u_in=0.02, rho_out=1.0, u_out=0.02, u_wall=(-0.03, 0.05),
                G=(0.0, 0.0) if is_open else (2e-5, 0.0), storage="f64")
    eps = W.grf_porosity(Lx, Ly, seed=72 + Lx, ell=2.5, lo=0.4, hi=0.95)
    s = lbm.Solver(spec.gpu(), eps)
    J, g = s.grad(60, 11)
    s.close()
    Jo, go = oracle.grad_outlet_flux(spec.oracle(), eps, 60)
    assert abs(J - Jo) <= 1e-12 * abs(Jo)
    assert np.abs(g.cpu().numpy() - go).max() <= 1e-10 * np.abs(go).max()


@functools.lru_cache(maxsize=None)
def _oracle_profile(case, steps):
    """Steady oracle profile of a Couette case (4 columns: the flow is x-independent)."""
    c = W.couette_case(*case)
    L, eps0 = W.COUETTE_L, W.COUETTE_EPS
    so = Spec(Lx=4, Ly=L, tau=c.tau, walls_y=True, d_p=c.d_p, u_wall=(0.0, c.U))
    mo, _ = oracle_run(so, np.full((L, 4), eps0), steps)
    return mo["ux"][:, 0]


def _ode_profile(c, L, eps):
    a = eps ** 2 * c.nu / c.K
    b = eps ** 3 * (1.75 / math.sqrt(150.0 * eps ** 3)) / math.sqrt(c.K)
    return refsol.bf_channel(float(L), c.nu, eps, a, b, 0.0, np.arange(L) + 0.5, u_top=c.U)


@pytest.mark.parametrize("storage", ["f64", "f32"])
@pytest.mark.parametrize("case", W.COUETTE_CASES, ids=lambda c: "Re%g_Da%g" % c)
def test_paper_couette_experiment(case, storage):
    """80 x 80, eps 0.1, 160000 steps on the GPU: the profile at x = H/2 against the
    oracle's steady profile (the flow does not depend on x, so the oracle runs 4
    columns) and against the solution of eq. (velocity)."""
    from paper_1406_6438_amd import lbm
    L, eps0, n = W.COUETTE_L, W.COUETTE_EPS, W.COUETTE_STEPS
    c = W.couette_case(*case)
    say(f"[couette {storage}] Re {c.Re} Da {c.Da} tau {c.tau} U {c.U:.4e}")
    spec = Spec(Lx=L, Ly=L, tau=c.tau, walls_y=True, d_p=c.d_p, u_wall=(0.0, c.U),
                storage=storage)
    s = lbm.Solver(spec.gpu(), np.full((L, L), eps0))
    s.step(n)
    m = s.moments()
    ux = m["ux"].double().cpu().numpy()
    uy = m["uy"].double().cpu().numpy()
    s.close()
    uo = _oracle_profile(case, n)
    ref = _ode_profile(c, L, eps0)
    prof = ux[:, L // 2]
    e_orc = np.abs(prof - uo).max() / c.U
    e_ode = np.abs(prof - ref).max() / c.U
    e_orc_ode = np.abs(uo - ref).max() / c.U
    say(f"  max|u - oracle|/U {e_orc:.3e}, max|u - eq.(velocity)|/U {e_ode:.3e} "
        f"(oracle's own {e_orc_ode:.3e}), x-variation {np.ptp(ux, axis=1).max() / c.U:.2e}")
    tol = 1e-10 * c.U if storage == "f64" else 8 * 2.0 ** -24 + 2e-4 * c.U
    assert e_orc * c.U <= tol
    assert e_ode * c.U <= e_orc_ode * c.U + tol
    assert np.ptp(ux, axis=1).max() <= tol       # no x dependence
    assert np.abs(uy).max() <= tol
