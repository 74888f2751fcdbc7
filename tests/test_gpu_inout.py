"""GPU parity of the velocity inlet / pressure outlet (bc_x = LBM_BC_INOUT) against
the FP64 oracle.

The inlet and outlet reservoirs take one quantity from the boundary node itself
(its density at the inlet, its velocity at the outlet).  The library keeps the
reservoir populations of the next step in the boundary node's slots whose
populations leave the domain, so every launch mode (one step per pass of either
width, two or three steps per pass in either chunk height, batches) and the state
copies must reproduce the oracle's step.

Tolerances are those of the other parity tests: FP64 a few ulp per step; FP32 four
roundings per step of the largest stored magnitude; FP16 two roundings per step at
2^-11; the FP64 gradient within 1e-10 of the largest |dJ/deps| of the oracle's
reverse pass, the FP32 gradient within rel. L2 1e-4.
"""
import dataclasses

import numpy as np
import pytest

import oracle
from parity_util import Spec, exec_mode, gpu_run, oracle_run, rel_l2, say
from paper_1406_6438_amd import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1406_6438_amd import lbm
    lbm.load()


def _spec(Lx, Ly, storage, walls_y=True, **kw):
    args = dict(Lx=Lx, Ly=Ly, tau=0.7, walls_y=walls_y, inout=True, d_p=6.0, u_in=0.03,
                rho_out=0.99, u0=(0.01, 0.002), G=(1e-5, 0.0), storage=storage,
                u_wall=(0.0, 0.02) if walls_y else (0.0, 0.0))
    args.update(kw)
    return Spec(**args)


# one-node-wide strips at the ends of ragged rows, two-node channels, several
# tiles and strips, several chunks of 24 and 28 rows with a short last one
GEOMS = [(12, 7, True), (13, 9, False), (130, 11, True), (2, 5, True), (61, 30, True),
         (260, 6, False), (130, 75, True), (3, 64, False)]


def _bound(spec, eps, fo, nsteps):
    if spec.storage == "f64":
        return 1e-13
    rest = oracle.init(dataclasses.replace(spec, u0=(0.0, 0.0)).oracle(), spec.input_eps(eps))
    de = max(np.abs(eps - np.roll(eps, s, axis=a)).max() for a in (0, 1) for s in (1, -1))
    D = np.abs(fo - rest).max() + de / 18.0
    if spec.storage == "f32":
        return 4 * (nsteps + 1) * 2.0 ** -24 * D
    return 2 * (nsteps + 1) * 2.0 ** -11 * D


@pytest.mark.parametrize("mode", ["auto", "triples", "short", "tiny", "tall", "quads", "pairs", "wide",
                                  "narrow"])
@pytest.mark.parametrize("storage", ["f64", "f32", "f16"])
@pytest.mark.parametrize("geom", GEOMS, ids=lambda g: "%dx%d_wy%d" % g)
def test_inout_forward_parity(geom, storage, mode):
    Lx, Ly, wy = geom
    if storage == "f64" and mode in ("triples", "short", "tiny", "tall", "quads", "pairs"):
        pytest.skip("FP64 storage steps one step per pass")
    if storage == "f16" and mode in ("short", "tiny", "tall", "quads"):
        pytest.skip("the FP16 multi-step passes have one chunk height and three steps")
    say(f"[inout forward {storage} {mode}] {Lx}x{Ly} walls_y={wy}")
    spec = _spec(Lx, Ly, storage, walls_y=wy, **exec_mode(mode, storage))
    eps = W.grf_porosity(Lx, Ly, seed=1200 + Lx, ell=3.0, lo=0.4, hi=1.0)
    for nsteps in (1, 7, 40):
        mg, fg = gpu_run(spec, eps, nsteps)
        mo, fo = oracle_run(spec, eps, nsteps)
        tol = _bound(spec, eps, fo, nsteps)
        assert np.abs(fg - fo).max() <= tol, nsteps
        assert np.abs(mg["ux"] - mo["ux"]).max() <= 6 * tol / 0.4, nsteps
        assert np.abs(mg["rho"] - mo["rho"]).max() <= 9 * tol / 0.4, nsteps


@pytest.mark.parametrize("storage", ["f64", "f32"])
def test_inout_state_set_get_and_continue(storage):
    """A perturbed state set through set_state comes back through get_state (the
    boundary slots included) and steps on as the oracle does from it."""
    Lx, Ly = 37, 11
    spec = _spec(Lx, Ly, storage)
    eps = W.grf_porosity(Lx, Ly, seed=1300, ell=3.0, lo=0.4, hi=1.0)
    f0 = oracle.init(spec.oracle(), spec.input_eps(eps)) * (1.0 + W.noise((9, Ly, Lx), 77, 2e-3))
    _, fg0 = gpu_run(spec, eps, 0, f0)
    tol0 = 1e-16 if storage == "f64" else 2.0 ** -22 * np.abs(f0).max() * 0.05
    assert np.abs(fg0 - f0).max() <= tol0
    mg, fg = gpu_run(spec, eps, 25, f0)
    mo, fo = oracle_run(spec, eps, 25, f0)
    assert np.abs(fg - fo).max() <= _bound(spec, eps, fo, 25)


def test_inout_pressure_driven_slab_reaches_ergun_gradient():
    """FP64: the steady flow through a uniform slab (no body force) on the GPU equals
    the oracle's steady state, whose density slope the oracle pins to Ergun."""
    Lx, Ly = 48, 3
    spec = Spec(Lx=Lx, Ly=Ly, tau=0.7, inout=True, u_in=0.02, rho_out=1.0, d_p=30.0,
                u0=(0.02, 0.0), storage="f64")
    eps = np.full((Ly, Lx), 0.6)
    mg, _ = gpu_run(spec, eps, 20000)
    mo, _ = oracle_run(spec, eps, 20000)
    assert np.abs(mg["rho"] - mo["rho"]).max() <= 1e-12
    assert np.abs(mg["ux"] - mo["ux"]).max() <= 1e-12 * 0.02


def _grad_gpu(spec, eps, nsteps, K):
    from paper_1406_6438_amd import lbm
    s = lbm.Solver(spec.gpu(), spec.input_eps(eps))
    J, g = s.grad(nsteps, K)
    s.close()
    return J, g.cpu().numpy()


@pytest.mark.parametrize("geom", [(24, 12, True), (26, 10, False), (132, 9, True)],
                         ids=lambda g: "%dx%d_wy%d" % g)
def test_inout_gradient_fp64_matches_oracle_adjoint(geom):
    Lx, Ly, wy = geom
    say(f"[inout grad f64] {Lx}x{Ly} walls_y={wy}")
    spec = _spec(Lx, Ly, "f64", walls_y=wy)
    eps = W.grf_porosity(Lx, Ly, seed=1400 + Lx, ell=3.0, lo=0.4, hi=0.98)
    nsteps = 80
    Jg, gg = _grad_gpu(spec, eps, nsteps, 16)
    Jo, go = oracle.grad_outlet_flux(spec.oracle(), spec.input_eps(eps), nsteps)
    assert abs(Jg - Jo) <= 1e-12 * abs(Jo)
    assert np.abs(gg - go).max() <= 1e-10 * np.abs(go).max()


@pytest.mark.parametrize("Lx", [96, 97])
def test_inout_gradient_fp32_matches_oracle_adjoint(Lx):
    say(f"[inout grad f32] {Lx}x40, 300 steps")
    spec = _spec(Lx, 40, "f32", tau=0.8, d_p=60.0, u0=(0.02, 0.0), u_in=0.02, rho_out=1.0,
                 G=(0.0, 0.0), u_wall=(0.0, 0.0))
    eps = W.grf_porosity(Lx, 40, seed=1500, ell=6.0, lo=0.4, hi=1.0)
    Jg, gg = _grad_gpu(spec, eps, 300, 50)
    Jo, go = oracle.grad_outlet_flux(spec.oracle(), spec.input_eps(eps), 300)
    say(f"  J rel err {abs(Jg - Jo) / abs(Jo):.3e}, grad rel L2 {rel_l2(gg, go):.3e}")
    assert abs(Jg - Jo) <= 1e-5 * abs(Jo)
    assert rel_l2(gg, go) <= 1e-4


@pytest.mark.parametrize("storage", ["f64", "f32"])
def test_inout_batch_forward_and_gradient(storage):
    """Members of uneven size with velocity inlets and pressure outlets: batched steps
    (three per launch, then single ones) and the batched gradient against the oracle."""
    from paper_1406_6438_amd import lbm
    sizes = [(24, 10), (61, 9), (130, 30), (3, 7)]
    members = []
    for k, (Lx, Ly) in enumerate(sizes):
        spec = _spec(Lx, Ly, storage, tau=0.6 + 0.07 * k, d_p=5.0 + k, u_in=0.02 + 0.004 * k,
                     rho_out=1.0 - 0.003 * k)
        members.append((spec, W.grf_porosity(Lx, Ly, seed=1600 + k, ell=3.0, lo=0.4, hi=1.0)))
    sv = [lbm.Solver(s.gpu(), s.input_eps(e)) for s, e in members]
    b = lbm.Batch(sv)
    b.step(31)
    for (spec, eps), s in zip(members, sv):
        f = s.get_state().cpu().numpy()
        _, fo = oracle_run(spec, eps, 31)
        err = np.abs(f - fo).max()
        say(f"[inout batch {storage}] {spec.Lx}x{spec.Ly}: max |f - f_oracle| {err:.2e}")
        assert err <= _bound(spec, eps, fo, 31)
    nsteps, K = 40, 9
    J, g = b.grad(nsteps, K)
    for (spec, eps), Jb, gb in zip(members, J, g):
        Jo, go = oracle.grad_outlet_flux(spec.oracle(), spec.input_eps(eps), nsteps)
        gb = gb.cpu().numpy()
        say(f"  grad {spec.Lx}x{spec.Ly}: J rel {abs(Jb - Jo) / abs(Jo):.2e}, "
            f"rel L2 {rel_l2(gb, go):.2e}")
        # J after 40 steps is a small net flux on the longer members (the inflow has
        # not crossed them yet): hold it against the inflow's scale, Ly u_in
        scale = spec.Ly * spec.u_in
        if storage == "f64":
            assert abs(Jb - Jo) <= 1e-12 * scale
            assert np.abs(gb - go).max() <= 1e-10 * np.abs(go).max()
        else:
            assert abs(Jb - Jo) <= 1e-5 * scale
            assert rel_l2(gb, go) <= 1e-4
    b.close()
    for s in sv:
        s.close()
