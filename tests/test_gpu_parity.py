"""GPU parity: the HIP library through its C-ABI against the FP64 oracle.

Tolerances (see the design notes for their derivation):
* FP64 storage and arithmetic: differences come only from fused multiply-adds
  and summation order, a few ulp per step: max |f_gpu - f_oracle| <= 1e-13 on
  O(0.1) populations after tens of steps; rel. L2 of u <= 1e-12 at 2000 steps.
* FP32 shifted storage, FP32 arithmetic: rel. L2 of u <= 1e-5 against the FP64
  oracle after 1000 steps on the 512^2 crop of the box workload (the accuracy
  statement the workload is quoted at); short runs use per-field bounds scaled
  by FP32 unit roundoff.
"""
import dataclasses
import math

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


# (Lx, Ly, walls_x, walls_y).  The sweep runs 4 FP32 / 2 FP64 nodes per lane;
# widths not divisible by that end each row in a ragged run (1..3 nodes, the
# rest of the vector in the row padding): single rows/columns, widths below one
# run, a partial last tile, a single partial tile, seams between tiles, walls
# on either axis.
GEOMS = [
    (7, 5, False, False),
    (65, 33, False, True),
    (131, 17, True, True),
    (3, 70, False, True),
    (1, 9, False, True),
    (64, 8, True, False),
    (200, 1, False, False),
    (4, 4, False, False),
    (8, 3, True, False),
    (260, 9, True, True),
    (516, 7, False, True),
    (1024, 5, False, False),
    (130, 11, True, False),
]


def _max_deviation(spec, eps, f):
    """Largest |f_i - w_i eps rho0|: a bound on the magnitude the shifted storage rounds
    (the link-midpoint shift stores less than this)."""
    p = dataclasses.replace(spec, u0=(0.0, 0.0)).oracle()
    return float(np.abs(f - oracle.init(p, spec.input_eps(eps))).max())


def _perturbed_start(spec, eps, seed, amp=2e-3):
    p = spec.oracle()
    return oracle.init(p, spec.input_eps(eps)) * (1.0 + W.noise((9, spec.Ly, spec.Lx), seed, amp))


@pytest.mark.parametrize("mode", ["auto", "triples", "pairs", "wide", "narrow"])
@pytest.mark.parametrize("geom", GEOMS, ids=lambda g: "%dx%d_w%d%d" % g)
def test_f64_parity_small_grids(geom, mode):
    Lx, Ly, wx, wy = geom
    say(f"[f64 parity {mode}] {Lx}x{Ly} walls=({wx},{wy})")
    spec = Spec(Lx=Lx, Ly=Ly, tau=0.62, walls_x=wx, walls_y=wy, d_p=6.0, G=(2e-5, -1e-5),
                u0=(0.01, 0.004), storage="f64", **exec_mode(mode, "f64"))
    eps = W.grf_porosity(Lx, Ly, seed=100 + Lx, ell=2.5, lo=0.35, hi=1.0)
    f0 = _perturbed_start(spec, eps, seed=Ly)
    mg, fg = gpu_run(spec, eps, 40, f0)
    mo, fo = oracle_run(spec, eps, 40, f0)
    assert np.abs(fg - fo).max() <= 1e-13
    assert np.abs(mg["ux"] - mo["ux"]).max() <= 1e-13
    assert np.abs(mg["rho"] - mo["rho"]).max() <= 1e-13


@pytest.mark.parametrize("mode", ["auto", "triples", "short", "tiny", "tall", "quads", "pairs",
                                  "wide", "narrow"])
@pytest.mark.parametrize("geom", GEOMS, ids=lambda g: "%dx%d_w%d%d" % g)
def test_f32_parity_small_grids(geom, mode):
    Lx, Ly, wx, wy = geom
    say(f"[f32 parity {mode}] {Lx}x{Ly} walls=({wx},{wy})")
    spec = Spec(Lx=Lx, Ly=Ly, tau=0.62, walls_x=wx, walls_y=wy, d_p=6.0, G=(2e-5, -1e-5),
                u0=(0.01, 0.004), storage="f32", **exec_mode(mode, "f32"))
    eps = W.grf_porosity(Lx, Ly, seed=100 + Lx, ell=2.5, lo=0.35, hi=1.0)
    f0 = _perturbed_start(spec, eps, seed=Ly)
    nsteps = 40
    mg, fg = gpu_run(spec, eps, nsteps, f0)
    mo, fo = oracle_run(spec, eps, nsteps, f0)
    # Each step rounds every stored deviation once (unit roundoff 2^-24) and the
    # collision adds a few more roundings of the same size: allow 4 per step on the
    # largest deviation D from the rest state, accumulated linearly.
    D = _max_deviation(spec, eps, fo)
    tol = 4 * nsteps * 2.0 ** -24 * D
    assert np.abs(fg - fo).max() <= tol
    # the velocity: six unit-weight terms of that size over eps rho >= 0.35 (the
    # smaller component can exceed a relative bar on a few nodes)
    assert rel_l2(mg["ux"], mo["ux"]) <= 1e-5
    assert np.abs(mg["uy"] - mo["uy"]).max() <= 6 * tol / 0.35
    assert np.abs(mg["rho"] - mo["rho"]).max() <= 9 * tol / 0.35


@pytest.mark.parametrize("storage", ["f64", "f32"])
def test_init_state_is_equilibrium(storage):
    spec = Spec(Lx=70, Ly=19, walls_y=True, d_p=8.0, u0=(0.02, -0.01), rho0=1.1,
                storage=storage)
    eps = W.grf_porosity(70, 19, seed=4, ell=3.0)
    mg, fg = gpu_run(spec, eps, 0)
    fo = oracle.init(spec.oracle(), spec.input_eps(eps))
    # f64: a couple of ulp of O(0.5) values; f32: one rounding when the deviation is
    # stored and one when the reader adds back the half porosity difference
    tol = 4e-16 if storage == "f64" else 2.0 ** -22 * _max_deviation(spec, eps, fo)
    assert np.abs(fg - fo).max() <= tol


def test_f64_set_get_roundtrip():
    spec = Spec(Lx=33, Ly=21, walls_x=True, walls_y=True, d_p=8.0, storage="f64")
    eps = W.grf_porosity(33, 21, seed=6, ell=3.0)
    f0 = _perturbed_start(spec, eps, seed=5, amp=0.05)
    _, fg = gpu_run(spec, eps, 0, f0)
    assert np.abs(fg - f0).max() <= 1e-16


def test_f64_porous_channel_workload():
    """The 64x32 FP64 channel workload, 2000 steps, against the oracle and against the
    Brinkman-Forchheimer profile."""
    import refsol
    w = W.CHANNEL_64x32
    say("[f64 channel 64x32, 2000 steps]")
    spec = Spec(Lx=w.Lx, Ly=w.Ly, tau=w.tau, walls_y=True, d_p=w.d_p, G=(w.Gx, w.Gy),
                storage="f64")
    eps = w.porosity()
    mg, fg = gpu_run(spec, eps, w.steps)
    mo, fo = oracle_run(spec, eps, w.steps)
    # a few ulp per step of FMA / summation-order differences over 2000 steps
    assert rel_l2(mg["ux"], mo["ux"]) <= 1e-12
    assert np.abs(mg["rho"] - mo["rho"]).max() <= 1e-12
    assert np.abs(mg["uy"]).max() <= 1e-12 * np.abs(mo["ux"]).max()
    nu = (w.tau - 0.5) / 3.0
    a, b = oracle.drag_coeffs(spec.oracle(), w.eps_value)
    y = np.arange(w.Ly) + 0.5
    ref = refsol.bf_channel(w.Ly, nu, w.eps_value, a, b, w.Gx, y)
    assert rel_l2(mg["ux"][:, 7], ref) <= 2e-3
    # diagnostics: mass and momentum sums against the oracle's fields
    d = mg["diag"]
    assert abs(d[0] - mo["eps_rho"].sum()) <= 1e-12 * mo["eps_rho"].sum()
    assert abs(d[1] - mo["mx"].sum()) <= 1e-12 * abs(mo["mx"].sum())
    assert abs(d[3] - (mo["eps_rho"] * mo["ux"]).sum()) <= 1e-12 * abs((mo["eps_rho"] * mo["ux"]).sum())
    assert abs(d[5] - np.hypot(mo["ux"], mo["uy"]).max()) <= 1e-12 * np.abs(mo["ux"]).max()
    assert d[6] == 0 and d[7] == w.steps


def test_f32_box_crop_1000_steps():
    """512^2 crop of the 4096^2 box workload, run periodic, 1000 steps: rel. L2(u) <= 1e-5."""
    w = W.BOX_4096_F32
    say("[f32 box crop 512^2, 1000 steps]")
    eps = W.crop_porosity(w)
    spec = Spec(Lx=512, Ly=512, tau=w.tau, d_p=w.d_p, G=(w.Gx, w.Gy), storage="f32")
    mg, _ = gpu_run(spec, eps, w.steps)
    mo, _ = oracle_run(spec, eps, w.steps)
    e_ux = rel_l2(mg["ux"], mo["ux"])
    e_uy = rel_l2(mg["uy"], mo["uy"])
    e_rho = np.abs(mg["rho"] - mo["rho"]).max()
    say(f"  rel L2 ux {e_ux:.3e} uy {e_uy:.3e} max|drho| {e_rho:.3e}")
    u_g = np.hypot(mg["ux"], mg["uy"])
    u_o = np.hypot(mo["ux"], mo["uy"])
    assert rel_l2(u_g, u_o) <= 1e-5
    assert e_ux <= 1e-5
    assert e_rho <= 1e-6


def _oracle_window(spec, eps_full, x0, y0, w, h, nsteps):
    """Oracle moments of the w x h block at (x0, y0) of a periodic problem after nsteps,
    computed on a periodic window with a margin the error front cannot cross."""
    M = nsteps + 2
    ys = np.arange(y0 - M, y0 + h + M) % spec.Ly
    xs = np.arange(x0 - M, x0 + w + M) % spec.Lx
    sw = dataclasses.replace(spec, Lx=w + 2 * M, Ly=h + 2 * M, walls_x=False, walls_y=False)
    mo, _ = oracle_run(sw, eps_full[np.ix_(ys, xs)], nsteps)
    return {k: v[M:M + h, M:M + w] for k, v in mo.items()}


def test_f32_full_size_box_sampled_windows():
    """The 4096^2 box at full size in the launch configuration the benchmark times:
    sampled 32x32 blocks (corners, seams, interior) against windowed oracle runs."""
    from paper_1406_6438_amd import lbm
    w = W.BOX_4096_F32
    nsteps = 24
    say(f"[f32 box 4096^2 full size, {nsteps} steps, sampled windows]")
    eps = w.porosity()
    spec = Spec(Lx=w.Lx, Ly=w.Ly, tau=w.tau, d_p=w.d_p, G=(w.Gx, w.Gy), storage="f32")
    s = lbm.Solver(spec.gpu(), spec.input_eps(eps))
    s.step(nsteps)
    m = s.moments()
    ux = m["ux"].double().cpu().numpy()
    rho = m["rho"].double().cpu().numpy()
    s.close()
    for (x0, y0) in [(0, 0), (4064, 4064), (2048 - 16, 1000), (4064, 17), (63, 4090 - 31)]:
        mo = _oracle_window(spec, spec.input_eps(eps), x0, y0, 32, 32, nsteps)
        blk = np.s_[y0:y0 + 32, x0:x0 + 32]
        # FP32 storage floor: ~1e-6 relative in u after tens of steps; bound 1e-5
        assert np.abs(ux[blk] - mo["ux"]).max() <= 1e-5 * np.abs(mo["ux"]).max()
        assert np.abs(rho[blk] - mo["rho"]).max() <= 1e-6


@pytest.mark.parametrize("Lx", [131, 132])
def test_every_slot_is_written(Lx):
    """Work memory filled with NaN bytes before init: after init and after each of
    two steps the state is finite everywhere (the store map covers every slot, and
    the NaN padding a ragged run computes on stays in the padding): 131 ends each
    row in a ragged run of 3 nodes, 132 does not."""
    from paper_1406_6438_amd import lbm
    spec = Spec(Lx=Lx, Ly=45, walls_y=True, d_p=8.0, G=(1e-5, 0.0), storage="f32")
    eps = W.grf_porosity(Lx, 45, seed=8, ell=3.0)
    p = spec.gpu()
    work = torch.full((lbm.lbm_vans_work_bytes(p),), 255, dtype=torch.uint8, device="cuda:0")
    e = torch.tensor(spec.input_eps(eps), dtype=torch.float32, device="cuda:0")
    h = lbm.lbm_vans_init(p, e, work, torch.cuda.current_stream().cuda_stream)
    try:
        f = torch.empty((9, 45, Lx), dtype=torch.float64, device="cuda:0")
        for _ in range(3):
            lbm.lbm_vans_get_state(h, f)
            torch.cuda.synchronize()
            assert torch.isfinite(f).all()
            lbm.lbm_vans_step(h, 1)
    finally:
        lbm.lbm_vans_destroy(h)


@pytest.mark.parametrize("storage", ["f64", "f32"])
def test_mass_conserved_and_momentum_budget_from_diag_ring(storage):
    """Periodic box: sum eps rho stays constant; sum m changes each step by sum T,
    where T = 2 (eps rho u - m) per node (eq. (1moment))."""
    from paper_1406_6438_amd import lbm
    L = 96
    spec = Spec(Lx=L, Ly=L, tau=0.6, d_p=5.0, G=(3e-5, 1e-5), u0=(0.005, 0.0),
                storage=storage, diag_every=1)
    eps = W.grf_porosity(L, L, seed=12, ell=6.0)
    s = lbm.Solver(spec.gpu(), spec.input_eps(eps))
    s.step(300)
    rec, rc = s.diag_records()
    s.close()
    assert rc == 0 and rec.shape == (300, 8)
    assert np.array_equal(rec[:, 7], np.arange(300))
    mass = rec[:, 0]
    tol = 1e-13 if storage == "f64" else 1e-9
    assert np.abs(mass - mass[0]).max() <= tol * mass[0]
    T = 2.0 * (rec[:-1, 3:5] - rec[:-1, 1:3])
    dm = rec[1:, 1:3] - rec[:-1, 1:3]
    scale = np.abs(rec[:, 1:3]).max()
    tolm = 1e-12 if storage == "f64" else 1e-6
    assert np.abs(dm - T).max() <= tolm * scale


def test_nonfinite_state_is_reported():
    from paper_1406_6438_amd import lbm
    spec = Spec(Lx=40, Ly=24, d_p=8.0, storage="f64")
    eps = W.grf_porosity(40, 24, seed=3, ell=3.0)
    s = lbm.Solver(spec.gpu(), spec.input_eps(eps))
    f = s.get_state().cpu().numpy()
    f[4, 10, 17] = np.nan
    s.set_state(f)
    m = s.moments()
    assert m["rc"] == lbm.ENONFINITE and m["diag"][6] == 1
    s.close()


def test_mach_warning_is_reported():
    """A flow faster than 0.3 c_s gives the positive warning LBM_VANS_WMACH from the
    diagnostics (moments and the in-sweep ring), with the call completed; a slower one
    does not."""
    from paper_1406_6438_amd import lbm
    for u, expect in ((0.15, lbm.OK), (0.2, lbm.WMACH)):     # Mach 0.26, 0.35
        spec = Spec(Lx=40, Ly=24, d_p=math.inf, u0=(u, 0.0), storage="f64", diag_every=1)
        s = lbm.Solver(spec.gpu(), W.uniform_porosity(40, 24, 1.0))
        m = s.moments()
        assert m["rc"] == expect and abs(m["diag"][5] - u) < 1e-12
        s.step(3)
        rec, rc = s.diag_records()
        assert rc == expect and rec.shape == (3, 8)
        if expect == lbm.WMACH:
            assert "Mach" in lbm.load().lbm_vans_last_error().decode()
        s.close()


def test_step_counter_and_zero_steps():
    from paper_1406_6438_amd import lbm
    spec = Spec(Lx=20, Ly=12, d_p=8.0, storage="f32")
    s = lbm.Solver(spec.gpu(), W.uniform_porosity(20, 12, 0.6))
    s.step(0)
    assert s.n == 0
    s.step(5)
    s.step(3)
    assert s.n == 8
    assert s.moments()["diag"][7] == 8
    s.close()


def test_init_rejects_porosity_outside_unit_interval():
    from paper_1406_6438_amd import lbm
    spec = Spec(Lx=20, Ly=12, d_p=8.0, storage="f32")
    eps = W.uniform_porosity(20, 12, 0.6)
    eps[3, 4] = 1.2
    with pytest.raises(lbm.LbmVansError) as ei:
        lbm.Solver(spec.gpu(), eps)
    assert ei.value.code == lbm.EINVAL
    eps[3, 4] = 0.0
    with pytest.raises(lbm.LbmVansError):
        lbm.Solver(spec.gpu(), eps)


# ------------------------------------------------------------------ FP16 shifted storage
# FP16 keeps 11 significant bits (unit roundoff 2^-11) of the stored deviation
# from the link-midpoint rest state; arithmetic is FP32.  The accuracy bar of
# the FP16 workload is rel. L2(u) <= 2e-3 against the FP64 oracle after 2000 steps.


@pytest.mark.parametrize("mode", ["auto", "triples", "pairs", "wide", "narrow"])
@pytest.mark.parametrize("geom", GEOMS, ids=lambda g: "%dx%d_w%d%d" % g)
def test_f16_parity_small_grids(geom, mode):
    Lx, Ly, wx, wy = geom
    say(f"[f16 parity {mode}] {Lx}x{Ly} walls=({wx},{wy})")
    spec = Spec(Lx=Lx, Ly=Ly, tau=0.62, walls_x=wx, walls_y=wy, d_p=6.0, G=(2e-5, -1e-5),
                u0=(0.01, 0.004), storage="f16", fp16_scale_log2=10,
                **exec_mode(mode, "f16"))
    eps = W.grf_porosity(Lx, Ly, seed=100 + Lx, ell=2.5, lo=0.35, hi=1.0)
    f0 = _perturbed_start(spec, eps, seed=Ly)
    nsteps = 40
    mg, fg = gpu_run(spec, eps, nsteps, f0)
    mo, fo = oracle_run(spec, eps, nsteps, f0)
    # Stored deviations are at most D; each step rounds them once at 2^-11.  The
    # momentum sums six of them with unit weights, so after n steps |du| is at most
    # 6 n 2^-11 D / (eps rho) with eps >= 0.35.  (These grids have a porosity far
    # rougher than the workloads -- correlation length 2.5 -- so D is large.)
    D = _max_deviation(spec, eps, fo)
    assert np.abs(fg - fo).max() <= 2 * nsteps * 2.0 ** -11 * D
    du = 6 * nsteps * 2.0 ** -11 * D / 0.35
    assert np.abs(mg["ux"] - mo["ux"]).max() <= du
    assert np.abs(mg["uy"] - mo["uy"]).max() <= du


def test_f16_box_crop_2000_steps():
    """512^2 crop of the 8192^2 FP16 box workload, run periodic, 2000 steps:
    rel. L2(u) <= 2e-3 against the FP64 oracle."""
    w = W.BOX_8192_F16
    say("[f16 box crop 512^2 of the 8192^2 field, 2000 steps]")
    eps = W.crop_porosity(w)
    spec = Spec(Lx=512, Ly=512, tau=w.tau, d_p=w.d_p, G=(w.Gx, w.Gy), storage="f16",
                fp16_scale_log2=10)
    mg, _ = gpu_run(spec, eps, w.steps)
    mo, _ = oracle_run(spec, eps, w.steps)
    u_g = np.hypot(mg["ux"], mg["uy"])
    u_o = np.hypot(mo["ux"], mo["uy"])
    e_u = rel_l2(u_g, u_o)
    say(f"  rel L2 |u| {e_u:.3e}  ux {rel_l2(mg['ux'], mo['ux']):.3e}")
    assert e_u <= 2e-3
    assert rel_l2(mg["ux"], mo["ux"]) <= 2e-3
    assert np.abs(mg["rho"] - mo["rho"]).max() <= 1e-4


def test_f16_full_size_box_sampled_windows():
    """The 8192^2 FP16 box at full size in the launch configuration the benchmark
    times: sampled 32x32 blocks against windowed oracle runs."""
    from paper_1406_6438_amd import lbm
    w = W.BOX_8192_F16
    nsteps = 20
    say(f"[f16 box 8192^2 full size, {nsteps} steps, sampled windows]")
    eps = w.porosity()
    spec = Spec(Lx=w.Lx, Ly=w.Ly, tau=w.tau, d_p=w.d_p, G=(w.Gx, w.Gy), storage="f16",
                fp16_scale_log2=10)
    s = lbm.Solver(spec.gpu(), spec.input_eps(eps))
    s.step(nsteps)
    m = s.moments()
    ux = m["ux"].double().cpu().numpy()
    rho = m["rho"].double().cpu().numpy()
    s.close()
    assert m["rc"] == 0
    for (x0, y0) in [(0, 0), (8160, 8160), (4096 - 16, 3000), (8160, 5), (100, 8190 - 31)]:
        mo = _oracle_window(spec, spec.input_eps(eps), x0, y0, 32, 32, nsteps)
        blk = np.s_[y0:y0 + 32, x0:x0 + 32]
        assert rel_l2(ux[blk], mo["ux"]) <= 2e-3
        assert np.abs(rho[blk] - mo["rho"]).max() <= 1e-4


# Two steps per pass: lbm_vans_step(n) with n >= 2 in FP32 or FP16 storage runs pairs
# of steps in one pass (the intermediate state stays in registers).  Against the
# oracle and against the same steps taken one per call.  x ends periodic, walls or
# open (the reservoirs start after the first step, inside the first pass).
TB_GEOMS = [(70, 40, "periodic", False), (130, 33, "periodic", True), (5, 7, "periodic", True),
            (1, 3, "periodic", False), (300, 1, "periodic", False), (64, 32, "periodic", True),
            (70, 21, "walls", True), (63, 9, "walls", False), (2, 5, "walls", True),
            (130, 17, "open", True), (62, 6, "open", False), (3, 4, "open", True),
            # three steps: the middle strip's halo lanes reach the last column, so it
            # takes the pass with the x-end rules; four steps: it is clear of the ends
            (122, 13, "open", True),
            # several chunks of 12, 24 and 28 rows, the last one short
            (64, 90, "periodic", False), (70, 61, "walls", True), (130, 75, "open", True)]


@pytest.mark.parametrize("per_pass, rows", [(2, 0), (3, 0), (3, 6), (3, 12), (3, 24), (3, 28),
                                            (4, 0)],
                         ids=["pairs", "triples", "triples_6rows", "triples_12rows",
                              "triples_24rows", "triples_28rows", "quads"])
@pytest.mark.parametrize("storage", ["f32", "f16"])
@pytest.mark.parametrize("geom", TB_GEOMS, ids=lambda g: "%dx%d_%s_wy%d" % g)
def test_multi_step_pass_matches_oracle_and_single_steps(geom, storage, per_pass, rows):
    """Two, three or four steps per pass (three in chunks of the automatic height or of
    6, 12, 24 or 28 rows, FP32; four in 24-row chunks, FP32) against the oracle and against
    one step per call; step counts that leave a shorter last pass (2, 7: 3+3+1,
    2+2+2+1 or 4+3) and that do not."""
    from paper_1406_6438_amd import lbm
    if rows and storage != "f32":
        pytest.skip("the FP16 three-step pass has one chunk height")
    if per_pass == 4 and storage != "f32":
        pytest.skip("the four-step pass is built for FP32 storage")
    Lx, Ly, bx, wy = geom
    say(f"[{per_pass}-step pass {storage} rows {rows or 'auto'}] {Lx}x{Ly} x={bx} walls_y={wy}")
    spec = Spec(Lx=Lx, Ly=Ly, tau=0.62, walls_x=bx == "walls", open_x=bx == "open",
                walls_y=wy, d_p=6.0, G=(0.0, 0.0) if bx == "open" else (2e-5, -1e-5),
                u0=(0.01, 0.004), rho_in=1.01, u_in=0.02, rho_out=0.99, u_out=0.015,
                u_wall=(0.0, 0.03) if wy else (0.0, 0.0), storage=storage,
                steps_per_pass=per_pass, pass_rows=rows)
    eps = W.grf_porosity(Lx, Ly, seed=900 + Lx, ell=2.5, lo=0.35, hi=1.0)
    for nsteps in (2, 3, 7, 40):
        mg, fg = gpu_run(spec, eps, nsteps)
        mo, fo = oracle_run(spec, eps, nsteps)
        # stored magnitudes: the deviation from rest plus the half porosity difference
        # of the link-midpoint shift (w_i rho0 |delta eps| / 2 <= |delta eps| / 18)
        de = max(np.abs(eps - np.roll(eps, sh, axis=a)).max() for a in (0, 1) for sh in (1, -1))
        D = _max_deviation(spec, eps, fo) + de / 18.0
        # per population: the storage bound of the single-step tests; the velocity: six
        # unit-weight terms of that size over eps rho >= 0.35
        tol = (4 * (nsteps + 1) * 2.0 ** -24 if storage == "f32" else
               2 * (nsteps + 1) * 2.0 ** -11) * D
        assert np.abs(fg - fo).max() <= tol
        assert np.abs(mg["ux"] - mo["ux"]).max() <= 6 * tol / 0.35
        s = lbm.Solver(dataclasses.replace(spec, steps_per_pass=1).gpu(), spec.input_eps(eps))
        s.step(nsteps)                                    # one step per pass
        f1 = s.get_state().cpu().numpy()
        s.close()
        assert np.abs(fg - f1).max() <= tol
