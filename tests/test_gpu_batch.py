"""GPU parity of the batched ensemble path (many members, one launch per vector
width per step, captured step graphs, autotuned launch shape) against the FP64
oracle, member by member, and against the same members run alone.

Tolerances are those of the single-problem parity tests:
* FP64: a few ulp per step (max |f - f_oracle| <= 1e-13 after 30 steps);
* FP32: FP32 roundoff, 4 per step, of the largest stored magnitude, and
  rel. L2(u) <= 1e-5 after 2000 steps at the full ensemble;
* FP16: 2 roundings per step at 2^-11 of the largest stored magnitude;
* gradients: FP64 <= 1e-10 of the largest |dJ/deps|, FP32 rel. L2 <= 1e-4,
  both against the oracle's FP64 reverse pass.
With FP32 / FP16 storage the batch advances three steps per launch by default
(the multi-step pass), like a problem run alone; two steps per launch and the
single-step kernels are covered with steps_per_pass = 2 and 1.
A member of a batch takes the same node update as a problem run alone, so the
batched results are also compared with lone runs, within the precision bound
above (the batched kernel is a different compilation of the same source and
may fuse other multiply-adds; the tests print whether the bits agree).  Launch
shapes of one width and graph replays run the same kernel and must agree bit
for bit.
"""
import dataclasses

import numpy as np
import pytest

import oracle
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


# Widths that are multiples of 4, of 2 only, odd (ragged last runs of 1..3
# nodes); one or several tiles wide; a single row; a width below one run.
SIZES = [(96, 9), (130, 7), (67, 12), (260, 5), (5, 6), (1030, 3), (64, 1), (3, 4)]
BCS = {"periodic": dict(), "walls": dict(walls_x=True, walls_y=True),
       "open_walls": dict(open_x=True, walls_y=True), "open_periodic": dict(open_x=True),
       "inout_walls": dict(inout=True, walls_y=True)}


def _member_specs(storage, bc, sizes=SIZES):
    out = []
    for k, (Lx, Ly) in enumerate(sizes):
        kw = dict(BCS[bc])
        is_open = kw.get("open_x", False) or kw.get("inout", False)
        spec = Spec(Lx=Lx, Ly=Ly, tau=0.58 + 0.06 * k, d_p=4.0 + 1.5 * k,
                    G=(0.0, 0.0) if is_open else (2e-5 * (1 + k % 2), -1e-5),
                    u0=(0.01 + 0.002 * k, 0.003), rho_in=1.0 + 0.004 * k, u_in=0.02 + 0.003 * k,
                    rho_out=0.995, u_out=0.015, storage=storage, **kw)
        eps = W.grf_porosity(Lx, Ly, seed=600 + 7 * k, ell=3.0, lo=0.4, hi=1.0)
        out.append((spec, eps))
    return out


def _bound(spec, eps, fo, nsteps):
    """Per-population bound of the storage precision (see the module docstring)."""
    if spec.storage == "f64":
        return 1e-13
    rest = oracle.init(dataclasses.replace(spec, u0=(0.0, 0.0)).oracle(), spec.input_eps(eps))
    de = max(np.abs(eps - np.roll(eps, s, axis=a)).max() for a in (0, 1) for s in (1, -1))
    D = np.abs(fo - rest).max() + de / 18.0
    if spec.storage == "f32":
        return 4 * (nsteps + 1) * 2.0 ** -24 * D
    return 2 * (nsteps + 1) * 2.0 ** -11 * D


def _solvers(members):
    from paper_1406_6438_amd import lbm
    return [lbm.Solver(s.gpu(), s.input_eps(e)) for s, e in members]


def _states(solvers):
    return [s.get_state().cpu().numpy() for s in solvers]


def _close(objs):
    for o in objs:
        o.close()


@pytest.mark.parametrize("storage", ["f64", "f32", "f16"])
@pytest.mark.parametrize("bc", list(BCS))
def test_batch_matches_oracle_and_lone_runs(storage, bc):
    from paper_1406_6438_amd import lbm
    say(f"[batch forward {storage} {bc}] members {SIZES}")
    members = _member_specs(storage, bc)
    nsteps = 30
    sv = _solvers(members)
    b = lbm.Batch(sv)
    b.step(nsteps)
    fb = _states(sv)
    assert all(s.n == nsteps for s in sv)
    for (spec, eps), f in zip(members, fb):
        mo, fo = oracle_run(spec, eps, nsteps)
        err = np.abs(f - fo).max()
        say(f"  {spec.Lx}x{spec.Ly}: max |f - f_oracle| {err:.3e} (bound "
            f"{_bound(spec, eps, fo, nsteps):.3e})")
        assert err <= _bound(spec, eps, fo, nsteps)
        _, fl = gpu_run(spec, eps, nsteps)
        say(f"    lone run: max diff {np.abs(f - fl).max():.3e}, same bits {np.array_equal(f, fl)}")
        assert np.abs(f - fl).max() <= _bound(spec, eps, fo, nsteps)
    b.close()
    _close(sv)


def _vmax(storage):
    return 2 if storage == "f64" else 4


def _launch_plan(nsteps, graph_steps, max_pass):
    """Steps of each launch lbm_vans_batch_step makes from state 0 (graphs replay whole
    chunks from state 1 on; every launch takes as many steps as it may).  Launch
    sequences that split the steps differently round the intermediate states
    differently, so only equal plans can give the same bits."""
    plan, k = [], 0
    while k < nsteps:
        if graph_steps > 0 and k >= 1 and nsteps - k >= graph_steps:
            j = 0
            while j < graph_steps:
                m = min(max_pass, graph_steps - j)
                plan.append(m)
                j += m
            k += graph_steps
        else:
            m = min(max_pass, nsteps - k)
            plan.append(m)
            k += m
    return tuple(plan)


@pytest.mark.parametrize("rows", [24, 28])
@pytest.mark.parametrize("bc", ["periodic", "walls", "open_walls"])
def test_batch_three_step_chunk_heights(bc, rows):
    """The batched three-step pass in chunks of 24 and of 28 rows (FP32) on members
    tall enough for several chunks (the last one short): against the oracle and
    against each member run alone in chunks of the same height, 13 steps."""
    from paper_1406_6438_amd import lbm
    members = _member_specs("f32", bc, sizes=[(96, 61), (130, 75), (67, 30), (5, 6)])
    nsteps = 13
    say(f"[batch chunk rows {rows} {bc}]")
    sv = _solvers(members)
    b = lbm.Batch(sv)
    b.configure(4, 0, 0, 3, rows)
    assert b.config["pass_rows"] == rows
    b.step(nsteps)
    fb = _states(sv)
    b.close()
    _close(sv)
    for (spec, eps), f in zip(members, fb):
        mo, fo = oracle_run(spec, eps, nsteps)
        bound = _bound(spec, eps, fo, nsteps)
        assert np.abs(f - fo).max() <= bound
        _, fl = gpu_run(dataclasses.replace(spec, steps_per_pass=3, pass_rows=rows), eps, nsteps)
        say(f"  {spec.Lx}x{spec.Ly}: max |f - f_oracle| {np.abs(f - fo).max():.3e} (bound "
            f"{bound:.3e}); lone run same bits {np.array_equal(f, fl)}")
        assert np.abs(f - fl).max() <= bound


@pytest.mark.parametrize("bc", ["periodic", "walls", "open_walls"])
def test_batch_four_step_pass(bc):
    """The batched four-step pass (FP32) on members tall enough for it and for several
    chunks (the last one short): against the oracle and against each member run alone
    with four steps per pass, 13 steps (4+4+4+1)."""
    from paper_1406_6438_amd import lbm
    members = _member_specs("f32", bc, sizes=[(96, 61), (130, 75), (67, 40), (5, 40)])
    nsteps = 13
    say(f"[batch four steps {bc}]")
    sv = _solvers(members)
    b = lbm.Batch(sv)
    b.configure(4, 0, 0, 4, 0)
    assert b.pass_plan == (4, 24)
    b.step(nsteps)
    fb = _states(sv)
    b.close()
    _close(sv)
    for (spec, eps), f in zip(members, fb):
        mo, fo = oracle_run(spec, eps, nsteps)
        bound = _bound(spec, eps, fo, nsteps)
        assert np.abs(f - fo).max() <= bound
        _, fl = gpu_run(dataclasses.replace(spec, steps_per_pass=4), eps, nsteps)
        say(f"  {spec.Lx}x{spec.Ly}: max |f - f_oracle| {np.abs(f - fo).max():.3e} (bound "
            f"{bound:.3e}); lone run same bits {np.array_equal(f, fl)}")
        assert np.abs(f - fl).max() <= bound


@pytest.mark.parametrize("storage", ["f32", "f16", "f64"])
def test_every_launch_shape(storage):
    """vec 4/2/1, one workgroup per tile or persistent grids, with and without
    graphs, one, two or three steps per launch (FP64 has single steps only): the
    same bits for one vec and one sequence of steps per launch, within the
    precision bound across them.  13 steps: e.g. 3+3+3+3+1, 2+2+2+2+2+2+1, or
    3+(3+1)+(3+1)+2 with 4-step graphs of triples."""
    from paper_1406_6438_amd import lbm
    members = _member_specs(storage, "open_walls")
    vmax = _vmax(storage)
    pairs = (1,) if storage == "f64" else (0, 1, 2)
    shapes = [(v, g, c, sp) for v in sorted({vmax, 2, 1}, reverse=True) for g in (0, 8, 64)
              for c in (0, 4, 6) for sp in pairs]
    nsteps = 13
    ref = {}
    orc = [oracle_run(spec, eps, nsteps)[1] for spec, eps in members]
    for v, g, c, sp in shapes:
        say(f"[batch shape {storage}] vec={v} grid={g} graph_steps={c} steps_per_pass={sp}")
        sv = _solvers(members)
        b = lbm.Batch(sv)
        b.configure(v, g, c, sp)
        cfg = b.config
        assert (cfg["vec"], cfg["grid"], cfg["graph_steps"], cfg["steps_per_pass"]) == (v, g, c, sp)
        b.step(nsteps)
        f = _states(sv)
        b.close()
        assert all(s.n == nsteps for s in sv)
        _close(sv)
        for (spec, eps), a, fo in zip(members, f, orc):
            assert np.abs(a - fo).max() <= _bound(spec, eps, fo, nsteps)
        key = (v, _launch_plan(nsteps, c, 1 if storage == "f64" else (sp or 3)))
        if key not in ref:
            ref[key] = f
            continue
        for a, r in zip(f, ref[key]):
            assert np.array_equal(a, r), key


@pytest.mark.parametrize("steps_per_pass", [0, 1, 2])
@pytest.mark.parametrize("chunk", [4, 6])
def test_graph_replays_match_plain_launches(chunk, steps_per_pass):
    """A graph replayed several times, with eager work and synchronisations in
    between, against plain launches of the same steps: every replay identical.
    A 6-step graph of pairs is three launches and a 4-step graph of triples is a
    triple and a single step, so a replay can end in the other state slot than
    it started from."""
    from paper_1406_6438_amd import lbm
    members = _member_specs("f32", "open_walls")
    sa, sb = _solvers(members), _solvers(members)
    ba, bb = lbm.Batch(sa), lbm.Batch(sb)
    ba.configure(4, 0, chunk, steps_per_pass)
    bb.configure(4, 0, 0, steps_per_pass)
    ba.step(1)
    bb.step(1)
    for r in range(4):
        ba.step(chunk)       # one replay of the graph
        bb.step(chunk)
        torch.cuda.synchronize()
        m = sa[r % len(sa)].moments()   # eager work between replays
        assert m["rc"] == 0
        for x, y in zip(_states(sa), _states(sb)):
            assert np.array_equal(x, y), f"replay {r}"
    assert all(s.n == 1 + 4 * chunk for s in sa)
    _close([ba, bb])
    _close(sa + sb)


def test_autotune_keeps_the_state_and_reports_trials():
    from paper_1406_6438_amd import lbm
    members = _member_specs("f32", "open_walls")
    sv = _solvers(members)
    b = lbm.Batch(sv)
    b.step(3)
    before = _states(sv)
    best, trials = b.tune(reps=3)
    say(f"[batch tune] best {best}; {len(trials)} trials")
    assert trials and best["us_per_step"] == min(t["us_per_step"] for t in trials)
    assert sorted({t["steps_per_pass"] for t in trials}) == [1, 2, 3, 4]   # FP32: four too
    assert all(b.config[k] == best[k] for k in ("vec", "grid", "steps_per_pass"))
    for x, y in zip(_states(sv), before):
        assert np.array_equal(x, y)
    assert all(s.n == 3 for s in sv)
    b.step(10)
    for (spec, eps), f in zip(members, _states(sv)):
        _, fl = gpu_run(spec, eps, 13)
        _, fo = oracle_run(spec, eps, 13)
        assert np.abs(f - fl).max() <= 2 * _bound(spec, eps, fo, 13)
    b.close()
    _close(sv)


def test_batch_rejects_mismatched_members_and_out_of_step_members():
    from paper_1406_6438_amd import lbm
    m32 = _member_specs("f32", "open_walls", sizes=[(16, 6), (20, 5)])
    m64 = _member_specs("f64", "open_walls", sizes=[(16, 6)])
    mp = _member_specs("f32", "walls", sizes=[(16, 6)])
    a, c = _solvers(m32)
    (d,) = _solvers(m64)
    (e,) = _solvers(mp)
    for bad in ([a, d], [a, e], [a, a]):
        with pytest.raises(lbm.LbmVansError):
            lbm.Batch(bad)
    spec, eps = m32[0]
    diag = lbm.Solver(dataclasses.replace(spec, diag_every=5).gpu(), spec.input_eps(eps))
    with pytest.raises(lbm.LbmVansError):
        lbm.Batch([diag, c])
    b = lbm.Batch([a, c])
    for cfg in ((3, 0, 16), (4, 12, 16), (4, 0, 3), (8, 0, 16), (4, 0, 16, 5),
                (4, 0, 16, -1), (4, 0, 16, 3, 16), (4, 0, 16, 3, -28), (4, 0, 16, 3, 12)):
        with pytest.raises(lbm.LbmVansError):
            b.configure(*cfg)
    a.step(1)                       # a member stepped on its own
    with pytest.raises(lbm.LbmVansError):
        b.step(1)
    c.step(1)                       # back in step
    b.step(2)
    assert a.n == 3 and c.n == 3
    b.close()
    _close([a, c, d, e, diag])


@pytest.mark.parametrize("storage", ["f64", "f32"])
def test_batch_gradient_matches_oracle_adjoint(storage):
    from paper_1406_6438_amd import lbm
    sizes = [(24, 10), (26, 9), (96, 12), (130, 8)]
    members = _member_specs(storage, "open_walls", sizes=sizes)
    nsteps, K = 60, 9
    sv = _solvers(members)
    b = lbm.Batch(sv)
    J, g = b.grad(nsteps, K)
    for (spec, eps), Jb, gb, s in zip(members, J, g, sv):
        Jo, go = oracle.grad_outlet_flux(spec.oracle(), spec.input_eps(eps), nsteps)
        gb = gb.cpu().numpy()
        say(f"[batch grad {storage}] {spec.Lx}x{spec.Ly}: J rel {abs(Jb - Jo) / abs(Jo):.2e}, "
            f"grad rel L2 {rel_l2(gb, go):.2e}")
        assert s.n == nsteps
        if storage == "f64":
            assert abs(Jb - Jo) <= 1e-12 * abs(Jo)
            assert np.abs(gb - go).max() <= 1e-10 * np.abs(go).max()
        else:
            assert abs(Jb - Jo) <= 1e-5 * abs(Jo)
            assert rel_l2(gb, go) <= 1e-4
        lone = lbm.Solver(spec.gpu(), spec.input_eps(eps))
        Jl, gl = lone.grad(nsteps, K)
        lone.close()
        gl = gl.cpu().numpy()
        say(f"    lone gradient: same bits {Jl == Jb and np.array_equal(gl, gb)}")
        if storage == "f64":
            assert abs(Jl - Jb) <= 1e-13 * abs(Jl)
            assert np.abs(gl - gb).max() <= 1e-11 * np.abs(gl).max()
        else:
            assert abs(Jl - Jb) <= 1e-6 * abs(Jl)
            assert rel_l2(gb, gl) <= 1e-5
    b.close()
    _close(sv)


def _ensemble_specs():
    U = W.ENSEMBLE_U
    out = []
    for m in W.ensemble():
        spec = Spec(Lx=m.Lx, Ly=m.Ly, tau=m.tau, walls_y=True, inout=True, d_p=m.d_p,
                    u0=(U, 0.0), u_in=U, rho_out=1.0, storage="f32")
        out.append((spec, m))
    return out


def test_batch_gradient_fp32_ignores_stale_workspace():
    """The batched gradient with its workspace filled with 0xFF bytes (NaN as FP32 and
    FP64) and 17 steps (checkpoints every 5, a short last segment): every member
    against the oracle's FP64 reverse pass."""
    from paper_1406_6438_amd import lbm
    members = _member_specs("f32", "open_walls", sizes=[(24, 10), (70, 9)])
    nsteps, K = 17, 5
    sv = _solvers(members)
    b = lbm.Batch(sv)
    nbytes = lbm.lbm_vans_batch_grad_work_bytes(b.b, lbm.OBJ_OUTLET_FLUX, nsteps, K)
    gw = torch.full((nbytes,), 0xFF, dtype=torch.uint8, device="cuda")
    gs = [torch.empty((spec.Ly, spec.Lx), dtype=torch.float64, device="cuda")
          for spec, _ in members]
    J = lbm.lbm_vans_batch_grad(b.b, lbm.OBJ_OUTLET_FLUX, nsteps, K, gw, gs)
    torch.cuda.synchronize()
    for (spec, eps), Jb, gb in zip(members, J, gs):
        Jo, go = oracle.grad_outlet_flux(spec.oracle(), spec.input_eps(eps), nsteps)
        gb = gb.cpu().numpy()
        say(f"[batch grad stale workspace] {spec.Lx}x{spec.Ly}: J rel {abs(Jb - Jo) / abs(Jo):.2e}, "
            f"grad rel L2 {rel_l2(gb, go):.2e}")
        assert np.isfinite(gb).all()
        assert abs(Jb - Jo) <= 1e-5 * abs(Jo)
        assert rel_l2(gb, go) <= 1e-4
    b.close()
    _close(sv)


def test_full_ensemble_2000_steps():
    """The 64-member ensemble, autotuned, 2000 steps: the three smallest members
    against the oracle (rel. L2(u) <= 1e-5), every member against a lone run
    (rel. L2(u) <= 1e-5)."""
    from paper_1406_6438_amd import lbm
    ens = _ensemble_specs()
    say(f"[ensemble] {len(ens)} members, {sum(s.Lx * s.Ly for s, _ in ens) / 1e6:.1f}M nodes")
    sv = [lbm.Solver(s.gpu(), s.input_eps(m.porosity())) for s, m in ens]
    b = lbm.Batch(sv)
    best, _ = b.tune(reps=3)
    say(f"  tuned: {best}")
    b.step(W.ENSEMBLE_STEPS)
    torch.cuda.synchronize()
    order = np.argsort([s.Lx * s.Ly for s, _ in ens])
    for k in order[:3]:
        spec, m = ens[k]
        eps = m.porosity()
        mo, _ = oracle_run(spec, eps, W.ENSEMBLE_STEPS)
        mg = sv[k].moments()
        e = rel_l2(mg["ux"].double().cpu().numpy(), mo["ux"])
        say(f"  member {k} {spec.Lx}x{spec.Ly} tau {spec.tau:.3f}: rel L2(ux) {e:.3e}")
        assert e <= 1e-5
        assert rel_l2(mg["uy"].double().cpu().numpy(), mo["uy"]) <= 1e-5 * max(
            1.0, np.linalg.norm(mo["ux"]) / max(np.linalg.norm(mo["uy"]), 1e-300))
    same = 0
    for k, ((spec, m), s) in enumerate(zip(ens, sv)):
        lone = lbm.Solver(spec.gpu(), spec.input_eps(m.porosity()))
        lone.step(W.ENSEMBLE_STEPS)
        same += int(torch.equal(s.get_state(), lone.get_state()))
        e = rel_l2(s.moments()["ux"].double().cpu().numpy(),
                   lone.moments()["ux"].double().cpu().numpy())
        assert e <= 1e-5, f"member {k}: rel L2(ux) {e:.2e} against its lone run"
        lone.close()
    say(f"  {same} of {len(ens)} members have the same bits as their lone runs")
    b.close()
    _close(sv)


def test_full_ensemble_gradient():
    """Gradient of every member's outlet flux after 2000 steps (checkpoints every
    45): the two smallest members against the oracle's FP64 reverse pass
    (rel. L2 <= 1e-4), the largest against its lone run (rel. L2 <= 3e-5).  The
    lone run and the batch may round the FP32 forward differently (a lone lattice
    and the batch may take different steps per pass), so they agree to the FP32
    gradient's own error (the reverse steps run in FP64 on both sides)."""
    from paper_1406_6438_amd import lbm
    ens = _ensemble_specs()
    sv = [lbm.Solver(s.gpu(), s.input_eps(m.porosity())) for s, m in ens]
    b = lbm.Batch(sv)
    J, g = b.grad(W.ENSEMBLE_STEPS, W.ENSEMBLE_CKPT)
    assert all(np.isfinite(J))
    order = np.argsort([s.Lx * s.Ly for s, _ in ens])
    for k in order[:2]:
        spec, m = ens[k]
        eps = spec.input_eps(m.porosity())
        Jo, go = oracle.grad_outlet_flux(spec.oracle(), eps, W.ENSEMBLE_STEPS)
        gb = g[k].cpu().numpy()
        say(f"[ensemble grad] member {k} {spec.Lx}x{spec.Ly}: J rel "
            f"{abs(J[k] - Jo) / abs(Jo):.2e}, grad rel L2 {rel_l2(gb, go):.2e}")
        assert abs(J[k] - Jo) <= 1e-5 * abs(Jo)
        assert rel_l2(gb, go) <= 1e-4
    k = int(order[-1])
    spec, m = ens[k]
    gk = g[k].clone()
    del g
    b.close()
    _close(sv)
    lone = lbm.Solver(spec.gpu(), spec.input_eps(m.porosity()))
    Jl, gl = lone.grad(W.ENSEMBLE_STEPS, W.ENSEMBLE_CKPT)
    lone.close()
    say(f"  largest member: lone gradient same bits {Jl == J[k] and torch.equal(gl, gk)}")
    assert abs(Jl - J[k]) <= 1e-6 * abs(Jl)
    e = rel_l2(gk.cpu().numpy(), gl.cpu().numpy())
    say(f"  largest member: rel L2 against the lone gradient {e:.2e}")
    assert e <= 3e-5
