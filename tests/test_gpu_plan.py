"""The launch plan lbm_vans_step and lbm_vans_batch_step follow (lbm_vans_pass_plan):
explicit settings are taken as given, and the automatic choice follows its rule.

The rule counts the waves of the three-step pass (60 columns x 24 or 28 rows each)
against the waves the GPU holds of that kernel at once: three steps per pass from
0.7 times as many, 28-row chunks from 4 times as many, else two steps when the
two-step pass has >= 2048 waves (62 columns x 8 rows), else one.  On MI355X (256
compute units) the periodic FP32 kernel holds 3 waves per SIMD (3072 on the chip)
and the FP32 kernel with walls and open ends 2 (2048), so the cases below sit
clearly on one side of each threshold:

* 4096^2 periodic box: 69 x 147 = 10143 waves of 28 rows < 4 x 3072 -> 24 rows;
  69 x 171 = 11799 >= 0.7 x 3072 -> (3, 24);
* 2048^2 box: 35 x 74 = 2590 < 12288 -> 24 rows; 35 x 86 = 3010 >= 2150 -> (3, 24);
* 1024^2 box: 18 x 43 = 774 < 2150; two-step 17 x 128 = 2176 >= 2048 -> (2, 24);
* 1024 x 512 channel (open x, walls y): 18 x 22 = 396 < 1434; 17 x 64 = 1088 < 2048
  -> (1, 24);
* 4096^2 channel: 10143 >= 4 x 2048 -> 28 rows -> (3, 28);
* FP64 storage: no multi-step pass -> (1, 0).
(Both 4096^2 choices sit within 1% of the other chunk height: box 163.6 / 163.0,
channel 151.9 / 155.0 GLUPS at 24 / 28 rows.)
"""
import numpy as np
import pytest

from parity_util import say

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1406_6438_amd import lbm
    lbm.load()


def _plan(Lx, Ly, channel=False, storage="f32", **kw):
    from paper_1406_6438_amd import lbm
    extra = dict(bc_x=lbm.BC_OPEN, bc_y=lbm.BC_BOUNCEBACK, u0=(0.02, 0.0), u_in=0.02,
                 u_out=0.02) if channel else {}
    p = lbm.Params(Lx=Lx, Ly=Ly, tau=0.7, d_p=20.0, storage=lbm.STORAGE[storage], **extra, **kw)
    eps = np.full((Ly, Lx), 0.7)
    s = lbm.Solver(p, eps)
    plan = s.pass_plan
    s.close()
    del s
    torch.cuda.empty_cache()
    say(f"[plan] {Lx}x{Ly} {'channel' if channel else 'box'} {storage} {kw}: {plan}")
    return plan


@pytest.mark.parametrize("Lx, Ly, channel, storage, expected", [
    (4096, 4096, False, "f32", (4, 24)),
    (2048, 2048, False, "f32", (4, 24)),
    (2048, 1024, False, "f32", (3, 12)),
    (1024, 1024, False, "f32", (3, 12)),
    (1024, 512, True, "f32", (3, 6)),
    (1024, 1024, True, "f32", (3, 6)),
    (2048, 2048, True, "f32", (3, 12)),
    (512, 512, False, "f32", (3, 6)),
    (512, 256, False, "f32", (1, 6)),
    (4096, 4096, True, "f32", (4, 24)),
    (4096, 4096, False, "f16", (3, 24)),
    (64, 32, False, "f64", (1, 0)),
])
def test_automatic_plan(Lx, Ly, channel, storage, expected):
    assert _plan(Lx, Ly, channel, storage) == expected


@pytest.mark.parametrize("kw, expected", [
    (dict(steps_per_pass=2, pass_rows=28), (2, 28)),
    (dict(steps_per_pass=3, pass_rows=24), (3, 24)),
    (dict(steps_per_pass=3, pass_rows=28), (3, 28)),
    (dict(steps_per_pass=3, pass_rows=12), (3, 12)),
    (dict(steps_per_pass=3, pass_rows=6), (3, 6)),
    (dict(steps_per_pass=4), (4, 24)),
    (dict(steps_per_pass=4, pass_rows=12), (4, 24)),
    (dict(steps_per_pass=1), (1, 6)),
])
def test_explicit_plan(kw, expected):
    assert _plan(96, 40, **kw) == expected


def test_batch_plan():
    from paper_1406_6438_amd import lbm
    eps = np.full((40, 96), 0.7)
    sv = [lbm.Solver(lbm.Params(Lx=96, Ly=40, tau=0.7, d_p=20.0), eps) for _ in range(2)]
    b = lbm.Batch(sv)
    assert b.pass_plan == (3, 24)            # default: three steps, small batch -> 24 rows
    b.configure(4, 0, 24, 3, 28)
    assert b.pass_plan == (3, 28)
    b.configure(4, 0, 24, 2, 0)
    assert b.pass_plan == (2, 24)
    b.configure(4, 0, 24, 4, 0)
    assert b.pass_plan == (4, 24)
    with pytest.raises(lbm.LbmVansError):      # the 12- and 6-row heights are for lone lattices
        b.configure(4, 0, 24, 3, 12)
    with pytest.raises(lbm.LbmVansError):
        b.configure(4, 0, 24, 3, 6)
    b.close()
    for s in sv:
        s.close()
    s64 = [lbm.Solver(lbm.Params(Lx=96, Ly=40, tau=0.7, d_p=20.0, storage=lbm.F64), eps)]
    b64 = lbm.Batch(s64)
    assert b64.pass_plan == (1, 0)
    b64.close()
    s64[0].close()


@pytest.mark.parametrize("storage, L", [("f64", (80, 80)), ("f32", (64, 32)), ("f32", (130, 40))])
def test_step_graph_replays_match_plain_launches(storage, L):
    """Lattices with fewer sweep tiles than twice the compute units replay their steps as
    captured graphs of 32 steps (lbm_vans_step with 32 or more steps); a single step per
    call launches plainly.  Several replays, with eager work (moments, a state copy) and
    synchronisations between them, against the same steps taken one per call: the same
    bits at every check."""
    from paper_1406_6438_amd import lbm, workloads as W
    Lx, Ly = L
    p = lbm.Params(Lx=Lx, Ly=Ly, tau=0.7, d_p=8.0, G=(1e-5, 0.0), bc_y=lbm.BC_BOUNCEBACK,
                   storage=lbm.STORAGE[storage], u_wall=(0.0, 0.01))
    eps = W.grf_porosity(Lx, Ly, seed=77, ell=4.0, lo=0.4, hi=1.0)
    a = lbm.Solver(p, eps)
    b = lbm.Solver(p, eps)
    a.step(1)                      # the graphs start from a state n >= 1
    b.step(1)
    for chunk in (32, 64, 40, 96):
        a.step(chunk)
        for _ in range(chunk):
            b.step(1)
        fa, fb = a.get_state(), b.get_state()
        ma = a.moments()
        torch.cuda.synchronize()
        say(f"[graphs {storage} {Lx}x{Ly}] n = {a.n}: same bits {torch.equal(fa, fb)}")
        assert a.n == b.n and torch.equal(fa, fb) and ma["rc"] == 0
    a.close()
    b.close()
