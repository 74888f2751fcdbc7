"""The launch plan lbm_vans_step and lbm_vans_batch_step follow (lbm_vans_pass_plan):
explicit settings are taken as given, and the automatic choice follows its rule.

The rule counts the waves of the three-step pass (60 columns x 24 or 28 rows each)
against the waves the GPU holds of that kernel at once: three steps per pass from
0.7 times as many, 28-row chunks from 4 times as many, else two steps when the
two-step pass has >= 2048 waves (62 columns x 8 rows), else one.  On MI355X (256
compute units) the periodic FP32 kernel holds 2 waves per SIMD (2048 on the chip)
and the kernels with walls 4 (4096), so the cases below sit clearly on one side
of each threshold:

* 4096^2 periodic box: 69 x 147 = 10143 waves of 28 rows >= 4 x 2048 -> (3, 28);
* 2048^2 box: 35 x 74 = 2590 < 8192 -> 24 rows; 35 x 86 = 3010 >= 0.7 x 2048 -> (3, 24);
* 1024^2 box: 18 x 43 = 774 < 1434; two-step 17 x 128 = 2176 >= 2048 -> (2, 24);
* 1024 x 512 channel (open x, walls y): 18 x 22 = 396 < 2867; 17 x 64 = 1088 < 2048
  -> (1, 24);
* 4096^2 channel: 10143 < 4 x 4096 -> 24 rows; 69 x 171 = 11799 >= 2867 -> (3, 24);
* FP64 storage: no multi-step pass -> (1, 0).
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
    (4096, 4096, False, "f32", (3, 28)),
    (2048, 2048, False, "f32", (3, 24)),
    (1024, 1024, False, "f32", (2, 24)),
    (1024, 512, True, "f32", (1, 24)),
    (4096, 4096, True, "f32", (3, 24)),
    (4096, 4096, False, "f16", (3, 24)),
    (64, 32, False, "f64", (1, 0)),
])
def test_automatic_plan(Lx, Ly, channel, storage, expected):
    assert _plan(Lx, Ly, channel, storage) == expected


@pytest.mark.parametrize("kw, expected", [
    (dict(steps_per_pass=2, pass_rows=28), (2, 28)),
    (dict(steps_per_pass=3, pass_rows=24), (3, 24)),
    (dict(steps_per_pass=3, pass_rows=28), (3, 28)),
    (dict(steps_per_pass=1), (1, 24)),
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
    b.close()
    for s in sv:
        s.close()
    s64 = [lbm.Solver(lbm.Params(Lx=96, Ly=40, tau=0.7, d_p=20.0, storage=lbm.F64), eps)]
    b64 = lbm.Batch(s64)
    assert b64.pass_plan == (1, 0)
    b64.close()
    s64[0].close()
