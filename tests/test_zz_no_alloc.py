"""The allocation-free gradient entry point, lbm_vans_grad_static, through the C-ABI.

For callers that cannot allocate device memory the library keeps the gradient's
workspace in a fixed array of its own on each GPU.  Its results must equal those of
lbm_vans_grad with a caller buffer (the same kernels on a workspace at another
address: the same bits), on two calls in a row on one GPU, the second on a smaller
problem (a shorter run on a smaller lattice, so that stale contents of the larger
first call sit beyond and inside the second's workspace), and must match the FP64
oracle's reverse pass as lbm_vans_grad does.  A problem whose workspace exceeds the
array is refused with EINVAL before any work is queued.
"""
import numpy as np
import pytest

import oracle
from parity_util import Spec, rel_l2, say
from paper_1406_6438_amd import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1406_6438_amd import lbm
    lbm.load()


def _spec(Lx, Ly, storage):
    return Spec(Lx=Lx, Ly=Ly, tau=0.75, walls_y=True, inout=True, d_p=8.0, u_in=0.02,
                rho_out=1.0, u0=(0.02, 0.0), storage=storage)


def _both(spec, eps, nsteps, K):
    """(J, dJ/deps) from lbm_vans_grad with a caller buffer and from lbm_vans_grad_static."""
    from paper_1406_6438_amd import lbm
    s = lbm.Solver(spec.gpu(), spec.input_eps(eps))
    nbytes = lbm.lbm_vans_grad_work_bytes(s.p, lbm.OBJ_OUTLET_FLUX, nsteps, K)
    assert nbytes <= lbm.GRAD_STATIC_BYTES
    gw = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    g1 = torch.empty((spec.Ly, spec.Lx), dtype=torch.float64, device="cuda")
    g2 = torch.empty_like(g1)
    J1 = lbm.lbm_vans_grad(s.h, lbm.OBJ_OUTLET_FLUX, nsteps, K, gw, g1)
    J2 = lbm.lbm_vans_grad_static(s.h, lbm.OBJ_OUTLET_FLUX, nsteps, K, g2)
    torch.cuda.synchronize()
    assert s.n == nsteps
    s.close()
    return J1, g1.cpu().numpy(), J2, g2.cpu().numpy()


@pytest.mark.parametrize("storage", ["f32", "f64"])
def test_static_gradient_equals_caller_buffer_gradient_twice(storage):
    for (Lx, Ly, nsteps, K) in [(130, 40, 120, 20), (61, 17, 45, 9)]:
        say(f"[grad static {storage}] {Lx}x{Ly}, {nsteps} steps, K = {K}")
        spec = _spec(Lx, Ly, storage)
        eps = W.grf_porosity(Lx, Ly, seed=2000 + Lx, ell=4.0, lo=0.4, hi=1.0)
        J1, g1, J2, g2 = _both(spec, eps, nsteps, K)
        assert J1 == J2 and np.array_equal(g1, g2)
        Jo, go = oracle.grad_outlet_flux(spec.oracle(), spec.input_eps(eps), nsteps)
        # J of these short runs is a small net flux (the inflow has not crossed the
        # channel yet): hold it against the inflow's scale, Ly u_in
        scale = spec.Ly * spec.u_in
        say(f"  J diff / (Ly u_in) {abs(J2 - Jo) / scale:.2e}, grad rel L2 {rel_l2(g2, go):.2e}")
        if storage == "f64":
            assert abs(J2 - Jo) <= 1e-12 * scale
            assert np.abs(g2 - go).max() <= 1e-10 * np.abs(go).max()
        else:
            assert abs(J2 - Jo) <= 1e-5 * scale
            assert rel_l2(g2, go) <= 1e-4


def test_static_gradient_refuses_a_workspace_beyond_its_size():
    from paper_1406_6438_amd import lbm
    spec = _spec(512, 256, "f32")
    s = lbm.Solver(spec.gpu(), spec.input_eps(W.uniform_porosity(512, 256, 0.6)))
    need = lbm.lbm_vans_grad_work_bytes(s.p, lbm.OBJ_OUTLET_FLUX, 400, 200)
    assert need > lbm.GRAD_STATIC_BYTES
    g = torch.zeros((256, 512), dtype=torch.float64, device="cuda")
    with pytest.raises(lbm.LbmVansError) as ei:
        lbm.lbm_vans_grad_static(s.h, lbm.OBJ_OUTLET_FLUX, 400, 200, g)
    assert ei.value.code == lbm.EINVAL and "bytes" in str(ei.value)
    assert s.n == 0                     # nothing ran
    s.close()
