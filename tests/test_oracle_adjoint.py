"""Pins of the oracle's open boundaries and of its reverse-mode gradient of the
outlet mass flux, against finite differences and exact fixed points."""
import math

import numpy as np
import pytest

from paper_1406_6438_amd import workloads as W

RNG = np.random.Generator(np.random.PCG64(6438))


def _open_channel(orc, Lx, Ly, walls=True, **kw):
    args = dict(Lx=Lx, Ly=Ly, tau=0.7, bc_x=orc.OPEN, bc_y=orc.WALL if walls else orc.PERIODIC,
                d_p=6.0, rho_in=1.0, u_in=0.02, rho_out=1.0, u_out=0.02)
    args.update(kw)
    return orc.Params(**args)


@pytest.mark.parametrize("eps", [0.3, 0.55, 0.8, 0.97])
@pytest.mark.parametrize("const", [False, True])
def test_drag_derivatives_match_finite_differences(orc, eps, const):
    p = (orc.Params(Lx=1, Ly=1, tau=0.8, drag=orc.DRAG_CONST, K=3.0, F_eps=0.4) if const
         else orc.Params(Lx=1, Ly=1, tau=0.8, d_p=9.0))
    h = 1e-6
    ap, bp = orc.drag_coeffs(p, eps + h)
    am, bm = orc.drag_coeffs(p, eps - h)
    da, db = orc.drag_derivs(p, eps)
    assert abs(da - (ap - am) / (2 * h)) <= 1e-8 * max(abs(da), 1e-12)
    assert abs(db - (bp - bm) / (2 * h)) <= 1e-8 * max(abs(db), 1e-12)


@pytest.mark.parametrize("trial", range(12))
def test_node_vjp_matches_directional_derivative(orc, trial):
    """<vjp(mu), delta> equals the central difference of <mu, fpost> + S_bar S + u_bar.u
    along a random direction delta in (f, eps, grad eps)."""
    p = orc.Params(Lx=1, Ly=1, tau=RNG.uniform(0.55, 1.2), d_p=RNG.uniform(2.0, 20.0),
                   Gx=RNG.uniform(-1e-3, 1e-3), Gy=RNG.uniform(-1e-3, 1e-3))
    eps = RNG.uniform(0.35, 0.95)
    f = orc.feq(eps * RNG.uniform(0.95, 1.05), *RNG.uniform(-0.05, 0.05, 2))
    f *= 1.0 + RNG.uniform(-0.02, 0.02, 9)
    gex, gey = RNG.uniform(-0.05, 0.05, 2)
    mu = RNG.standard_normal(9)
    sb, uxb, uyb = RNG.standard_normal(3)
    df, de, dgx, dgy = RNG.standard_normal(9), RNG.standard_normal(), *RNG.standard_normal(2)

    def phi(t):
        ff = f + t * df
        e = eps + t * de
        gx, gy = gex + t * dgx, gey + t * dgy
        post = orc.node_collide(p, ff, e, gx, gy)
        ux, uy, rho = orc.velocity(p, ff.sum(), *(np.array([[0, 1, 0, -1, 0, 1, -1, -1, 1],
                                                             [0, 0, 1, 0, -1, 1, 1, -1, -1]]) @ ff),
                                   e, gx, gy)
        return mu @ post + sb * ff.sum() + uxb * ux + uyb * uy

    h = 1e-6
    fd = (phi(h) - phi(-h)) / (2 * h)
    fb, eb, gxb, gyb = orc.node_vjp(p, f, eps, gex, gey, mu, sb, uxb, uyb)
    ad = fb @ df + eb * de + gxb * dgx + gyb * dgy
    assert abs(ad - fd) <= 1e-7 * max(1.0, abs(fd))


def test_open_channel_keeps_uniform_through_flow(orc):
    """Uniform porosity, no drag, no force, periodic in y, reservoirs at the flow's own
    density and velocity: the uniform flow f^eq(eps rho0, U) is a fixed point, so the
    reservoir populations enter in the right directions with the right velocity."""
    Lx, Ly, U = 16, 5, 0.03
    p = orc.Params(Lx=Lx, Ly=Ly, tau=0.7, bc_x=orc.OPEN, rho_in=1.0, u_in=U, rho_out=1.0,
                   u_out=U, u0x=U)
    eps = np.full((Ly, Lx), 0.6)
    f0 = orc.init(p, eps)
    f = orc.steps(p, eps, f0, 100)
    assert np.abs(f - f0).max() < 1e-15
    m = orc.moments(p, eps, f)
    assert np.allclose(m["ux"], U, rtol=1e-13) and np.allclose(m["rho"], 1.0, rtol=1e-14)


def test_open_channel_mass_budget(orc):
    """Sum of eps rho changes each step by what the reservoirs inject minus what leaves
    across the open sections."""
    p = _open_channel(orc, 14, 8, u0x=0.01)
    eps = W.grf_porosity(14, 8, seed=21, ell=3.0, lo=0.4, hi=1.0)
    ex, ey, *_ = orc.lattice()
    f = orc.steps(p, eps, orc.init(p, eps), 30)
    post = orc.collide(p, eps, f)
    f1 = orc.stream(p, eps, post)
    left = sum(post[i, :, 0].sum() for i in range(9) if ex[i] < 0 and ey[i] == 0)
    right = sum(post[i, :, -1].sum() for i in range(9) if ex[i] > 0 and ey[i] == 0)
    # diagonals leave unless they bounce at a wall row
    for i in range(9):
        if ex[i] != 0 and ey[i] != 0:
            col = 0 if ex[i] < 0 else -1
            rows = [y for y in range(8) if 0 <= y + ey[i] < 8]
            if ex[i] < 0:
                left += post[i, rows, col].sum()
            else:
                right += post[i, rows, col].sum()
    inj = 0.0
    for i in range(9):
        for y in range(8):
            if ex[i] > 0 and 0 <= y - ey[i] < 8:
                inj += f1[i, y, 0]
            if ex[i] < 0 and 0 <= y - ey[i] < 8:
                inj += f1[i, y, -1]
    assert abs(f1.sum() - (post.sum() - left - right + inj)) < 1e-13


@pytest.mark.parametrize("walls", [True, False])
def test_gradient_matches_central_differences(orc, walls):
    """dJ/deps from the reverse pass against central differences of J for every
    node of a small open channel (FP64, h = 1e-6)."""
    Lx, Ly, n = 12, 6, 60
    p = _open_channel(orc, Lx, Ly, walls=walls, Gx=2e-5, u0x=0.01)
    eps = W.grf_porosity(Lx, Ly, seed=33, ell=2.5, lo=0.4, hi=0.95)
    J, g = orc.grad_outlet_flux(p, eps, n)
    assert abs(J - orc.outlet_flux(p, eps, orc.run(p, eps, n))) == 0.0
    h = 1e-6
    fd = np.zeros_like(eps)
    for y in range(Ly):
        for x in range(Lx):
            e = eps.copy()
            e[y, x] += h
            jp = orc.outlet_flux(p, e, orc.run(p, e, n))
            e[y, x] -= 2 * h
            jm = orc.outlet_flux(p, e, orc.run(p, e, n))
            fd[y, x] = (jp - jm) / (2 * h)
    err = np.abs(g - fd).max() / np.abs(fd).max()
    assert err <= 1e-7, err


def test_gradient_periodic_and_const_drag(orc):
    """Periodic box with a body force and the constant-K drag law (no open boundary,
    no walls): the gradient still matches central differences."""
    Lx, Ly, n = 9, 7, 40
    p = orc.Params(Lx=Lx, Ly=Ly, tau=0.9, drag=orc.DRAG_CONST, K=5.0, F_eps=0.3, Gx=3e-5,
                   Gy=-1e-5, u0x=0.02)
    eps = W.grf_porosity(Lx, Ly, seed=34, ell=2.0, lo=0.4, hi=0.95)
    J, g = orc.grad_outlet_flux(p, eps, n)
    h = 1e-6
    for (y, x) in [(0, 0), (3, 4), (6, 8), (2, 7), (5, 1)]:
        e = eps.copy()
        e[y, x] += h
        jp = orc.outlet_flux(p, e, orc.run(p, e, n))
        e[y, x] -= 2 * h
        jm = orc.outlet_flux(p, e, orc.run(p, e, n))
        fd = (jp - jm) / (2 * h)
        assert abs(g[y, x] - fd) <= 1e-7 * np.abs(g).max()


def test_gradient_with_sliding_walls(orc):
    """Open channel between plates sliding in opposite directions: the reverse pass
    against central differences of J at every node."""
    Lx, Ly, n = 10, 6, 50
    p = _open_channel(orc, Lx, Ly, walls=True, uw_bot=-0.03, uw_top=0.05, u0x=0.01)
    eps = W.grf_porosity(Lx, Ly, seed=35, ell=2.5, lo=0.4, hi=0.95)
    J, g = orc.grad_outlet_flux(p, eps, n)
    h = 1e-6
    fd = np.zeros_like(eps)
    for y in range(Ly):
        for x in range(Lx):
            e = eps.copy()
            e[y, x] += h
            jp = orc.outlet_flux(p, e, orc.run(p, e, n))
            e[y, x] -= 2 * h
            jm = orc.outlet_flux(p, e, orc.run(p, e, n))
            fd[y, x] = (jp - jm) / (2 * h)
    assert np.abs(g - fd).max() <= 1e-7 * np.abs(fd).max()
