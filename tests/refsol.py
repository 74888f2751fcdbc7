"""Independent reference results used to pin the oracle (test-side only).

Nothing here calls the oracle or the GPU library.  Each function states the
source of the result it returns:

* ``brinkman_channel``      -- closed form of the fully developed porous channel
                               without the Forchheimer term;
* ``bf_channel``            -- the same ODE with the Forchheimer term, solved as a
                               boundary value problem by scipy;
* ``ergun_pressure_gradient`` -- Ergun's packed-bed equation in its textbook form;
* ``uniform_steady_velocity`` -- root of the uniform Darcy-Forchheimer balance by
                               bracketing (no closed form is used);
* ``TextbookLBGK``          -- plain D2Q9 LBGK with Guo forcing in Hermite form,
                               its own velocity ordering and pull streaming.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.integrate import solve_bvp
from scipy.optimize import brentq


def brinkman_channel(H: float, nu: float, eps: float, a: float, G: float,
                     y: np.ndarray) -> np.ndarray:
    """Solution of nu*eps*u'' - a*u + G = 0, u(0) = u(H) = 0.

    This is the x-momentum balance of the forced volume-averaged equations
    (eq. (VNS3)) for fully developed flow between plates at rest, rho = 1,
    uniform eps, linear drag a*u.
    """
    r = math.sqrt(a / (nu * eps))
    return (G / a) * (1.0 - np.cosh(r * (y - 0.5 * H)) / math.cosh(0.5 * r * H))


def bf_channel(H: float, nu: float, eps: float, a: float, b: float, G: float,
               y: np.ndarray, u_top: float = 0.0) -> np.ndarray:
    """Solution of nu*eps*u'' - a*u - b*|u|*u + G = 0, u(0) = 0, u(H) = u_top.

    With G = 0 and u_top = u0 this is the Couette ODE of the paper (eq. (velocity))
    multiplied by eps; with G > 0 and u_top = 0 it is the body-force driven channel.
    """
    def rhs(s, Y):
        u, du = Y
        return np.vstack([du, (a * u + b * np.abs(u) * u - G) / (nu * eps)])

    def bc(Ya, Yb):
        return np.array([Ya[0], Yb[0] - u_top])

    s = np.linspace(0.0, H, 401)
    guess = np.vstack([np.zeros_like(s), np.zeros_like(s)])
    sol = solve_bvp(rhs, bc, s, guess, tol=1e-10, max_nodes=200000)
    assert sol.status == 0, sol.message
    return sol.sol(y)[0]


def ergun_pressure_gradient(U_s: float, mu: float, rho: float, eps: float, d_p: float) -> float:
    """Ergun (1952): -dP/dL = 150 mu (1-eps)^2 U_s / (eps^3 d_p^2)
                              + 1.75 rho (1-eps) U_s^2 / (eps^3 d_p),
    U_s the superficial velocity."""
    return (150.0 * mu * (1.0 - eps) ** 2 * U_s / (eps ** 3 * d_p ** 2)
            + 1.75 * rho * (1.0 - eps) * U_s ** 2 / (eps ** 3 * d_p))


def uniform_steady_velocity(G: float, drag_of_u) -> float:
    """u* > 0 with drag_of_u(u*) = G, found by bracketing."""
    hi = 1.0
    while drag_of_u(hi) < G:
        hi *= 2.0
    return brentq(lambda u: drag_of_u(u) - G, 0.0, hi, xtol=1e-300, rtol=1e-15, maxiter=500)


class TextbookLBGK:
    """D2Q9 LBGK with the Guo-Zheng-Shi forcing, written in Hermite form.

    f^eq_k = w_k rho [1 + c_k.u/cs2 + (c_k c_k - cs2 I):uu / (2 cs2^2)]
    F_k    = (1 - 1/(2 tau)) w_k [c_k.F/cs2 + (c_k c_k - cs2 I):(uF + Fu) / (2 cs2^2)]
    rho = sum f,  rho u = sum c f + F/2,  pull streaming with np.roll.
    Velocities are ordered (0,0),(1,0),(-1,0),(0,1),(0,-1),(1,1),(-1,-1),(1,-1),(-1,1)
    and weights follow from |c|^2.  ``walls_y`` puts half-way bounce-back walls
    below row 0 and above row Ly-1.
    """

    C = np.array([(0, 0), (1, 0), (-1, 0), (0, 1), (0, -1), (1, 1), (-1, -1), (1, -1), (-1, 1)])

    def __init__(self, tau: float, G=(0.0, 0.0), walls_y: bool = False):
        self.tau = tau
        self.G = np.asarray(G, dtype=np.float64)
        self.walls_y = walls_y
        c2 = (self.C ** 2).sum(1)
        self.w = np.where(c2 == 0, 4.0 / 9.0, np.where(c2 == 1, 1.0 / 9.0, 1.0 / 36.0))
        self.cs2 = 1.0 / 3.0
        self.Q = (self.C[:, :, None] * self.C[:, None, :]).astype(np.float64) \
            - self.cs2 * np.eye(2)[None]
        self.opp = np.array([int(np.where((self.C == -c).all(1))[0][0]) for c in self.C])

    def permutation_from(self, ex, ey):
        """perm[k] = index in the (ex, ey) ordering of this class's velocity k."""
        vecs = list(zip(ex, ey))
        return np.array([vecs.index((int(c[0]), int(c[1]))) for c in self.C])

    def macros(self, f):
        rho = f.sum(0)
        j = np.einsum("kd,kyx->dyx", self.C.astype(np.float64), f)
        u = (j + 0.5 * self.G[:, None, None]) / rho
        return rho, u

    def feq(self, rho, u):
        cu = np.einsum("kd,dyx->kyx", self.C.astype(np.float64), u)
        Quu = np.einsum("kab,ayx,byx->kyx", self.Q, u, u)
        return self.w[:, None, None] * rho * (1.0 + cu / self.cs2 + Quu / (2 * self.cs2 ** 2))

    def force(self, u):
        F = np.broadcast_to(self.G[:, None, None], u.shape)
        cF = np.einsum("kd,dyx->kyx", self.C.astype(np.float64), F)
        QuF = np.einsum("kab,ayx,byx->kyx", self.Q, u, F)
        return (1 - 0.5 / self.tau) * self.w[:, None, None] * (
            cF / self.cs2 + 2.0 * QuF / (2 * self.cs2 ** 2))

    def step(self, f):
        rho, u = self.macros(f)
        post = f - (f - self.feq(rho, u)) / self.tau + self.force(u)
        new = np.empty_like(post)
        for k, (cx, cy) in enumerate(self.C):
            new[k] = np.roll(post[k], shift=(cy, cx), axis=(0, 1))
            if self.walls_y and cy == 1:
                new[k][0, :] = post[self.opp[k]][0, :]
            if self.walls_y and cy == -1:
                new[k][-1, :] = post[self.opp[k]][-1, :]
        return new
