"""Seeded synthetic inputs shared by the GPU path and the oracle.

This module holds input synthesis and workload parameters only: porosity
fields, noise arrays and the numeric constants of the benchmark workloads.  It
contains none of the method's arithmetic (no equilibrium, force, velocity or
streaming), so both sides can take their inputs from here without sharing any
part of the computation.

Porosity recipe (the paper treats eps(x) as a given local porosity field;
Section "Conclusions" notes it may vary in space):
  1. white N(0, 1) noise on the lattice from numpy's PCG64 with the given seed;
  2. a periodic Gaussian filter exp(-|k|^2 l^2 / 4) applied in Fourier space,
     so that the filtered field has covariance exp(-r^2 / (2 l^2));
  3. standardisation to zero mean and unit variance;
  4. eps = lo + (hi - lo) Phi(z), Phi the standard normal CDF, which gives
     uniform marginals on [lo, hi] with no clipping.
All of it runs in float64; the result is cast once to the precision a side
needs, so both sides receive bit-identical porosities.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np
from scipy.special import ndtr

SEED = 1406


def grf_porosity(Lx: int, Ly: int, seed: int = SEED, ell: float = 16.0, lo: float = 0.3,
                 hi: float = 1.0) -> np.ndarray:
    """Smooth periodic Gaussian-random-field porosity in [lo, hi], shape (Ly, Lx), float64."""
    rng = np.random.Generator(np.random.PCG64(seed))
    white = rng.standard_normal((Ly, Lx))
    spec = np.fft.rfft2(white)
    ky = 2.0 * np.pi * np.fft.fftfreq(Ly)[:, None]
    kx = 2.0 * np.pi * np.fft.rfftfreq(Lx)[None, :]
    spec *= np.exp(-(kx * kx + ky * ky) * (ell * ell) / 4.0)
    z = np.fft.irfft2(spec, s=(Ly, Lx))
    del spec, white
    z -= z.mean()
    sd = z.std()
    if sd > 0:
        z /= sd
    return lo + (hi - lo) * ndtr(z)


def uniform_porosity(Lx: int, Ly: int, eps: float) -> np.ndarray:
    return np.full((Ly, Lx), float(eps))


def sine_porosity(Lx: int, Ly: int, mean: float = 0.7, amp: float = 0.2) -> np.ndarray:
    """Porosity varying along x only: mean + amp sin(2 pi x / Lx)."""
    x = np.arange(Lx)
    return np.tile(mean + amp * np.sin(2.0 * np.pi * x / Lx), (Ly, 1))


def noise(shape, seed: int, scale: float = 1.0) -> np.ndarray:
    """Seeded uniform noise in [-scale, scale) (float64)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return scale * (2.0 * rng.random(shape) - 1.0)


@dataclasses.dataclass(frozen=True)
class Workload:
    """One synthetic workload: lattice, boundaries, tau, drag, force, steps, porosity recipe."""
    name: str
    Lx: int
    Ly: int
    tau: float
    d_p: float
    Gx: float
    Gy: float
    steps: int
    walls_y: bool
    storage: str                      # "f64", "f32", "f16"
    eps_kind: str                     # "uniform" or "grf"
    eps_value: float = 0.5            # uniform porosity
    eps_lo: float = 0.3
    eps_hi: float = 1.0
    ell: float = 16.0
    seed: int = SEED
    rho0: float = 1.0

    def porosity(self, Lx: int | None = None, Ly: int | None = None) -> np.ndarray:
        Lx = self.Lx if Lx is None else Lx
        Ly = self.Ly if Ly is None else Ly
        if self.eps_kind == "uniform":
            return uniform_porosity(Lx, Ly, self.eps_value)
        return grf_porosity(Lx, Ly, self.seed, self.ell, self.eps_lo, self.eps_hi)


def ergun_dp_for_darcy(Da: float, L: float, eps_ref: float) -> float:
    """Particle diameter that gives permeability K = Da L^2 at porosity eps_ref under the
    Ergun closure K = eps^3 d_p^2 / (150 (1 - eps)^2) (parameter choice, not method)."""
    return math.sqrt(150.0 * Da) * L * (1.0 - eps_ref) / eps_ref ** 1.5


# Porous channel, 64 x 32 nodes, periodic in x, half-way bounce-back walls in y,
# uniform eps = 0.5, tau = 0.8 (nu = 0.1), Da = K/H^2 = 1e-2 on H = 32
# (K = 10.24, d_p = sqrt(3072)), body force chosen so that the peak velocity of
# the Brinkman profile is nu/H (Re = 1 on the channel width), 2000 steps, FP64.
CHANNEL_64x32 = Workload(
    name="porous_channel_64x32_f64", Lx=64, Ly=32, tau=0.8,
    d_p=ergun_dp_for_darcy(1e-2, 32.0, 0.5), Gx=8.1012e-6, Gy=0.0, steps=2000,
    walls_y=True, storage="f64", eps_kind="uniform", eps_value=0.5)

# Periodic box 4096^2, GRF porosity (l = 16) mapped into [0.3, 1.0], tau = 0.6,
# body force 1e-6 along x, d_p from Da = 1e-2 on the correlation length at the
# median porosity 0.65, 1000 steps, FP32 populations.
BOX_4096_F32 = Workload(
    name="porous_box_4096x4096_f32", Lx=4096, Ly=4096, tau=0.6,
    d_p=ergun_dp_for_darcy(1e-2, 16.0, 0.65), Gx=1e-6, Gy=0.0, steps=1000,
    walls_y=False, storage="f32", eps_kind="grf")

# The same box at 8192^2 with FP16 populations, 2000 steps.
BOX_8192_F16 = dataclasses.replace(
    BOX_4096_F32, name="porous_box_8192x8192_f16", Lx=8192, Ly=8192, steps=2000, storage="f16")

# 512 x 512 crop runs used for accuracy statements of the box workloads: the
# top-left 512^2 block of the full porosity field, run periodic.
CROP = 512


def crop_porosity(w: Workload, n: int = CROP) -> np.ndarray:
    """Top-left n x n block of the workload's full porosity field."""
    return np.ascontiguousarray(w.porosity()[:n, :n])

# Porous channel with through-flow for the gradient of the outlet mass flux:
# 1024 x 512 nodes, half-way bounce-back walls in y, a velocity inlet
# (x-velocity 0.02) at x = 0 and a pressure outlet (density 1) at x = Lx-1,
# GRF porosity in [0.4, 1.0] (l = 16, seed 1407), tau = 0.8, d_p from Da = 1e-2
# on the channel width at porosity 0.7, plug-flow start (u0 = 0.02), 4000
# steps, FP32, gradient through checkpoints every 200 steps.
ADJOINT_CHANNEL = Workload(
    name="porous_open_channel_1024x512_f32", Lx=1024, Ly=512, tau=0.8,
    d_p=ergun_dp_for_darcy(1e-2, 512.0, 0.7), Gx=0.0, Gy=0.0, steps=4000,
    walls_y=True, storage="f32", eps_kind="grf", eps_lo=0.4, eps_hi=1.0, seed=SEED + 1)
ADJOINT_U_IN = 0.02
ADJOINT_RHO_OUT = 1.0
ADJOINT_CKPT = 200

# Ensemble of independent porous channels advanced together: 64 members, each
# with Lx drawn uniformly from the integers 256..2048 and Ly = Lx // 2 (aspect
# 2:1), tau drawn uniformly from [0.55, 1.0] (both from PCG64(ENSEMBLE_SEED)),
# its own GRF porosity in [0.3, 1.0] (l = 16, seed ENSEMBLE_SEED + 1 + k),
# half-way bounce-back walls in y, a velocity inlet (x-velocity 0.02) and a
# pressure outlet (density 1), plug-flow start, d_p from
# Da = 1e-2 on the member's width at porosity 0.65, no body force, FP32,
# 2000 steps.  The gradient of each member's outlet flux uses a checkpoint
# every 45 steps (about sqrt(2000), which minimises checkpoints + segment).
ENSEMBLE_SEED = SEED + 2
ENSEMBLE_MEMBERS = 64
ENSEMBLE_STEPS = 2000
ENSEMBLE_CKPT = 45
ENSEMBLE_U = 0.02


@dataclasses.dataclass(frozen=True)
class Member:
    """One channel of an ensemble."""
    Lx: int
    Ly: int
    tau: float
    d_p: float
    seed: int
    eps_lo: float = 0.3
    eps_hi: float = 1.0
    ell: float = 16.0

    def porosity(self) -> np.ndarray:
        return grf_porosity(self.Lx, self.Ly, self.seed, self.ell, self.eps_lo, self.eps_hi)


def ensemble(n: int = ENSEMBLE_MEMBERS, lmin: int = 256, lmax: int = 2048,
             seed: int = ENSEMBLE_SEED) -> list:
    """The members of an ensemble of n channels with Lx in [lmin, lmax]."""
    rng = np.random.Generator(np.random.PCG64(seed))
    Lx = rng.integers(lmin, lmax + 1, size=n)
    tau = rng.uniform(0.55, 1.0, size=n)
    out = []
    for k in range(n):
        lx = int(Lx[k])
        ly = max(lx // 2, 1)
        out.append(Member(Lx=lx, Ly=ly, tau=float(tau[k]),
                          d_p=ergun_dp_for_darcy(1e-2, float(ly), 0.65), seed=seed + 1 + k))
    return out

# The paper's Couette experiment (Section "Examples and discussions"): an
# 80 x 80 lattice of uniform porosity 0.1 between two plates, the lower at
# rest (wall at y = -1/2), the upper sliding along x with velocity U (wall at
# y = 79.5), periodic in x; tau = 0.6574 at Re = 50, else 0.8; U = Re nu / 80;
# K = Da 80^2 through the Ergun closure; density 1 and velocity 0 at the
# start.  The paper's figure plots profiles "at different Re and Da" without
# listing them; the cases below span Re 0.1..50 and Da 1e-3..1e-1.  160000
# steps bring every case to a steady state (changes below 1e-11 U per 5000
# steps).
COUETTE_L = 80
COUETTE_EPS = 0.1
COUETTE_STEPS = 160000
COUETTE_CASES = ((50.0, 1e-2), (10.0, 1e-2), (1.0, 1e-2), (0.1, 1e-2), (1.0, 1e-1), (1.0, 1e-3))


@dataclasses.dataclass(frozen=True)
class CouetteCase:
    Re: float
    Da: float
    tau: float
    nu: float
    U: float
    K: float
    d_p: float


def couette_case(Re: float, Da: float, L: int = COUETTE_L, eps: float = COUETTE_EPS) -> CouetteCase:
    tau = 0.6574 if Re == 50.0 else 0.8
    nu = (tau - 0.5) / 3.0
    K = Da * L * L
    d_p = math.sqrt(150.0 * K * (1.0 - eps) ** 2 / eps ** 3)
    return CouetteCase(Re=Re, Da=Da, tau=tau, nu=nu, U=Re * nu / L, K=K, d_p=d_p)
