"""Seeded synthetic inputs for the ultra-relativistic lattice Boltzmann update.

This module holds input recipes only: initial fields (energy density eps,
velocity u, particle density n), obstacle masks, boundary conditions and run
parameters.  It contains none of the lattice update's arithmetic; the same
arrays are handed to the HIP library and to the CPU oracle.

Lattice units: ambient temperature T = 1, n = 1, eps = 3 T^4 = 3 (eps = 3p,
p = nT), nu = 27^(1/4) unless stated.  Seeds are 1302112500 + k for
workload k.  The five workloads are synthetic stand-ins shaped like the
paper's Riemann-problem and shock-cloud experiments (Sec. III); no dataset is
involved.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np

NU_DEFAULT = 27.0 ** 0.25
SEED_BASE = 1302112500

BC_PERIODIC, BC_FIXED, BC_OUTFLOW = 0, 1, 2
FP64, MIXED = 0, 1
COLL_IMPLICIT, COLL_EULER = 0, 1
TAU_UNIFORM, TAU_ETA_OVER_S = 0, 1
LATTICE_EXTENDED, LATTICE_BASIC = 0, 1
DENSW_PAPER, DENSW_ISOTROPIC = 0, 1  # density weights of Eq. (58): Eqs. (59)-(60) | isotropic
FLUX_MINMOD, FLUX_RUSANOV = 0, 1  # streaming flux: Eqs. (47)-(53) | first-order Rusanov (1D)


@dataclass
class Workload:
    name: str
    nx: int
    ny: int
    nz: int
    steps: int
    precision: int = FP64
    collision: int = COLL_IMPLICIT
    tau_mode: int = TAU_ETA_OVER_S
    tau: float = 1.0
    eta_over_s: float = 0.0
    alpha: float = 0.0
    with_density: bool = False
    nu: float = NU_DEFAULT
    dt: float = 0.25
    bc: List[int] = field(default_factory=lambda: [BC_PERIODIC] * 6)
    face_states: List[List[float]] = field(default_factory=lambda: [[3.0, 0.0, 0.0, 0.0, 1.0]] * 6)
    guard_umax: float = 0.0
    guard_efloor: float = 1e-10
    lattice: int = LATTICE_EXTENDED
    density_weights: int = DENSW_PAPER
    flux: int = FLUX_MINMOD
    eps: Optional[np.ndarray] = None
    ux: Optional[np.ndarray] = None
    uy: Optional[np.ndarray] = None
    uz: Optional[np.ndarray] = None
    n: Optional[np.ndarray] = None
    obstacle: Optional[np.ndarray] = None

    @property
    def shape(self):
        return (self.nz, self.ny, self.nx)

    @property
    def ncell(self) -> int:
        return self.nx * self.ny * self.nz

    def fields(self):
        return self.eps, self.ux, self.uy, self.uz, self.n

    def copy_with(self, **kw) -> "Workload":
        d = dict(self.__dict__)
        d.update(kw)
        return Workload(**d)


def _zeros(shape):
    return np.zeros(shape, dtype=np.float64)


def shock_tube_1d(nx=1000, steps=500, T_left=2.0, T_right=1.0, eta_over_s=0.1,
                  alpha=0.0, with_density=False, precision=FP64, collision=COLL_IMPLICIT,
                  dt=0.25, nu=NU_DEFAULT, bc_ends=BC_FIXED) -> Workload:
    """Workload 1: quasi-1D viscous shock tube, left half T=2, right half T=1
    (energy ratio 16), fluid at rest, fixed-state ends, periodic transverse."""
    x = np.arange(nx)
    T = np.where(x < nx // 2, T_left, T_right)
    eps = 3.0 * T ** 4
    n = T ** 3
    shape = (1, 1, nx)
    w = Workload("shock_tube_1d", nx, 1, 1, steps, precision=precision, collision=collision,
                 tau_mode=TAU_ETA_OVER_S, eta_over_s=eta_over_s, alpha=alpha,
                 with_density=with_density, nu=nu, dt=dt,
                 bc=[bc_ends, bc_ends] + [BC_PERIODIC] * 4,
                 face_states=[[3.0 * T_left ** 4, 0, 0, 0, T_left ** 3],
                              [3.0 * T_right ** 4, 0, 0, 0, T_right ** 3]] + [[3.0, 0, 0, 0, 1.0]] * 4)
    w.eps = eps.reshape(shape)
    w.ux, w.uy, w.uz = _zeros(shape), _zeros(shape), _zeros(shape)
    w.n = n.reshape(shape)
    return w


def colliding_slabs_1d(nx=8192, steps=4000, gamma=10.0, eta_over_s=0.05, zeta_over_eta=0.5,
                       precision=FP64, seed=SEED_BASE + 2, nu=NU_DEFAULT, dt=0.25,
                       guard_umax=0.9999) -> Workload:
    """Workload 2: two slabs with opposite velocities at Lorentz factor gamma,
    eps = 3, n = 1 (1 + 0.01 U(-1,1)) per cell, inflow (fixed-state) ends.
    The bulk constant alpha follows from zeta/eta through the paper's
    eta_b = 4 p alpha nu^6 / 27 with eta = (eta/s) s, s = 4n at the ambient
    state (T = n = p = 1)."""
    rng = np.random.default_rng(seed)
    beta = math.sqrt(1.0 - 1.0 / gamma ** 2)
    x = np.arange(nx)
    ux = np.where(x < nx // 2, beta, -beta)
    n = 1.0 + 0.01 * rng.uniform(-1.0, 1.0, nx)
    eta = eta_over_s * 4.0
    alpha = zeta_over_eta * eta * 27.0 / (4.0 * 1.0 * nu ** 6)
    shape = (1, 1, nx)
    w = Workload("colliding_slabs_1d", nx, 1, 1, steps, precision=precision,
                 tau_mode=TAU_ETA_OVER_S, eta_over_s=eta_over_s, alpha=alpha,
                 with_density=True, nu=nu, dt=dt,
                 bc=[BC_FIXED, BC_FIXED] + [BC_PERIODIC] * 4,
                 face_states=[[3.0, beta, 0, 0, 1.0], [3.0, -beta, 0, 0, 1.0]] + [[3.0, 0, 0, 0, 1.0]] * 4,
                 guard_umax=guard_umax)
    w.eps = np.full(shape, 3.0)
    w.ux = ux.reshape(shape).astype(np.float64)
    w.uy, w.uz = _zeros(shape), _zeros(shape)
    w.n = n.reshape(shape)
    return w


def planar_shock_state(gamma_s: float, p_a=1.0, n_a=1.0):
    """State behind a planar shock moving into fluid at rest with eps = 3p:
    post-shock speed u with gamma_s, pressure from the jump condition
    u^2 (3 p_a + p)(3 p + p_a) = 3 (p - p_a)^2, front speed from energy
    conservation and density from the particle-flux condition."""
    u = math.sqrt(1.0 - 1.0 / gamma_s ** 2)
    a = 3.0 - 3.0 * u * u
    b = -(6.0 * p_a + 10.0 * u * u * p_a)
    c = (3.0 - 3.0 * u * u) * p_a * p_a
    p = (-b + math.sqrt(b * b - 4 * a * c)) / (2 * a)
    g2 = gamma_s ** 2
    T00b, T0xb = 4 * p * g2 - p, 4 * p * g2 * u
    Vs = T0xb / (T00b - 3.0 * p_a)
    n = n_a * Vs / (gamma_s * (Vs - u))
    return p, u, Vs, n


def shock_cloud_2d(nx=2048, ny=1024, steps=20000, gamma_s=3.0, cloud_radius=96.0,
                   shock_x=256, cloud_center=(768.0, 512.0), eta_over_s=0.01, alpha=0.2,
                   precision=MIXED, seed=SEED_BASE + 3, nu=NU_DEFAULT, dt=0.15,
                   guard_umax=0.999) -> Workload:
    """Workload 3: planar shock (post-shock gamma = 3) moving towards a
    circular cloud of radius 96 cells whose edge carries seeded Fourier modes
    1..16 of amplitude 2%.  The cloud is an obstacle held at the equilibrium
    of (eps_a, 10 n_a, u = 0) (the paper's shock-cloud mechanism, Sec. III).
    Left face: fixed inflow of the shocked state; other faces: outflow.
    Geometry scales with (nx, ny) relative to 2048 x 1024.  The
    admissibility guard is on by default: without it the scheme as read
    leaves the admissible set at the shock front within a few steps."""
    rng = np.random.default_rng(seed)
    sx, sy = nx / 2048.0, ny / 1024.0
    p_s, u_s, _, n_s = planar_shock_state(gamma_s)
    shape = (1, ny, nx)
    X, Y = np.meshgrid(np.arange(nx) + 0.5, np.arange(ny) + 0.5)
    eps = np.where(X < shock_x * sx, 3.0 * p_s, 3.0)
    ux = np.where(X < shock_x * sx, u_s, 0.0)
    n = np.where(X < shock_x * sx, n_s, 1.0)
    am = rng.uniform(-1, 1, 16)
    bm = rng.uniform(-1, 1, 16)
    cx, cy = cloud_center[0] * sx, cloud_center[1] * sy
    theta = np.arctan2(Y - cy, X - cx)
    m = np.arange(1, 17)
    rho = (am[None, None, :] * np.cos(m * theta[..., None]) +
           bm[None, None, :] * np.sin(m * theta[..., None])).sum(-1)
    tt = np.linspace(-math.pi, math.pi, 4097)
    rho_max = np.abs((am[None, :] * np.cos(m * tt[:, None]) + bm[None, :] * np.sin(m * tt[:, None])).sum(-1)).max()
    R = cloud_radius * min(sx, sy) * (1.0 + 0.02 * rho / rho_max)
    cloud = np.hypot(X - cx, Y - cy) < R
    eps = np.where(cloud, 3.0, eps)
    n = np.where(cloud, 10.0, n)
    ux = np.where(cloud, 0.0, ux)
    w = Workload("shock_cloud_2d", nx, ny, 1, steps, precision=precision,
                 tau_mode=TAU_ETA_OVER_S, eta_over_s=eta_over_s, alpha=alpha,
                 with_density=True, nu=nu, dt=dt,
                 bc=[BC_FIXED, BC_OUTFLOW, BC_OUTFLOW, BC_OUTFLOW, BC_PERIODIC, BC_PERIODIC],
                 face_states=[[3.0 * p_s, u_s, 0, 0, n_s]] + [[3.0, 0, 0, 0, 1.0]] * 5,
                 guard_umax=guard_umax)
    w.eps = eps.reshape(shape)
    w.ux = ux.reshape(shape)
    w.uy, w.uz = _zeros(shape), _zeros(shape)
    w.n = n.reshape(shape)
    w.obstacle = cloud.reshape(shape).astype(np.uint8)
    return w


def blast_wave_3d(n=384, steps=2000, radius=32.0, energy_ratio=1e3, eta_over_s=0.02,
                  alpha=0.2, precision=MIXED, seed=SEED_BASE + 5, nu=NU_DEFAULT,
                  dt=0.15, guard_umax=0.999, nz=None) -> Workload:
    """Workload 5: periodic cube with an overpressure sphere of radius 32
    cells (energy ratio 1e3) at the centre of a medium with seeded 1%
    log-normal density fluctuations n = exp(0.01 g - 0.5e-4), g ~ N(0,1).
    The radius scales with n / 384.  The admissibility guard is on by
    default (the density distribution turns inadmissible at the blast front
    within a few tens of steps without it).  nz (default n) makes the box
    n x n x nz with the sphere at its centre."""
    nz = n if nz is None else nz
    rng = np.random.default_rng(seed)
    shape = (nz, n, n)
    g = rng.standard_normal(shape, dtype=np.float64)
    dens = np.exp(0.01 * g - 0.5e-4)
    del g
    r = radius * n / 384.0
    ax = np.arange(n) + 0.5 - n / 2.0
    az = np.arange(nz) + 0.5 - nz / 2.0
    d2 = az[:, None, None] ** 2 + ax[None, :, None] ** 2 + ax[None, None, :] ** 2
    eps = np.where(d2 < r * r, 3.0 * energy_ratio, 3.0)
    del d2
    w = Workload("blast_wave_3d", n, n, nz, steps, precision=precision,
                 tau_mode=TAU_ETA_OVER_S, eta_over_s=eta_over_s, alpha=alpha,
                 with_density=True, nu=nu, dt=dt, bc=[BC_PERIODIC] * 6,
                 guard_umax=guard_umax)
    w.eps = eps
    w.ux, w.uy, w.uz = _zeros(shape), _zeros(shape), _zeros(shape)
    w.n = dens
    return w


def shock_cloud_3d(nx=200, ny=100, nz=100, regime="weak", viscous=False, steps=None,
                   precision=MIXED, nu=NU_DEFAULT, alpha=0.2, dt=0.15, tau=1.0,
                   guard_umax=0.999) -> Workload:
    """The paper's 3D astrophysical application (Sec. III): a Riemann
    discontinuity at the plane x = 65 of a 200 x 100 x 100 lattice drives a
    shock into a solid spherical cloud of radius 10 centred at (100, 50, 50).
    Driver state (n0, T0) on the inlet side x <= 65 (the reading also taken
    for the 2D cloud), ambient (n1, T1) = (1, 1) beyond; p = n T, eps = 3 p.
    The cloud is an obstacle held at the equilibrium of (n1, T1, u = 0); the
    x = 0 face is an inlet fixed to the driver equilibrium, the other faces
    are open (outflow).  regime 'weak': T0 = 2.71 T1, n0 = 0.9 n1 (the
    paper's beta ~ 0.2); 'strong': T0 = 54.77 T1, n0 = 10.95 n1 (beta ~ 0.9).
    Inviscid: Euler mode, alpha = 0.2, dt/dx = 0.15, 1000 steps; viscous:
    uniform tau = 1, 600 steps.  Geometry scales with (nx, ny, nz)."""
    T0, n0 = (2.71, 0.9) if regime == "weak" else (54.77, 10.95)
    e0 = 3.0 * n0 * T0
    sx, sy, sz = nx / 200.0, ny / 100.0, nz / 100.0
    shape = (nz, ny, nx)
    Z, Y, X = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    drive = X <= 65.0 * sx
    r = 10.0 * min(sx, sy, sz)
    cloud = (X - 100.0 * sx) ** 2 + (Y - 50.0 * sy) ** 2 + (Z - 50.0 * sz) ** 2 <= r * r
    eps = np.where(drive & ~cloud, e0, 3.0)
    n = np.where(drive & ~cloud, n0, 1.0)
    if steps is None:
        steps = 600 if viscous else 1000
    name = f"shock_cloud_3d_{regime}" + ("_viscous" if viscous else "")
    w = Workload(name, nx, ny, nz, steps, precision=precision,
                 collision=COLL_IMPLICIT if viscous else COLL_EULER,
                 tau_mode=TAU_UNIFORM, tau=tau, alpha=alpha, with_density=True, nu=nu, dt=dt,
                 bc=[BC_FIXED] + [BC_OUTFLOW] * 5,
                 face_states=[[e0, 0.0, 0.0, 0.0, n0]] + [[3.0, 0.0, 0.0, 0.0, 1.0]] * 5,
                 guard_umax=guard_umax)
    w.eps = eps.astype(np.float64)
    w.ux, w.uy, w.uz = _zeros(shape), _zeros(shape), _zeros(shape)
    w.n = n.astype(np.float64)
    w.obstacle = cloud.astype(np.uint8)
    return w


def as_basic(w: Workload, nu=1.0) -> Workload:
    """The same initial and boundary set-up for the basic model of Sec. II:
    standard D3Q19, exact streaming, explicit Marle collision, energy-momentum
    distribution only (no density, no bulk term, no guard; Euler mode does not
    exist for it, so an inviscid recipe keeps its own relaxation time).
    nu = 1 by default: the explicit collision needs omega = nu^2/(sqrt(19)
    tau) < 2, which at nu = 27^(1/4) fails for tau below 0.6 (eta/s = 0.01)."""
    b = w.copy_with(name=w.name + "_basic", lattice=LATTICE_BASIC, nu=nu, collision=COLL_IMPLICIT,
                    alpha=0.0, with_density=False, guard_umax=0.0)
    b.n = None
    return b


def basic_vs_extended_tube(lattice=LATTICE_BASIC, nx=1000, ratio=32.0, eta_over_s=0.01,
                           precision=FP64) -> Workload:
    """The paper's comparison of the two models (Sec. III): a 1D tube with
    pressure ratio 32 (2.495e-7 / 7.785e-9 in its numerical units; the exact
    plateau moves at beta = 0.64), at rest, eta/s = 0.01, fixed-state ends.
    Basic model: nu = 1, 300 steps of dt = sqrt(27/19); extended model:
    nu = 27^(1/4), dt/dx = 0.25, alpha = 0.15, 1400 steps (the same time)."""
    x = np.arange(nx)
    shape = (1, 1, nx)
    eps = np.where(x < nx // 2, 3.0 * ratio, 3.0).astype(np.float64).reshape(shape)
    basic = lattice == LATTICE_BASIC
    w = Workload("basic_vs_extended_tube" + ("_basic" if basic else "_extended"), nx, 1, 1,
                 300 if basic else 1400, precision=precision, tau_mode=TAU_ETA_OVER_S,
                 eta_over_s=eta_over_s, alpha=0.0 if basic else 0.15, nu=1.0 if basic else NU_DEFAULT,
                 dt=0.25, bc=[BC_FIXED, BC_FIXED] + [BC_PERIODIC] * 4,
                 face_states=[[3.0 * ratio, 0.0, 0.0, 0.0, 1.0], [3.0, 0.0, 0.0, 0.0, 1.0]]
                 + [[3.0, 0.0, 0.0, 0.0, 1.0]] * 4, lattice=lattice)
    w.eps = eps
    w.ux, w.uy, w.uz = _zeros(shape), _zeros(shape), _zeros(shape)
    return w


def uniform_state(nx, ny, nz, eps=3.0, u=(0.0, 0.0, 0.0), n=1.0, **kw) -> Workload:
    """A uniform state (a fixed point of the update under periodic boundaries)."""
    shape = (nz, ny, nx)
    w = Workload("uniform", nx, ny, nz, kw.pop("steps", 10), **kw)
    w.eps = np.full(shape, float(eps))
    w.ux, w.uy, w.uz = (np.full(shape, float(v)) for v in u)
    w.n = np.full(shape, float(n))
    return w


def random_smooth_state(nx, ny, nz, seed, amp_eps=0.3, umax=0.3, **kw) -> Workload:
    """Seeded smooth random fields (a few Fourier modes) for parity tests."""
    rng = np.random.default_rng(seed)
    shape = (nz, ny, nx)
    Z, Y, X = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")

    def field_():
        s = np.zeros(shape)
        for _ in range(4):
            kx, ky, kz = rng.integers(0, 3, 3)
            ph = rng.uniform(0, 2 * math.pi)
            s += rng.uniform(-1, 1) * np.cos(2 * math.pi * (kx * X / nx + ky * Y / ny + kz * Z / nz) + ph)
        return s / 4.0

    w = Workload("random_smooth", nx, ny, nz, kw.pop("steps", 10), **kw)
    w.eps = 3.0 * np.exp(amp_eps * field_())
    w.ux = umax * field_()
    w.uy = umax * field_() if ny > 1 else np.zeros(shape)
    w.uz = umax * field_() if nz > 1 else np.zeros(shape)
    w.n = np.exp(0.2 * field_())
    return w


@dataclass
class ServingRequest:
    """One independent 1D solve of the serving workload."""
    n: int
    steps: int
    eps: np.ndarray
    ux: np.ndarray
    uy: np.ndarray
    uz: np.ndarray
    dens: np.ndarray
    eta_over_s: float
    alpha: float
    bc_lo: int
    bc_hi: int
    face_lo: List[float]
    face_hi: List[float]
    tau: float = 1.0
    arrival: float = 0.0  # seconds after the start of the stream

    def workload(self, precision=MIXED, guard_umax=0.9999, dt=0.25, nu=NU_DEFAULT) -> Workload:
        """The same solve as a stand-alone Workload (for the oracle and the
        one-at-a-time path)."""
        shape = (1, 1, self.n)
        w = Workload("serving_request", self.n, 1, 1, self.steps, precision=precision,
                     tau_mode=TAU_ETA_OVER_S, eta_over_s=self.eta_over_s, alpha=self.alpha,
                     with_density=True, nu=nu, dt=dt,
                     bc=[self.bc_lo, self.bc_hi] + [BC_PERIODIC] * 4,
                     face_states=[list(self.face_lo), list(self.face_hi)] + [[3.0, 0, 0, 0, 1.0]] * 4,
                     guard_umax=guard_umax)
        w.eps, w.ux, w.uy, w.uz, w.n = (a.reshape(shape).copy() for a in
                                         (self.eps, self.ux, self.uy, self.uz, self.dens))
        return w


def serving_requests(count=512, nmin=512, nmax=65536, seed=SEED_BASE + 4, steps_factor=2,
                     ratio_range=(1.5, 20.0), gamma_range=(1.0, 10.0), eta_range=(1e-3, 0.2),
                     alpha=0.2, rate=None) -> List[ServingRequest]:
    """Workload 4: independent boosted shock tubes.  Grid sizes log-uniform in
    [nmin, nmax], temperature ratios log-uniform in ratio_range (eps ratio =
    ratio^4), a boost with gamma uniform in gamma_range applied to both halves,
    eta/s log-uniform in eta_range, steps = steps_factor * n, fixed-state ends
    holding the initial end states.  With `rate` (requests per second) the
    arrival times follow a Poisson process."""
    rng = np.random.default_rng(seed)
    out = []
    t = 0.0
    for _ in range(count):
        n = int(round(math.exp(rng.uniform(math.log(nmin), math.log(nmax)))))
        ratio = math.exp(rng.uniform(math.log(ratio_range[0]), math.log(ratio_range[1])))
        g0 = rng.uniform(*gamma_range)
        eos = math.exp(rng.uniform(math.log(eta_range[0]), math.log(eta_range[1])))
        u0 = math.sqrt(1.0 - 1.0 / (g0 * g0))
        x = np.arange(n)
        T = np.where(x < n // 2, ratio, 1.0)
        eps = 3.0 * T ** 4
        dens = T ** 3
        ux = np.full(n, u0)
        z = np.zeros(n)
        if rate:
            t += rng.exponential(1.0 / rate)
        out.append(ServingRequest(n=n, steps=int(round(steps_factor * n)), eps=eps, ux=ux, uy=z, uz=z.copy(),
                                  dens=dens, eta_over_s=eos, alpha=alpha, bc_lo=BC_FIXED,
                                  bc_hi=BC_FIXED, face_lo=[3.0 * ratio ** 4, u0, 0.0, 0.0, ratio ** 3],
                                  face_hi=[3.0, u0, 0.0, 0.0, 1.0], arrival=t))
    return out


def workload(k: int, **kw) -> Workload:
    """Workload k (1, 2, 3 or 5) at its full size unless overridden."""
    if k == 1:
        return shock_tube_1d(**kw)
    if k == 2:
        return colliding_slabs_1d(**kw)
    if k == 3:
        return shock_cloud_2d(**kw)
    if k == 5:
        return blast_wave_3d(**kw)
    raise ValueError(f"no grid workload {k}")


# A parameter set under which uniform flows are (nearly) linearly stable at
# high speed (von Neumann analysis of the scheme, relaxation times 0.54 - 1.3):
# flows along a lattice axis are stable up to |u| = 0.95 and grow by at most
# 5e-4 per step at u = 0.995; oblique flows grow by at most 5e-4 per step at
# |u| = 0.9 and 1.2e-3 at 0.95; the density part is stable up to |u| = 0.995.
# nu = 4 keeps the density part stable, and the bulk term at
# kappa = (nu^2 / sqrt 27) alpha dt = 0.023 damps the short waves of the
# energy-momentum part without the over-damping that a larger kappa causes
# in 2D and 3D.  The bulk term acts here as a numerical stabiliser:
# alpha = 0.1 at nu = 4 is a bulk viscosity eta_b = 4 p alpha nu^6 / 27 ~ 61 p.
STABILISED = dict(nu=4.0, alpha=0.1, dt=0.075)


def stabilised(w: Workload) -> Workload:
    """The same recipe and physical run time under the STABILISED parameters
    (nu, alpha and dt replaced; the step count scaled by the old dt / new dt;
    eta/s and tau unchanged)."""
    steps = int(round(w.steps * w.dt / STABILISED["dt"]))
    return w.copy_with(steps=steps, **STABILISED)

