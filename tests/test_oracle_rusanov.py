"""Pins of the oracle's Rusanov flux (ORC_FLUX_RUSANOV; beyond the paper), CPU
only.

The option replaces the minmod-limited upwind flux of Eqs. (47)-(53) by the
first-order local Lax-Friedrichs (Rusanov) flux 1/2 p (f_L + f_R) - 1/2 s
(f_R - f_L) with one dissipation speed s = xi^0 (the speed of light) for every
population.  Since sum_i xi^0 xi^mu f_i = T^{0 mu} and, at the equilibrium,
sum_i xi^x xi^mu f_i = T^{x mu} (Eq. (36)), the moments of one Euler-mode step
are the Rusanov scheme of the ideal-fluid equations:
    T* = T - dt [1/2 (F(x+1) - F(x-1)) - 1/2 (T(x+1) - 2 T(x) + T(x-1))]
with F the flux T^{x mu} and dt in units of dx and c; likewise for N^mu.
That update is a convex combination of T(x) and T(x -+ 1) +- F(x -+ 1),
whose energy exceeds the momentum for every admissible state of the
ultra-relativistic fluid, so the Euler mode keeps admissible states
admissible.

Independent evidence:
  * one step against that formula, evaluated from the fields with the
    closed-form ideal-fluid tensor (not from the populations), for T^{0 mu}
    and N^0 -- a wrong dissipation speed moves it by 1e-3;
  * conservation of sum T^{0 mu} and sum N^0 on a periodic domain;
  * the gamma = 10 colliding slabs in the Euler mode stay admissible without
    the guard (the minmod flux leaves the admissible set in the first step)
    and reach the exact centre state of the ideal-fluid solution;
  * the checkerboard mode of a uniform flow at |u| = 0.995 follows the
    von Neumann matrix of the Rusanov step and decays;
  * the pressure-ratio-16 Riemann problem: plateaus of the exact solution.
"""
import math

import numpy as np
import pytest

from oracle import riemann as R
from paper_1302_1125_amd import workloads as W
from tests._helpers import oracle_for
from tests.test_oracle_step import _sums
from tests.test_oracle_stability import NU0, _checkerboard, _f_linear, _odd_even, _speeds, _stream_rusanov


def _ideal(eps, ux, uy, uz, n):
    """T^{0 mu}, the x flux T^{x mu}, N^0 and N^x of the ideal fluid (eps = 3p)."""
    g2 = 1.0 / (1.0 - (ux * ux + uy * uy + uz * uz))
    T = np.array([eps * (4.0 * g2 - 1.0) / 3.0] + [4.0 / 3.0 * eps * g2 * u for u in (ux, uy, uz)])
    F = np.array([T[1], 4.0 / 3.0 * eps * g2 * ux * ux + eps / 3.0,
                  4.0 / 3.0 * eps * g2 * ux * uy, 4.0 / 3.0 * eps * g2 * ux * uz])
    g = np.sqrt(g2)
    return T, F, n * g, n * g * ux


def _ideal_3d(eps, ux, uy, uz, n):
    """T^{0 mu}, the fluxes T^{a mu} (a = x, y, z), N^0 and N^a of the ideal fluid."""
    u = (ux, uy, uz)
    g2 = 1.0 / (1.0 - (ux * ux + uy * uy + uz * uz))
    T = np.array([eps * (4.0 * g2 - 1.0) / 3.0] + [4.0 / 3.0 * eps * g2 * v for v in u])
    F = [np.array([T[1 + a]] + [4.0 / 3.0 * eps * g2 * u[a] * u[b] + (eps / 3.0 if a == b else 0.0)
                                for b in range(3)]) for a in range(3)]
    g = np.sqrt(g2)
    return T, F, n * g, [n * g * v for v in u]


def _rusanov(U, G, dt, s=1.0):
    r = lambda a, k: np.roll(a, -k, axis=-1)
    return U - dt * (0.5 * (r(G, 1) - r(G, -1)) - 0.5 * s * (r(U, 1) - 2.0 * U + r(U, -1)))


def _lap(U, ax=-1):
    return np.roll(U, -1, axis=ax) - 2.0 * U + np.roll(U, 1, axis=ax)


@pytest.mark.parametrize("umax,alpha", [(0.3, 0.0), (0.8, 0.0), (0.8, 0.2)])
def test_euler_step_is_the_rusanov_scheme_of_the_fluid(umax, alpha):
    """With the bulk term (alpha > 0) the update adds kappa times the
    Laplacian of every T^{0 mu}, kappa = (nu^2 / sqrt 27) alpha dt: the rest
    population takes the term too under this flux (without it T^{00} would
    differ by kappa times the Laplacian of the rest population's energy)."""
    w = W.random_smooth_state(40, 1, 1, seed=11, with_density=True, alpha=alpha, tau_mode=W.TAU_UNIFORM,
                              tau=1.0, dt=0.25, umax=umax)
    w = w.copy_with(collision=W.COLL_EULER, flux=W.FLUX_RUSANOV)
    o = oracle_for(w)
    T, F, N0, Nx = _ideal(*[a.ravel() for a in w.fields()])
    assert o.step(1) == 0
    T1, _, N1, _ = _ideal(*[a.ravel() for a in o.fields()])
    scale = np.abs(T).max()
    kappa = w.nu ** 2 / math.sqrt(27.0) * alpha * w.dt
    assert np.abs(T1 - (_rusanov(T, F, w.dt) + kappa * _lap(T))).max() < 1e-13 * scale
    assert np.abs(N1 - _rusanov(N0, Nx, w.dt)).max() < 1e-13 * np.abs(N0).max()
    # the dissipation speed is the speed of light, not the axis speed sqrt(13/27)
    assert np.abs(T1 - _rusanov(T, F, w.dt, math.sqrt(13.0 / 27.0))).max() > 1e-4 * scale


def test_euler_step_is_the_rusanov_scheme_in_3d():
    """The same in 3D (periodic 7 x 6 x 5 grid, dt = 0.15, alpha = 0.2): the
    update sums the Rusanov differences of the three axes, each with the
    axis's flux, and the bulk term of each axis."""
    w = W.random_smooth_state(7, 6, 5, seed=13, with_density=True, alpha=0.2, tau_mode=W.TAU_UNIFORM,
                              tau=1.0, dt=0.15, umax=0.5)
    w = w.copy_with(collision=W.COLL_EULER, flux=W.FLUX_RUSANOV)
    o = oracle_for(w)
    T, F, N0, Nf = _ideal_3d(*w.fields())
    assert o.step(1) == 0
    T1, _, N1, _ = _ideal_3d(*o.fields())
    dt = w.dt
    Tp, Np = T.copy(), N0.copy()
    for a, ax in enumerate((3, 2, 1)):  # x, y, z are the last three array axes of [mu][z][y][x]
        r = lambda q, k, ax=ax: np.roll(q, -k, axis=ax)
        rn = lambda q, k, ax=ax: np.roll(q, -k, axis=ax - 1)
        Tp -= dt * (0.5 * (r(F[a], 1) - r(F[a], -1)) - 0.5 * (r(T, 1) - 2.0 * T + r(T, -1)))
        Tp += w.nu ** 2 / math.sqrt(27.0) * w.alpha * dt * (r(T, 1) - 2.0 * T + r(T, -1))
        Np -= dt * (0.5 * (rn(Nf[a], 1) - rn(Nf[a], -1)) - 0.5 * (rn(N0, 1) - 2.0 * N0 + rn(N0, -1)))
    assert np.abs(T1 - Tp).max() < 1e-13 * np.abs(T).max()
    assert np.abs(N1 - Np).max() < 1e-13 * np.abs(N0).max()


def test_strong_3d_shock_cloud_stays_admissible():
    """The paper's 3D shock-cloud in the strong regime (driver T0 = 54.77, Euler
    mode, dt = 0.15, so dt s = 0.45 summed over the axes) at 40 x 20 x 20, 200
    steps, guard off: admissible throughout with the Rusanov flux; the minmod
    flux leaves the admissible set at step 20 of the same run."""
    w = W.shock_cloud_3d(nx=40, ny=20, nz=20, regime="strong", precision=W.FP64, steps=200, guard_umax=0.0)
    assert oracle_for(w.copy_with(flux=W.FLUX_RUSANOV)).step(200) == 0
    assert 0 < oracle_for(w).step(200) <= 30


@pytest.mark.parametrize("euler", [True, False])
def test_conservation_periodic(euler):
    """Uniform relaxation time (with eta/s the equilibrium source of the
    implicit update varies from cell to cell and conserves only
    approximately, as with the minmod flux)."""
    w = W.random_smooth_state(64, 1, 1, seed=12, with_density=True, alpha=0.1,
                              tau_mode=W.TAU_UNIFORM, tau=0.8, dt=0.25)
    w = w.copy_with(collision=int(euler), flux=W.FLUX_RUSANOV)
    o = oracle_for(w)
    s0 = _sums(o, w.nu)
    assert o.step(20) == 0
    s1 = _sums(o, w.nu)
    assert np.abs(s1 - s0).max() < 1e-12 * np.abs(s0).max()


def test_gamma10_inviscid_slabs_stay_admissible():
    """2048 cells, 1000 steps, no guard: admissible throughout, centre energy
    density at the exact ideal-fluid value (measured 2e-5); the minmod flux
    leaves the admissible set in the first step of the same run."""
    w = W.colliding_slabs_1d(nx=2048, steps=1000, guard_umax=0.0)
    w = w.copy_with(collision=W.COLL_EULER, flux=W.FLUX_RUSANOV)
    o = oracle_for(w)
    assert o.step(1000) == 0
    assert o.guard_events == 0
    eps = o.fields()[0].ravel()
    s = R.solve(1.0, math.sqrt(0.99), 1.0, -math.sqrt(0.99))
    c = len(eps) // 2
    assert abs(np.median(eps[c - 10:c + 10]) / (3.0 * s.pstar) - 1.0) < 2e-4
    assert 0 < oracle_for(w.copy_with(flux=W.FLUX_MINMOD)).step(10) <= 2


def test_checkerboard_follows_the_rusanov_matrix():
    """The shortest wave on a uniform flow at u = 0.995 in the Euler mode: the
    oracle's populations follow J K S with the Rusanov streaming factors
    (every factor 1 - 2 dt = 1/2 for this wave) and decay by 1/2 per step;
    the minmod flux lets the same wave grow by e^0.09 per step."""
    from oracle import oracle as O
    u, dt, nx, amp = 0.995, 0.25, 16, 1e-5
    lin = _f_linear(O, NU0, u)
    K, J, dfe, _ = lin
    S = np.diag(_stream_rusanov(_speeds(O, NU0), dt, math.pi))
    G = (J @ K @ S).real
    cfg = O.Config(nx=nx, nu=NU0, dt=dt, euler=True, bc=[O.BC_PERIODIC] * 6, flux=O.FLUX_RUSANOV)
    z = np.zeros(nx)
    init = (3.0 + amp * _checkerboard((1, 1, nx)).ravel(), np.full(nx, u), z, z, None)
    worst, gain = _odd_even(O, cfg, init, dfe * amp, G, 5, "f")
    assert worst < 1e-6, worst
    assert abs(gain - 0.5 ** 5) < 1e-6


def test_riemann_plateaus():
    """Pressure ratio 16 with density, Euler mode, t = 250: u* within 0.2%,
    p* within 1%, the density plateaus within 3% (measured 0.06%, 0.4%, 1.1%,
    1.4%; the first-order flux smears the contact more than the minmod flux)."""
    nx, steps, ratio = 1600, 1000, 16.0
    w = W.shock_tube_1d(nx=nx, steps=steps, T_left=ratio ** 0.25, T_right=1.0, alpha=0.0,
                        collision=W.COLL_EULER, bc_ends=W.BC_OUTFLOW, with_density=True)
    w = w.copy_with(flux=W.FLUX_RUSANOV, tau_mode=W.TAU_UNIFORM, tau=1.0)
    o = oracle_for(w)
    assert o.step(steps) == 0
    eps, ux, _, _, n = [a.ravel() for a in o.fields()]
    s = R.solve(ratio, 0.0, 1.0, 0.0, nL=ratio ** 0.75, nR=1.0)
    t = steps * w.dt
    vs = s.vstar
    cell = lambda x: int(nx / 2 + t * x)
    a, b = s.left_tail + 0.2 * (vs - s.left_tail), vs - 0.2 * (vs - s.left_tail)
    c, d = vs + 0.2 * (s.right_head - vs), s.right_head - 0.2 * (s.right_head - vs)
    assert abs(np.median(ux[cell(a):cell(d)]) / vs - 1.0) < 2e-3
    assert abs(np.median(eps[cell(a):cell(d)]) / (3.0 * s.pstar) - 1.0) < 1e-2
    assert abs(np.median(n[cell(a):cell(b)]) / s.nstarL - 1.0) < 3e-2
    assert abs(np.median(n[cell(c):cell(d)]) / s.nstarR - 1.0) < 3e-2


def test_rusanov_needs_the_extended_set():
    from oracle import oracle as O
    with pytest.raises(O.OracleError):
        O.Oracle(O.Config(nx=8, basic=True, flux=O.FLUX_RUSANOV))
    with pytest.raises(O.OracleError):
        O.Oracle(O.Config(nx=8, flux=5))
