"""CPU pins of the oracle's basic model (Sec. II): the standard D3Q19 set with
c_a = sqrt(19)/nu, exact streaming with dt = c_t dx/(c_a c_0) and the
explicit Marle collision, no bulk term, no limiter, energy-momentum
distribution f only (the paper introduces the density distribution with the
extended set).

Pinned by: closed-form weights; lattice moments equal to the extended set's
(the two sets share every moment up to fourth order); the moment condition
Eq. (36) of the shared equilibrium; exact one-link streaming along +e_i; the relaxation rate
omega = nu^2 / (sqrt(19) tau) of a moment-free perturbation; conservation;
the exact Riemann solution of a weak tube; and the paper's comparison of
Sec. III: at beta ~ 0.64 the basic model overshoots the exact plateau with a
non-monotone profile while the extended model does not.
"""
import math

import numpy as np
import pytest

from oracle import oracle as O
from oracle import riemann as R

NUS = [1.0, 27.0 ** 0.25, 3.0]
ETA = np.diag([1.0, -1.0, -1.0, -1.0])


@pytest.mark.parametrize("nu", NUS)
def test_basic_weights_closed_form(nu):
    e, xi, w, wp = O.lattice(nu, basic=True)
    n2 = (e * e).sum(1)
    assert sorted(n2.tolist()) == [0] + [1] * 6 + [2] * 12
    assert np.abs(e).max() == 1
    np.testing.assert_allclose(w[n2 == 0], -44.0 / 361.0, rtol=1e-13)
    np.testing.assert_allclose(w[n2 == 1], 99.0 / 722.0, rtol=1e-13)
    np.testing.assert_allclose(w[n2 == 2], 9.0 / 361.0, rtol=1e-13)
    np.testing.assert_allclose(xi[:, 0], math.sqrt(27.0) / nu, rtol=1e-14)
    np.testing.assert_allclose(xi[:, 1:], math.sqrt(19.0) / nu * e, rtol=1e-14)


@pytest.mark.parametrize("nu", NUS)
def test_basic_moments_equal_extended(nu):
    for basic in (True, False):
        _, xi, w, _ = O.lattice(nu, basic=basic)
        m2 = np.einsum("i,ia,ib->ab", w, xi, xi)
        np.testing.assert_allclose(m2, np.diag([27.0, 9.0, 9.0, 9.0]) / nu ** 2, atol=1e-12)
        assert abs(w.sum() - 1.0) < 1e-14
        x = xi[:, 1:]
        assert abs((w * x[:, 0] ** 4).sum() - 171.0 / nu ** 4) < 1e-11
        assert abs((w * x[:, 0] ** 2 * x[:, 1] ** 2).sum() - 36.0 / nu ** 4) < 1e-11
        # odd moments vanish
        assert np.abs(np.einsum("i,ia->a", w, x)).max() < 1e-14
        assert np.abs(np.einsum("i,ia,ib,ic->abc", w, x, x, x)).max() < 1e-12


@pytest.mark.parametrize("nu", NUS)
def test_basic_equilibrium_moment_condition(nu):
    rng = np.random.default_rng(11)
    _, xi, _, _ = O.lattice(nu, basic=True)
    worst = 0.0
    for _ in range(200):
        eps = rng.uniform(0.1, 10.0)
        u = rng.uniform(-1, 1, 3)
        u *= rng.uniform(0, 0.95) / np.linalg.norm(u)
        f = O.feq(nu, eps, *u, basic=True)
        g = 1.0 / math.sqrt(1.0 - u @ u)
        U = np.r_[g, g * u]
        T = (eps + eps / 3.0) * np.outer(U, U) - eps / 3.0 * ETA
        Td = np.einsum("i,ia,ib->ab", f, xi, xi)
        worst = max(worst, np.abs(Td - T).max() / np.abs(T).max())
    assert worst < 1e-13


def _periodic_basic(shape, tau=1.0, nu=1.0, **kw):
    nz, ny, nx = shape
    return O.Config(nx=nx, ny=ny, nz=nz, nu=nu, dt=0.0, tau_mode=O.TAU_UNIFORM, tau=tau,
                    bc=[O.BC_PERIODIC] * 6, basic=True, **kw)


def _smooth_state(shape, seed, a=1.0):
    rng = np.random.default_rng(seed)
    nz, ny, nx = shape
    Z, Y, X = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    ph = rng.uniform(0, 2 * np.pi, 6)
    eps = 3.0 * (1.0 + 0.3 * a * np.sin(2 * np.pi * X / nx + ph[0]) * np.cos(2 * np.pi * Y / ny + ph[1]))
    ux = 0.2 * a * np.sin(2 * np.pi * Z / nz + ph[2])
    uy = 0.15 * a * np.cos(2 * np.pi * X / nx + ph[3])
    uz = 0.1 * a * np.sin(2 * np.pi * Y / ny + ph[4])
    return eps, ux, uy, uz


def test_basic_streams_one_link_along_e():
    """From an equilibrium state the collision is the identity, so one step
    moves every population exactly one link along +e_i."""
    shape = (3, 4, 5)
    o = O.Oracle(_periodic_basic(shape))
    st = _smooth_state(shape, 1)
    o.init(*st)
    f0, _ = o.pops()
    assert o.step(1) == 0
    f1, _ = o.pops()
    e, _, _, _ = O.lattice(1.0, basic=True)
    for i in range(O.Q):
        src = np.roll(f0[i].reshape(shape), shift=(e[i][2], e[i][1], e[i][0]), axis=(0, 1, 2))
        np.testing.assert_allclose(f1[i].reshape(shape), src, rtol=1e-13, atol=1e-15)


@pytest.mark.parametrize("nu,tau", [(1.0, 0.7), (27.0 ** 0.25, 1.3)])
def test_basic_relaxation_rate(nu, tau):
    """A spatially uniform state f = f^eq + d with a moment-free d relaxes as
    d -> (1 - omega) d per step, omega = c_0 nu dt / (c_t tau) with
    dt = c_t / (c_a c_0): omega = nu^2 / (sqrt(19) tau)."""
    shape = (2, 2, 3)
    o = O.Oracle(_periodic_basic(shape, tau=tau, nu=nu))
    eps, u = 3.3, np.array([0.2, -0.1, 0.05])
    o.init(*(np.full(shape, v) for v in (eps, *u)))
    _, xi, _, _ = O.lattice(nu, basic=True)
    M = xi[:, 0:1] * xi  # rows xi^0 xi^mu: the conserved moments
    d = np.random.default_rng(2).normal(size=O.Q)
    d -= M @ np.linalg.lstsq(M, d, rcond=None)[0]
    d *= 1e-3
    fe = O.feq(nu, eps, *u, basic=True)
    ncell = int(np.prod(shape))
    o.set_pops(np.repeat((fe + d)[:, None], ncell, axis=1))
    assert o.step(1) == 0
    f1, _ = o.pops()
    omega = nu * nu / (math.sqrt(19.0) * tau)
    np.testing.assert_allclose(f1[:, 0] - fe, (1.0 - omega) * d, rtol=1e-9, atol=1e-15)


def test_basic_conserves_on_periodic_grid():
    shape = (5, 6, 7)
    o = O.Oracle(_periodic_basic(shape, tau=0.9))
    o.init(*_smooth_state(shape, 4))
    _, xi, _, _ = O.lattice(1.0, basic=True)

    def sums():
        f, _ = o.pops()
        return np.einsum("ia,ic->a", xi[:, 0:1] * xi, f)

    s0 = sums()
    assert o.step(12) == 0
    np.testing.assert_allclose(sums(), s0, rtol=1e-12, atol=1e-10)


def _tube(basic, ratio, steps, nu=1.0, nx=1000):
    x = np.arange(nx)
    eps = np.where(x < nx // 2, 3.0 * ratio, 3.0)
    z = np.zeros(nx)
    cfg = O.Config(nx=nx, nu=nu, dt=0.0 if basic else 0.25, tau_mode=O.TAU_ETA_OVER_S,
                   eta_over_s=0.01, alpha=0.0 if basic else 0.15, bc=[O.BC_FIXED] * 2 + [O.BC_PERIODIC] * 4,
                   face=[[3.0 * ratio, 0, 0, 0, 1.0], [3.0, 0, 0, 0, 1.0]] + [[3.0, 0, 0, 0, 1.0]] * 4,
                   basic=basic)
    o = O.Oracle(cfg)
    o.init(eps, z, z, z)
    assert o.step(steps) == 0
    return [a.ravel() for a in o.fields()[:4]]


def test_basic_weak_tube_matches_exact_riemann():
    """Pressure ratio 4 (beta ~ 0.29): plateau within 1% of the exact solution."""
    ratio, steps, nx = 4.0, 300, 1000
    eps, ux, _, _ = _tube(True, ratio, steps, nx=nx)
    s = R.solve(ratio, 0.0, 1.0, 0.0)
    t = steps * math.sqrt(27.0 / 19.0)  # dt = sqrt(27/19) dx
    # cells well inside the plateau (between the rarefaction tail and the shock)
    xs = (np.arange(nx) + 0.5 - nx // 2) / t
    mid = (xs > s.left_tail + 0.05) & (xs < s.right_head - 0.05)
    assert mid.sum() > 50
    assert abs(np.median(ux[mid]) / s.vstar - 1.0) < 0.01
    assert abs(np.median(eps[mid]) / 3.0 / s.pstar - 1.0) < 0.01


def test_basic_model_fails_at_high_velocity_extended_does_not():
    """Sec. III comparison: pressure ratio 32 (plateau beta = 0.64), eta/s =
    0.01, the same physical time (300 basic steps of dt = sqrt(27/19), 1400
    extended steps of dt = 0.25).  The basic model (nu = 1: with eta/s =
    0.01 its explicit collision needs omega = nu^2/(sqrt(19) tau) < 2)
    overshoots the exact plateau by 6% with a non-monotone velocity profile
    (the artificial discontinuity); the extended model (nu = 27^(1/4),
    dt/dx = 0.25, alpha = 0.15) stays within 1% and monotone."""
    ratio = 32.0
    vstar = R.solve(ratio, 0.0, 1.0, 0.0).vstar
    _, ub, _, _ = _tube(True, ratio, 300)
    _, ue, _, _ = _tube(False, ratio, 1400, nu=27.0 ** 0.25)
    tv = lambda u: np.abs(np.diff(u)).sum()
    # basic: overshoot and oscillation
    assert ub.max() > 1.03 * vstar
    assert tv(ub) > 1.04 * 2.0 * ub.max()
    # extended: no visible overshoot, monotone up and down (total variation 2 max u)
    assert abs(ue.max() / vstar - 1.0) < 0.015
    assert tv(ue) < 1.01 * 2.0 * ue.max()


def test_basic_config_rejects_extended_only_terms():
    base = dict(nx=8, basic=True, bc=[O.BC_PERIODIC] * 6)
    for bad in ({"euler": True}, {"alpha": 0.1}, {"guard_umax": 0.99}, {"with_h": True}):
        with pytest.raises(O.OracleError):
            O.Oracle(O.Config(**base, **bad))


def test_basic_obstacle_holds_state_and_edges_are_filled():
    """2D run with an obstacle, a fixed face and outflow faces: obstacle
    cells keep their equilibrium; diagonal links read filled edge ghosts
    (the oracle's unfilled ghosts are NaN), so the run stays finite."""
    shape = (1, 12, 16)
    st = _smooth_state(shape, 9)
    ob = np.zeros(shape, np.uint8)
    ob[0, 5:8, 6:9] = 1
    cfg = O.Config(nx=16, ny=12, nz=1, nu=1.0, dt=0.0, tau=0.8, basic=True,
                   bc=[O.BC_FIXED, O.BC_OUTFLOW, O.BC_OUTFLOW, O.BC_FIXED, O.BC_PERIODIC, O.BC_PERIODIC],
                   face=[[4.0, 0.1, 0, 0, 1.2], [3, 0, 0, 0, 1], [3, 0, 0, 0, 1], [2.5, 0, -0.1, 0, 0.9],
                         [3, 0, 0, 0, 1], [3, 0, 0, 0, 1]])
    o = O.Oracle(cfg)
    o.init(*st, obstacle=ob)
    assert o.step(20) == 0
    fl = o.fields()
    assert all(np.isfinite(a).all() for a in fl)
    m = ob.astype(bool)
    np.testing.assert_allclose(fl[0][m], st[0][m], rtol=1e-12)
    np.testing.assert_allclose(fl[1][m], st[1][m], atol=1e-13)
