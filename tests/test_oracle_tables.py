"""Pins of the oracle's lattice tables and equilibria (CPU only).

Independent evidence used here:
  * exact rationals of the extended weights, obtained by hand by substituting
    c_a = sqrt(13)/nu and c_t/c_0 = sqrt(27)/nu (Sec. II.A) into the weight
    formulas; they are nu-independent;
  * lattice moment identities (isotropy up to second order and the fourth
    moments 171/nu^4, 36/nu^4), derived by hand from the velocity set;
  * the energy-momentum moment condition (Sec. II, Eq. (36)) with eps = 3p
    (Eq. (38)) for random states, and N^mu = n U^mu for the density
    distribution (Sec. II.A, Eq. (58));
  * brute-force momentum-space quadrature of the continuum Maxwell-Juttner
    moments (Sec. II, Eqs. (18)-(20)) against modified Bessel functions.
"""
import math

import numpy as np
import pytest
from scipy import special

NUS = [1.0, 27.0 ** 0.25, 3.0]
ETA = np.diag([1.0, -1.0, -1.0, -1.0])


def test_velocity_set_is_extended_d3q19(oracle_mod):
    e, xi, w, wp = oracle_mod.lattice(27.0 ** 0.25)
    vecs = {tuple(v) for v in e}
    assert len(vecs) == 19
    n2 = (e ** 2).sum(1)
    assert sorted(n2.tolist()) == [0] + [1] * 6 + [8] * 12
    # diagonals are 2(+-1,+-1,0) and permutations
    for v in e[n2 == 8]:
        assert sorted(abs(v).tolist()) == [0, 2, 2]


@pytest.mark.parametrize("nu", NUS)
def test_weights_closed_form(oracle_mod, nu):
    e, xi, w, wp = oracle_mod.lattice(nu)
    n2 = (e ** 2).sum(1)
    np.testing.assert_allclose(w[n2 == 0], -539.0 / 676.0, rtol=1e-14)
    np.testing.assert_allclose(w[n2 == 1], 99.0 / 338.0, rtol=1e-14)
    np.testing.assert_allclose(w[n2 == 8], 9.0 / 2704.0, rtol=1e-14)
    assert abs(w.sum() - 1.0) < 1e-14
    ca2 = 13.0 / nu ** 2
    np.testing.assert_allclose(wp[n2 == 0], 0.1, rtol=1e-14)
    np.testing.assert_allclose(wp[n2 == 1], 6.0 / 35.0 - 1.0 / (42.0 * ca2), rtol=1e-14)
    assert abs(wp.sum() - 1.0) < 1e-14


@pytest.mark.parametrize("nu", NUS)
def test_lattice_moments(oracle_mod, nu):
    e, xi, w, wp = oracle_mod.lattice(nu)
    x = xi[:, 1:]
    np.testing.assert_allclose(np.einsum("i,ia,ib->ab", w, x, x), 9.0 / nu ** 2 * np.eye(3), atol=1e-13)
    np.testing.assert_allclose((w * xi[:, 0] ** 2).sum(), 27.0 / nu ** 2, rtol=1e-13)
    assert abs(np.einsum("i,ia->a", w, x)).max() < 1e-14
    m4 = np.einsum("i,ia,ib,ic,id->abcd", w, x, x, x, x)
    assert abs(m4[0, 0, 0, 0] - 171.0 / nu ** 4) < 1e-12
    assert abs(m4[0, 0, 1, 1] - 36.0 / nu ** 4) < 1e-12
    assert abs(m4[0, 0, 0, 1]) < 1e-13
    # density weights: sum w' c^a c^b = delta / 3 (Sec. II.A, Eqs. (59)-(60))
    np.testing.assert_allclose(np.einsum("i,ia,ib->ab", wp, x, x), np.eye(3) / 3.0, atol=1e-13)
    assert abs(np.einsum("i,ia,ib,ic->abc", wp, x, x, x)).max() < 1e-13


def test_c0_value_matches_first_order_coefficient():
    """The lattice constant c_0 = (3/8)(9 - 2 sqrt 3) of Sec. II.A is exactly
    the value for which gamma (sqrt27/2 - 1)/c_0 equals 4 gamma/sqrt27, the
    first-order coefficient required by the moment condition."""
    c0 = 3.0 / 8.0 * (9.0 - 2.0 * math.sqrt(3.0))
    assert abs((math.sqrt(27.0) / 2.0 - 1.0) / c0 - 4.0 / math.sqrt(27.0)) < 1e-15


def _rand_states(rng, k, umax=0.995):
    out = []
    for _ in range(k):
        d = rng.standard_normal(3)
        d /= np.linalg.norm(d)
        u = d * umax * rng.uniform(0, 1) ** 0.5
        out.append((float(np.exp(rng.uniform(np.log(0.1), np.log(10.0)))), u, float(rng.uniform(0.2, 5.0))))
    return out


@pytest.mark.parametrize("nu", NUS)
def test_equilibrium_moment_condition(oracle_mod, nu):
    """Sum_i xi^a xi^b f^eq_i = (eps+p) U^a U^b - p eta^{ab}, p = eps/3 (Eq. (36), Eq. (38))."""
    rng = np.random.default_rng(11)
    e, xi, w, wp = oracle_mod.lattice(nu)
    for eps, u, n in _rand_states(rng, 200):
        f = oracle_mod.feq(nu, eps, *u)
        g = 1.0 / math.sqrt(1.0 - u @ u)
        U = g * np.r_[1.0, u]
        T = np.einsum("ia,ib,i->ab", xi, xi, f)
        Tex = 4.0 / 3.0 * eps * np.outer(U, U) - eps / 3.0 * ETA
        assert abs(T - Tex).max() <= 1e-13 * abs(Tex).max()
        h = oracle_mod.heq(nu, n, *u)
        N = np.einsum("ia,i->a", xi, h)
        assert abs(N - n * U).max() <= 1e-13 * n * g


def test_printed_expansion_violates_moment_condition(oracle_mod):
    """Documented negative: the second-order expansion as printed (Eq. (29)),
    discretised with xi^0 = c_t/c_0 and chi^0 -> chi^0/c_0, does not satisfy
    Eq. (36); the oracle's reading does (previous test)."""
    nu = 27.0 ** 0.25
    e, xi, w, wp = oracle_mod.lattice(nu)
    c0 = 3.0 / 8.0 * (9.0 - 2.0 * math.sqrt(3.0))
    u = np.array([0.3, 0.0, 0.0])
    g = 1.0 / math.sqrt(1 - u @ u)
    chi = nu * g * u
    chi0 = nu * g / c0
    x0 = math.sqrt(27.0) / nu
    f = []
    for i in range(19):
        x = xi[i, 1:]
        first = (chi0 * x0 + 3) / 2 - chi0 / nu - x0 * nu / 4
        dia = (x ** 2 * chi ** 2).sum()
        off = x[0] * x[1] * chi[0] * chi[1] + x[0] * x[2] * chi[0] * chi[2] + x[1] * x[2] * chi[1] * chi[2]
        iso = ((1 - nu ** 2) / nu * x0 - (4 - 2 * nu ** 2) / nu ** 2) * (chi @ chi)
        f.append(w[i] * (1 + first * (x @ chi) + off + 4 / (nu ** 4 - 6 * nu ** 2 - 15) * (dia + iso)))
    f = np.array(f)
    T = np.einsum("ia,ib,i->ab", xi, xi, f)
    U = g * np.r_[1.0, u]
    shape = 4 * np.outer(U, U) - ETA
    ratio = T[[0, 0, 1, 2], [0, 1, 1, 2]] / shape[[0, 0, 1, 2], [0, 1, 1, 2]]
    assert ratio.max() / ratio.min() > 1.5


def _mj_quadrature(nu, u, n_r=96, n_mu=64, n_phi=48):
    """Brute-force integrals of 1, xi^a, xi^a xi^b times exp(-chi_mu xi^mu)
    over d^3 xi / xi^0 with xi^0 = sqrt(|xi|^2 + nu^2), chi = nu U."""
    g = 1.0 / math.sqrt(1.0 - u @ u)
    chi = nu * g * np.r_[1.0, u]
    r, wr = special.roots_genlaguerre(n_r, 2.0)  # int r^2 e^{-r} g(r)
    mu, wmu = np.polynomial.legendre.leggauss(n_mu)
    phi = np.linspace(0, 2 * math.pi, n_phi, endpoint=False)
    wphi = 2 * math.pi / n_phi
    # scale radius so the exponential decay is resolved: r = s * rho
    s = 1.0 / (nu * g * (1.0 - math.sqrt(u @ u)) + 1e-300)
    R, MU, PHI = np.meshgrid(r * s, mu, phi, indexing="ij")
    W = (wr * np.exp(r))[:, None, None] * s ** 3 * wmu[None, :, None] * wphi
    st = np.sqrt(1 - MU ** 2)
    X = np.stack([R * st * np.cos(PHI), R * st * np.sin(PHI), R * MU])
    X0 = np.sqrt(R ** 2 + nu ** 2)
    arg = chi[0] * X0 - (chi[1] * X[0] + chi[2] * X[1] + chi[3] * X[2])
    F = np.exp(-arg) / X0 * W
    XI = np.concatenate([X0[None], X])
    m0 = F.sum()
    m1 = (XI * F[None]).reshape(4, -1).sum(1)
    XF = (XI * F[None]).reshape(4, -1)
    m2 = XF @ XI.reshape(4, -1).T
    return m0, m1, m2, chi


@pytest.mark.parametrize("nu,u", [(1.0, (0.0, 0.0, 0.0)), (1.0, (0.3, -0.2, 0.1)),
                                  (2.0, (0.5, 0.0, 0.0)), (0.5, (0.0, 0.4, 0.3))])
def test_continuum_moments_match_bessel(nu, u):
    """Eqs. (18)-(20): 4 pi K_1(nu^2), 4 pi K_2(nu^2) chi^a,
    -4 pi (K_2 eta^{ab} - K_3 chi^a chi^b) (A = 1)."""
    u = np.array(u)
    m0, m1, m2, chi = _mj_quadrature(nu, u)
    z = nu * nu
    K1, K2, K3 = special.kv(1, z), special.kv(2, z), special.kv(3, z)
    assert abs(m0 - 4 * math.pi * K1) < 3e-5 * 4 * math.pi * K1
    np.testing.assert_allclose(m1, 4 * math.pi * K2 * chi, rtol=3e-5, atol=3e-6 * abs(m1).max())
    ex = -4 * math.pi * (K2 * ETA - K3 * np.outer(chi, chi))
    np.testing.assert_allclose(m2, ex, rtol=3e-5, atol=3e-6 * abs(ex).max())


def test_ultrarelativistic_limit_structure():
    """As nu -> 0 the continuum second moment tends to a multiple of
    4 U U - eta (eps = 3p), the tensor the lattice equilibrium must carry."""
    u = np.array([0.4, 0.2, 0.0])
    g = 1.0 / math.sqrt(1 - u @ u)
    U = g * np.r_[1.0, u]
    nu = 0.05
    _, _, m2, _ = _mj_quadrature(nu, u)
    shape = 4 * np.outer(U, U) - ETA
    c = m2[0, 0] / shape[0, 0]
    np.testing.assert_allclose(m2, c * shape, rtol=1e-4, atol=1e-5 * abs(m2).max())
