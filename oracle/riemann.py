"""Exact Riemann problem of a one-dimensional ideal fluid with the
ultra-relativistic equation of state eps = 3p (c_s = 1/sqrt(3)).

TEST INFRASTRUCTURE ONLY.  This is the analytic inviscid reference against
which the paper validates its extended model in Euler mode (Sec. III,
inviscid case; the solution itself is the textbook one the paper cites).
It is written independently of the lattice code and shares nothing with it.

Waves: a left-facing rarefaction keeps J+ = atanh(v) + (sqrt3/4) ln p
constant, a right-facing one J- = atanh(v) - (sqrt3/4) ln p; a shock between
states a and b has relative speed
    |v_b - v_a| / (1 - v_a v_b) = |p_b - p_a| sqrt(3 / ((3 p_a + p_b)(3 p_b + p_a)))
and moves with V_s = [T^{0x}] / [T^{00}].  Density follows p^{3/4} along
rarefactions and the particle-flux jump condition across shocks.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

CS = 1.0 / math.sqrt(3.0)


def _shock_w(p, pa):
    return abs(p - pa) * math.sqrt(3.0 / ((3.0 * pa + p) * (3.0 * p + pa)))


def _vstar_left(p, pL, vL):
    """Velocity behind the left-facing wave as a function of star pressure."""
    if p <= pL:  # rarefaction
        return math.tanh(math.atanh(vL) + math.sqrt(3.0) / 4.0 * math.log(pL / p))
    w = _shock_w(p, pL)
    return (vL - w) / (1.0 - vL * w)


def _vstar_right(p, pR, vR):
    if p <= pR:
        return math.tanh(math.atanh(vR) - math.sqrt(3.0) / 4.0 * math.log(pR / p))
    w = _shock_w(p, pR)
    return (vR + w) / (1.0 + vR * w)


def _T00(p, v):
    g2 = 1.0 / (1.0 - v * v)
    return 4.0 * p * g2 - p


def _T0x(p, v):
    g2 = 1.0 / (1.0 - v * v)
    return 4.0 * p * g2 * v


def shock_speed(pa, va, pb, vb):
    """V_s = [T^{0x}]/[T^{00}] (energy conservation across the front)."""
    return (_T0x(pb, vb) - _T0x(pa, va)) / (_T00(pb, vb) - _T00(pa, va))


@dataclass
class RiemannSolution:
    pL: float
    vL: float
    nL: float
    pR: float
    vR: float
    nR: float
    pstar: float
    vstar: float
    left_shock: bool
    right_shock: bool
    nstarL: float
    nstarR: float
    left_head: float   # x/t of the left wave's leading edge (or shock)
    left_tail: float
    right_head: float
    right_tail: float

    def sample(self, xi):
        """(p, v, n) at similarity coordinates xi = (x - x0)/t."""
        xi = np.asarray(xi, dtype=np.float64)
        p = np.empty_like(xi)
        v = np.empty_like(xi)
        n = np.empty_like(xi)
        for k, s in np.ndenumerate(xi):
            p[k], v[k], n[k] = self._at(float(s))
        return p, v, n

    def _at(self, s):
        if s <= self.left_head:
            return self.pL, self.vL, self.nL
        if s < self.left_tail:  # inside the left fan
            v = (s + CS) / (1.0 + s * CS)
            p = self.pL * math.exp(4.0 / math.sqrt(3.0) * (math.atanh(self.vL) - math.atanh(v)))
            return p, v, self.nL * (p / self.pL) ** 0.75
        if s < self.vstar:
            return self.pstar, self.vstar, self.nstarL
        if s < self.right_tail:
            return self.pstar, self.vstar, self.nstarR
        if s < self.right_head:  # inside the right fan
            v = (s - CS) / (1.0 - s * CS)
            p = self.pR * math.exp(4.0 / math.sqrt(3.0) * (math.atanh(v) - math.atanh(self.vR)))
            return p, v, self.nR * (p / self.pR) ** 0.75
        return self.pR, self.vR, self.nR


def _n_behind_shock(na, va, vb, Vs):
    """Particle flux through the front: n_a g_a (v_a - V_s) = n_b g_b (v_b - V_s)."""
    ga = 1.0 / math.sqrt(1.0 - va * va)
    gb = 1.0 / math.sqrt(1.0 - vb * vb)
    return na * ga * (va - Vs) / (gb * (vb - Vs))


def solve(pL, vL, pR, vR, nL=1.0, nR=1.0) -> RiemannSolution:
    """Star state by bisection on log p of v*_left(p) = v*_right(p)."""
    lo, hi = math.log(min(pL, pR)) - 40.0, math.log(max(pL, pR)) + 40.0

    def g(lp):
        p = math.exp(lp)
        return _vstar_left(p, pL, vL) - _vstar_right(p, pR, vR)

    for _ in range(400):
        mid = 0.5 * (lo + hi)
        if g(mid) > 0:
            lo = mid
        else:
            hi = mid
    ps = math.exp(0.5 * (lo + hi))
    vs = 0.5 * (_vstar_left(ps, pL, vL) + _vstar_right(ps, pR, vR))

    left_shock = ps > pL
    if left_shock:
        Vs = shock_speed(pL, vL, ps, vs)
        lh = lt = Vs
        nsl = _n_behind_shock(nL, vL, vs, Vs)
    else:
        lh = (vL - CS) / (1.0 - vL * CS)
        lt = (vs - CS) / (1.0 - vs * CS)
        nsl = nL * (ps / pL) ** 0.75
    right_shock = ps > pR
    if right_shock:
        Vs = shock_speed(pR, vR, ps, vs)
        rh = rt = Vs
        nsr = _n_behind_shock(nR, vR, vs, Vs)
    else:
        rh = (vR + CS) / (1.0 + vR * CS)
        rt = (vs + CS) / (1.0 + vs * CS)
        nsr = nR * (ps / pR) ** 0.75
    return RiemannSolution(pL, vL, nL, pR, vR, nR, ps, vs, left_shock, right_shock,
                           nsl, nsr, lh, lt, rh, rt)
