"""Pins of the analytic ideal-fluid Riemann solver used as the inviscid
reference (CPU only).  Evidence: Rankine-Hugoniot jump conditions checked
directly in the shock frame, the known product v_1 v_2 = c_s^2 = 1/3 of the
pre- and post-shock speeds for eps = 3p, Riemann-invariant constancy across
the fan, and the plateau/shock speeds printed in the paper (Sec. III)."""
import json
import math
import os

import numpy as np
import pytest

from oracle import riemann as R

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_riemann.json")


def _boost(v, V):
    return (v - V) / (1 - v * V)


@pytest.mark.parametrize("ratio", [2.4389, 16.0, 1000.0, 1e5])
def test_shock_jump_conditions(ratio):
    s = R.solve(ratio, 0.0, 1.0, 0.0)
    Vs = s.right_head
    v1 = _boost(0.0, Vs)       # pre-shock speed in the shock frame
    v2 = _boost(s.vstar, Vs)   # post-shock speed in the shock frame
    assert abs(v1 * v2 - 1.0 / 3.0) < 1e-10
    # energy and momentum fluxes through the front (shock frame), eps = 3p
    def flux(p, v):
        g2 = 1 / (1 - v * v)
        return 4 * p * g2 * v, 4 * p * g2 * v * v + p
    a = flux(1.0, v1)
    b = flux(s.pstar, v2)
    assert abs(a[0] - b[0]) < 1e-9 * abs(a[0])
    assert abs(a[1] - b[1]) < 1e-9 * abs(a[1])


@pytest.mark.parametrize("ratio", [2.4389, 16.0, 1000.0])
def test_rarefaction_invariant(ratio):
    s = R.solve(ratio, 0.0, 1.0, 0.0)
    xi = np.linspace(s.left_head, s.left_tail, 50)
    p, v, _ = s.sample(xi)
    J = np.arctanh(v) + math.sqrt(3) / 4 * np.log(p)
    assert np.ptp(J) < 1e-12 * max(1.0, abs(J).max())
    # the fan's characteristic speeds equal x/t
    lam = (v - R.CS) / (1 - v * R.CS)
    np.testing.assert_allclose(lam, xi, atol=1e-12)


def test_colliding_slabs_symmetric_solution():
    beta = math.sqrt(1 - 1 / 100.0)
    s = R.solve(1.0, beta, 1.0, -beta)
    assert abs(s.vstar) < 1e-12
    assert abs(s.left_head + s.right_head) < 1e-12
    # jump conditions hold for each reflected shock
    v1 = _boost(beta, s.left_head)
    v2 = _boost(0.0, s.left_head)
    assert abs(v1 * v2 - 1 / 3) < 1e-9


def test_paper_quoted_speeds():
    g = json.load(open(GOLDEN))
    P0 = g["P0"]
    for c in g["cases"]:
        s = R.solve(P0, 0.0, c["P1"], 0.0)
        if "beta" in c["check"]:
            assert abs(s.vstar - c["beta"]) <= 0.02, c
        if "v_shock" in c["check"]:
            assert abs(s.right_head - c["v_shock"]) <= 0.02, c
