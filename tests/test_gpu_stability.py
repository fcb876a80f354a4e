"""The HIP step against the linear theory of uniform flows, through the C ABI
(FP64), without the oracle in the loop.

A uniform flow perturbed by a checkerboard pattern (-1)^(x), (-1)^(x+y) or
(-1)^(x+y+z) keeps the minmod correction exactly idle, so one step acts on
the perturbation as a fixed matrix (the von Neumann matrices of
test_oracle_stability, built from the lattice tables and equilibria).  The
checkerboard amplitude of eps (energy part) or n (density part) read back
after every step must follow that matrix: a growing case (flow along x at
u = 0.8), damped oblique cases in 2D and 3D (staged tiles, z loads, bulk
term) and the density part.
"""
import math

import numpy as np
import pytest

from paper_1302_1125_amd import workloads as W
from tests.test_oracle_stability import (NU0, _checkerboard, _f_linear, _f_matrix, _h_linear,
                                         _h_matrix)

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def rlb():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1302_1125_amd import rlb as R
    R.load()
    return R


def _workload(shape, u, dt, tau, alpha, with_density, eps, n):
    nz, ny, nx = shape
    w = W.Workload("checkerboard", nx, ny, nz, 0, precision=W.FP64, tau_mode=W.TAU_UNIFORM, tau=tau,
                   alpha=alpha, with_density=with_density, nu=NU0, dt=dt)
    ones = np.ones(shape)
    w.eps, w.ux, w.uy, w.uz = eps, u[0] * ones, u[1] * ones, u[2] * ones
    w.n = n if with_density else None
    return w


def _follow(R, w, axes, x0, G, out_vec, steps, min_gain=1e-2):
    """Largest deviation of the read-back checkerboard amplitude from the
    linear prediction, relative to the predicted amplitude; and the gain."""
    print(f"[gpu-case] checkerboard {w.shape} axes={axes} steps={steps}", flush=True)
    sgn = _checkerboard(w.shape, axes)
    ctx = R.context_for_workload(w)
    x, worst, a0 = x0, 0.0, abs(out_vec @ x0)
    try:
        for _ in range(steps):
            ctx.rlb_step(1)
            x = G @ x
            eps, ux, uy, uz, n = ctx.rlb_moments()
            field = n if w.with_density else eps
            meas = float((field.reshape(-1) * sgn).mean())
            pred = float(out_vec @ x)
            if abs(pred) > min_gain * a0:
                worst = max(worst, abs(meas - pred) / abs(pred))
    finally:
        ctx.close()
    return worst, abs(out_vec @ x) / a0


@pytest.mark.parametrize("shape,axes,u,dt,tau,alpha,steps", [
    ((1, 1, 64), (0,), (0.8, 0.0, 0.0), 0.25, 1.0, 0.0, 100),          # grows e^{0.029} per step
    ((1, 8, 64), (0, 1), (0.6, 0.4, 0.0), 0.25, 1.0, 0.0, 10),         # 2D staged tiles, damped
    ((4, 4, 64), (0, 1, 2), (0.5, 0.3, 0.2), 0.15, 0.7, 0.2, 5),       # 3D, bulk term, damped
])
def test_energy_part_follows_linear_theory(rlb, shape, axes, u, dt, tau, alpha, steps):
    from oracle import oracle as O
    amp = 1e-6
    lin = _f_linear(O, NU0, u)
    K, J, dfe, deps = lin
    th = np.array([math.pi if a in axes else 0.0 for a in range(3)])
    G = _f_matrix(O, NU0, u, dt, tau, alpha, th, lin).real
    x0 = np.concatenate([dfe * amp, K @ dfe * amp])
    out_vec = np.concatenate([deps @ K, np.zeros(4)])  # eps amplitude of the populations
    eps = 3.0 + amp * _checkerboard(shape, axes).reshape(shape)
    w = _workload(shape, u, dt, tau, alpha, False, eps, None)
    worst, gain = _follow(rlb, w, axes, x0, G, out_vec, steps)
    print(f"max rel. deviation from the linear prediction {worst:.1e}, gain {gain:.3g}")
    assert worst < 1e-6, worst
    assert (gain > 2.0) if u == (0.8, 0.0, 0.0) else (gain < 1.0)


@pytest.mark.parametrize("shape,axes,u,tau,steps,grows", [
    ((1, 1, 64), (0,), (0.6, 0.0, 0.0), None, 30, True),       # Euler mode: grows e^{0.18} per step
    ((4, 4, 64), (0, 1, 2), (0.3, 0.3, 0.1), 0.8, 10, False),  # 3D, implicit, damped
])
def test_density_part_follows_linear_theory(rlb, shape, axes, u, tau, steps, grows):
    from oracle import oracle as O
    amp, dt = 1e-6, (0.25 if len(axes) == 1 else 0.15)
    he1, kn = _h_linear(O, NU0, u)
    th = np.array([math.pi if a in axes else 0.0 for a in range(3)])
    G = _h_matrix(O, NU0, u, dt, tau, th).real
    x0 = he1 * amp if tau is None else np.concatenate([he1 * amp, [amp]])
    out_vec = kn if tau is None else np.concatenate([kn, [0.0]])
    n = 1.0 + amp * _checkerboard(shape, axes).reshape(shape)
    w = _workload(shape, u, dt, tau or 1.0, 0.0, True, np.full(shape, 3.0), n)
    if tau is None:
        w.collision = W.COLL_EULER
    worst, gain = _follow(rlb, w, axes, x0, G, out_vec, steps)
    print(f"max rel. deviation from the linear prediction {worst:.1e}, gain {gain:.3g}")
    assert worst < 1e-6, worst
    assert (gain > 2.0) if grows else (gain < 1.0)


@pytest.mark.parametrize("mode", [3, 8])
def test_basic_model_follows_linear_theory(rlb, mode):
    """The basic-model kernel (k_step_basic, FP64) on a uniform flow at
    u = 0.7 with a small perturbation of eps and of every velocity component:
    the Fourier amplitude of eps read back after every step follows the
    basic model's linear matrix (the paper's beta ~ 0.6 limit: it grows)."""
    import math as m
    from oracle import oracle as O
    from tests.test_oracle_stability import _basic_linear, _basic_matrix, _fd
    nx, u, tau, amp, steps = 16, 0.7, 0.6, 1e-8, 40
    theta = 2.0 * m.pi * mode / nx
    lin = _basic_linear(O, 1.0, u)
    K, J, dfe = lin
    G = _basic_matrix(O, 1.0, u, tau, theta, lin)
    U0 = O.moments(1.0, O.feq(1.0, 3.0, u, 0.0, 0.0, basic=True), basic=True)[0]
    deps = np.array([_fd(lambda U: np.array([O.recover(U, 0.0, with_h=False)[1][0]]), U0, k, 1e-5 * U0[0])[0]
                     for k in range(4)])
    d = amp * np.array([3.0, 0.7, 0.5, 0.3])
    x = np.arange(nx)
    c = np.cos(theta * x).reshape(1, 1, nx)
    w = W.Workload("basic_mode", nx, 1, 1, steps, precision=W.FP64, tau_mode=W.TAU_UNIFORM, tau=tau,
                   nu=1.0, lattice=W.LATTICE_BASIC)
    w.eps, w.ux, w.uy, w.uz = 3.0 + d[0] * c, u + d[1] * c, d[2] * c, d[3] * c
    print(f"[gpu-case] basic model mode {mode} of {nx}, u = {u}, {steps} steps", flush=True)
    proj = np.exp(-1j * theta * x) * (1.0 if mode == nx // 2 else 2.0) / nx
    a = (dfe @ d).astype(complex)
    a0 = abs(deps @ K @ a)
    ctx = rlb.context_for_workload(w)
    worst = 0.0
    try:
        for _ in range(steps):
            ctx.rlb_step(1)
            a = G @ a
            meas = ctx.rlb_moments()[0].reshape(-1) @ proj
            pred = deps @ K @ a
            worst = max(worst, abs(meas - pred) / abs(pred))
    finally:
        ctx.close()
    gain = abs(deps @ K @ a) / a0
    print(f"max rel. deviation from the linear prediction {worst:.1e}, gain {gain:.3g}")
    assert worst < 1e-5, worst
    assert gain > 2.0
