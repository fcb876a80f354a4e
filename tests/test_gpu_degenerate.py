"""Degenerate grids on the GPU against the FP64 oracle: axes of 2 and 3
cells (shorter than the 5-cell stencil, so periodic neighbours wrap onto the
cell itself or its only neighbour, and fixed or outflow faces are read by
every cell), in 1D (the temporally blocked step), 2D and 3D (the staged
step), implicit and Euler mode; the z-marching step on 2 x 2 and 2 x 3
columns; and a zero-step call, which leaves the fields as initialised.
FP64: rel. L2 <= 1e-10 per field; mixed precision: the per-field bounds of
the parity tests."""
import numpy as np
import pytest

from paper_1302_1125_amd import workloads as W
from tests._helpers import field_errors, oracle_for

pytestmark = pytest.mark.gpu

_P, _F, _O = W.BC_PERIODIC, W.BC_FIXED, W.BC_OUTFLOW
STEPS = 30
MIXED_BOUNDS = {"eps": 2e-5, "p": 2e-5, "n": 2e-5, "gux": 2e-4, "guy": 2e-4, "guz": 2e-4}


@pytest.fixture(scope="module")
def rlb():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1302_1125_amd import rlb as R
    R.load()
    return R


def _tiny(shape, bc, euler=False, precision=W.FP64):
    nz, ny, nx = shape
    w = W.random_smooth_state(nx, ny, nz, seed=5 + nx + 3 * ny + 7 * nz, with_density=True, alpha=0.15,
                              tau_mode=W.TAU_ETA_OVER_S, eta_over_s=0.05, dt=0.15,
                              collision=int(euler), precision=precision)
    faces = [[3.0 + 0.1 * k, 0.05 * (k - 2), -0.03, 0.02 * (k - 3), 1.0 + 0.05 * k] for k in range(6)]
    if ny == 1:
        faces = [[f[0], f[1], 0.0, 0.0, f[4]] for f in faces]
    return w.copy_with(bc=list(bc) + [_P] * (6 - len(bc)), face_states=faces)


def _gpu(R, w, steps, precision):
    print(f"[gpu-case] degenerate {w.nx}x{w.ny}x{w.nz} bc={w.bc} coll={w.collision} "
          f"prec={precision} steps={steps}", flush=True)
    ctx = R.context_for_workload(w, precision=precision)
    ctx.rlb_step(steps)
    out = ctx.rlb_moments()
    st = ctx.rlb_stats_get()
    ctx.close()
    return out, st


@pytest.mark.parametrize("shape,bc", [
    ((1, 1, 2), [_P, _P]), ((1, 1, 3), [_F, _O]), ((1, 1, 2), [_O, _F]), ((1, 1, 5), [_P, _P]),
    ((1, 2, 2), [_P] * 4), ((1, 3, 2), [_F, _O, _P, _P]), ((1, 2, 5), [_P, _P, _F, _O]),
    ((2, 2, 2), [_P] * 6), ((3, 2, 3), [_F, _O, _P, _P, _O, _F]), ((2, 3, 2), [_P, _P, _F, _F, _P, _P]),
])
@pytest.mark.parametrize("euler", [False, True])
def test_tiny_grids_fp64(rlb, shape, bc, euler):
    w = _tiny(shape, bc, euler)
    g, st = _gpu(rlb, w, STEPS, W.FP64)
    o = oracle_for(w)
    assert o.step(STEPS) == 0
    errs = field_errors(g, o.fields())
    print(errs)
    assert max(errs.values()) <= 1e-10, errs
    assert st.steps == STEPS and st.guard_events == o.guard_events


@pytest.mark.parametrize("shape,bc", [((8, 2, 2), [_P] * 6), ((9, 3, 2), [_F, _O, _P, _P, _O, _F]),
                                      ((17, 2, 3), [_P, _P, _F, _O, _P, _P])])
def test_tiny_columns_zmarch_mixed(rlb, shape, bc):
    """Mixed precision, implicit, 3D with nz >= 8: the z-marching step, whose
    64 x 4 column then holds 2 or 3 real cells per row and plane."""
    w = _tiny(shape, bc, precision=W.MIXED)
    g, _ = _gpu(rlb, w, STEPS, W.MIXED)
    o = oracle_for(w)
    assert o.step(STEPS) == 0
    errs = field_errors(g, o.fields())
    print(errs)
    for k, v in errs.items():
        assert v <= MIXED_BOUNDS[k], (k, v)


@pytest.mark.parametrize("shape", [(1, 1, 7), (1, 5, 9), (3, 4, 6)])
@pytest.mark.parametrize("precision", [W.FP64, W.MIXED])
def test_zero_steps_leave_the_initial_fields(rlb, shape, precision):
    """rlb_step(0) launches nothing: the moments read back are the
    initialised equilibria's (the fields to the recovery's rounding)."""
    w = _tiny(shape, [_P] * 6, precision=precision)
    g, st = _gpu(rlb, w, 0, precision)
    assert st.steps == 0
    tol = 1e-13 if precision == W.FP64 else 2e-6
    for a, ref in zip(g, (w.eps, w.ux, w.uy, w.uz, w.n)):
        np.testing.assert_allclose(a, ref, rtol=tol, atol=tol)
