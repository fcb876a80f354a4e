"""The Rusanov flux (RLB_FLUX_RUSANOV, beyond the paper) on the GPU: the
blocked 1D step and the staged 2D/3D step against the FP64 oracle with the
same flux, the gamma = 10 inviscid colliding slabs and the paper's strong 3D
shock-cloud without the guard.  FP64: rel. L2 <= 1e-10 per field; mixed
precision: the bounds of test_gpu_parity."""
import math
import os

import numpy as np
import pytest

from oracle import riemann as R
from paper_1302_1125_amd import workloads as W
from tests._helpers import field_errors, oracle_for

pytestmark = pytest.mark.gpu

MIXED_BOUNDS = {"eps": 2e-5, "p": 2e-5, "n": 2e-5, "gux": 2e-4}
KEYS = ("eps", "p", "n", "gux")


@pytest.fixture(scope="module")
def rlb():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1302_1125_amd import rlb as R_
    R_.load()
    return R_


def _gpu(R_, w, steps, precision, tb=None):
    print(f"[gpu-case] rusanov {w.name} nx={w.nx} steps={steps} precision={precision} tb={tb}", flush=True)
    old = os.environ.get("RLB_TB_STEPS")
    if tb is not None:
        os.environ["RLB_TB_STEPS"] = str(tb)
    try:
        ctx = R_.context_for_workload(w, precision=precision)
    finally:
        if tb is not None:
            if old is None:
                del os.environ["RLB_TB_STEPS"]
            else:
                os.environ["RLB_TB_STEPS"] = old
    try:
        ctx.rlb_step(steps)
        out = ctx.rlb_moments()
        st = ctx.rlb_stats_get()
    finally:
        ctx.close()
    return out, st


def _smooth(bc, euler, nx=700):
    w = W.random_smooth_state(nx, 1, 1, seed=31 + nx, with_density=True, alpha=0.1,
                              tau_mode=W.TAU_ETA_OVER_S, eta_over_s=0.05, dt=0.25, umax=0.5)
    return w.copy_with(collision=int(euler), flux=W.FLUX_RUSANOV, bc=list(bc) + [W.BC_PERIODIC] * 4,
                       face_states=[[3.4, 0.2, 0, 0, 1.1], [2.7, -0.3, 0, 0, 0.95]] + [[3.0, 0, 0, 0, 1.0]] * 4)


@pytest.mark.parametrize("euler", [True, False])
@pytest.mark.parametrize("bc", [(W.BC_PERIODIC, W.BC_PERIODIC), (W.BC_FIXED, W.BC_OUTFLOW),
                                (W.BC_OUTFLOW, W.BC_FIXED)])
def test_fp64_parity(rlb, euler, bc):
    w = _smooth(bc, euler)
    steps = 60
    o = oracle_for(w)
    assert o.step(steps) == 0
    ref = o.fields()
    for tb in (None, 1):  # 8 steps per launch, and one
        out, st = _gpu(rlb, w, steps, W.FP64, tb)
        errs = field_errors(out, ref, keys=KEYS)
        print(errs)
        assert max(errs.values()) <= 1e-10, (tb, errs)


@pytest.mark.parametrize("euler", [True, False])
def test_mixed_within_bounds(rlb, euler):
    w = _smooth((W.BC_FIXED, W.BC_OUTFLOW), euler, nx=1000)
    o = oracle_for(w)
    assert o.step(100) == 0
    out, _ = _gpu(rlb, w, 100, W.MIXED)
    errs = field_errors(out, o.fields(), keys=KEYS)
    print(errs)
    for k, v in errs.items():
        assert v <= MIXED_BOUNDS[k], (k, v)


def test_inviscid_slabs_parity(rlb):
    """gamma = 10 inviscid slabs, 2048 cells, 1000 steps, guard off: FP64
    parity with the oracle and admissible throughout."""
    w = W.colliding_slabs_1d(nx=2048, steps=1000, guard_umax=0.0)
    w = w.copy_with(collision=W.COLL_EULER, flux=W.FLUX_RUSANOV)
    o = oracle_for(w)
    assert o.step(1000) == 0
    out, st = _gpu(rlb, w, 1000, W.FP64)
    assert st.first_bad_step == -1 and st.guard_events == 0
    errs = field_errors(out, o.fields(), keys=KEYS)
    print(errs)
    assert max(errs.values()) <= 1e-10, errs


@pytest.mark.parametrize("precision", [W.FP64, W.MIXED])
def test_inviscid_slabs_full_length(rlb, precision):
    """The colliding-slabs recipe (8192 cells, gamma = 10, density jitter) in
    the Euler mode over its 4000 steps with the guard off: admissible in FP64
    and mixed precision, the centre energy density at the exact ideal-fluid
    value (the minmod flux leaves the admissible set in the first step)."""
    w = W.colliding_slabs_1d(steps=4000, guard_umax=0.0)
    w = w.copy_with(collision=W.COLL_EULER, flux=W.FLUX_RUSANOV)
    out, st = _gpu(rlb, w, 4000, precision)
    assert st.first_bad_step == -1 and st.guard_events == 0
    eps = out[0].ravel()
    s = R.solve(1.0, math.sqrt(0.99), 1.0, -math.sqrt(0.99))
    c = len(eps) // 2
    centre = np.median(eps[c - 10:c + 10]) / (3.0 * s.pstar)
    print("centre / exact", centre)
    assert abs(centre - 1.0) < 2e-4


@pytest.mark.parametrize("shape", [(1, 33, 70), (10, 12, 16), (9, 6, 70)])
@pytest.mark.parametrize("euler", [True, False])
def test_staged_2d_3d_parity(rlb, shape, euler):
    """The staged step (2D and 3D; the 3D mixed implicit case would otherwise
    take the z-march) with fixed, outflow and periodic faces: FP64 against the
    oracle, and mixed precision within the parity bounds."""
    nz, ny, nx = shape
    w = W.random_smooth_state(nx, ny, nz, seed=41 + nx, with_density=True, alpha=0.15,
                              tau_mode=W.TAU_ETA_OVER_S, eta_over_s=0.05, dt=0.15)
    bc = [W.BC_FIXED, W.BC_OUTFLOW, W.BC_OUTFLOW, W.BC_FIXED] + ([W.BC_PERIODIC] * 2 if nz == 1 else
                                                                [W.BC_FIXED, W.BC_OUTFLOW])
    faces = [[3.0 + 0.1 * k, 0.05 * (k - 2), -0.03, 0.02 * (k - 3) if nz > 1 else 0.0, 1.0 + 0.05 * k]
             for k in range(6)]
    w = w.copy_with(collision=int(euler), flux=W.FLUX_RUSANOV, bc=bc, face_states=faces)
    steps = 20
    o = oracle_for(w)
    assert o.step(steps) == 0
    ref = o.fields()
    out, _ = _gpu(rlb, w, steps, W.FP64)
    errs = field_errors(out, ref)
    print("FP64", errs)
    assert max(errs.values()) <= 1e-10, errs
    out, _ = _gpu(rlb, w, steps, W.MIXED)
    errs = field_errors(out, ref, keys=KEYS)
    print("mixed", errs)
    for k, v in errs.items():
        assert v <= MIXED_BOUNDS[k], (k, v)


def test_strong_3d_shock_cloud_parity_without_guard(rlb):
    """The paper's 3D shock-cloud, strong regime (Euler mode), at 60 x 30 x 30
    with the guard off (the minmod flux leaves the admissible set at step 34
    of this run).  The flow amplifies rounding from about step 150 on: in the
    oracle a one-ulp change of the input moves the fields by 2e-14 at step
    180 and 1.5e-7 at step 300.  So FP64 parity is checked at step 120, and
    the run continues to step 300 admissible."""
    w = W.shock_cloud_3d(nx=60, ny=30, nz=30, regime="strong", precision=W.FP64, steps=300,
                         guard_umax=0.0).copy_with(flux=W.FLUX_RUSANOV)
    o = oracle_for(w)
    assert o.step(120) == 0
    out, st = _gpu(rlb, w, 120, W.FP64)
    assert st.first_bad_step == -1 and st.guard_events == 0
    errs = field_errors(out, o.fields(), keys=KEYS)
    print(errs)
    assert max(errs.values()) <= 1e-10, errs
    _, st = _gpu(rlb, w, 300, W.FP64)
    assert st.first_bad_step == -1 and st.guard_events == 0


@pytest.mark.parametrize("precision", [W.FP64, W.MIXED])
def test_strong_3d_shock_cloud_full_size(rlb, precision):
    """200 x 100 x 100, 1000 steps, the recipe's bulk term (alpha = 0.2), guard
    off: admissible throughout with the Rusanov flux in FP64 and mixed
    precision.  Under this flux the bulk term acts on the rest population too;
    when it acted on the moving populations only (as Eq. (55) has it), it
    removed the rest population's (negative-weight) energy at the cell, the
    update was no longer a convex combination of admissible states, and this
    run left the admissible set at step 359 in FP64 (357 in the oracle) and
    262 in mixed precision."""
    w = W.shock_cloud_3d(regime="strong", precision=precision, guard_umax=0.0)
    w = w.copy_with(flux=W.FLUX_RUSANOV)
    out, st = _gpu(rlb, w, w.steps, precision)
    assert st.first_bad_step == -1 and st.guard_events == 0
    assert all(np.all(np.isfinite(a)) for a in out)


def test_rusanov_is_rejected_by_the_server_and_the_basic_lattice(rlb):
    common = rlb.config_from(8, with_density=True, flux=rlb.RLB_FLUX_RUSANOV)
    with pytest.raises(rlb.RLBError):
        rlb.Server(common, 1 << 26, 8)
    w = W.as_basic(W.shock_tube_1d()).copy_with(flux=W.FLUX_RUSANOV)
    with pytest.raises(rlb.RLBError):
        rlb.context_for_workload(w)
