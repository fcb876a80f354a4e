"""The Rusanov flux (RLB_FLUX_RUSANOV, beyond the paper) on the GPU: the
blocked 1D step against the FP64 oracle with the same flux, and the gamma = 10
inviscid colliding slabs at full size without the guard.  FP64: rel. L2 <=
1e-10 per field; mixed precision: the bounds of test_gpu_parity."""
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


def test_rusanov_is_rejected_outside_1d_and_in_the_server(rlb):
    w = W.random_smooth_state(16, 8, 1, seed=3).copy_with(flux=W.FLUX_RUSANOV)
    with pytest.raises(rlb.RLBError):
        rlb.context_for_workload(w)
    common = rlb.config_from(8, with_density=True, flux=rlb.RLB_FLUX_RUSANOV)
    with pytest.raises(rlb.RLBError):
        rlb.Server(common, 1 << 26, 8)
