"""Whole-length runs on the GPU under the STABILISED parameter set of the
workloads module (nu = 4, alpha = 0.1, dt = 0.075; same recipes and physical
run times): the gamma = 10 colliding slabs, the strong 3D shock-cloud and a
192^3 blast wave stay admissible without a single guard event, in FP64 and
in mixed precision.  Under the default parameters the slabs become
inadmissible before the end even with the guard firing (linear instability
of fast uniform flows, see test_oracle_stability).
"""
import numpy as np
import pytest

from paper_1302_1125_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def rlb():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1302_1125_amd import rlb as R
    R.load()
    return R


def _run(R, w, precision, chunk=1000):
    """Status (0 or the step status), stats and final fields."""
    print(f"[gpu-case] {w.name} {w.shape} nu={w.nu} alpha={w.alpha} dt={w.dt} steps={w.steps} "
          f"prec={precision}", flush=True)
    ctx = R.context_for_workload(w, precision=precision)
    done, rc = 0, 0
    try:
        while done < w.steps and rc == 0:
            k = min(chunk, w.steps - done)
            rc = ctx.status_of_step(k)
            done += k
        st = ctx.rlb_stats_get()
        out = ctx.rlb_moments() if rc == 0 else None
    finally:
        ctx.close()
    print(f"  status {rc} guard events {st.guard_events} first bad step {st.first_bad_step}", flush=True)
    return rc, st, out


def _gamma(out):
    eps, ux, uy, uz, n = out
    return 1.0 / np.sqrt(1.0 - ux ** 2 - uy ** 2 - uz ** 2)


@pytest.mark.parametrize("precision", [W.FP64, W.MIXED])
def test_colliding_slabs_stabilised_full_length(rlb, precision):
    w = W.stabilised(W.colliding_slabs_1d(precision=precision))
    assert w.steps == 13333  # 4000 steps of dt = 0.25
    rc, st, out = _run(rlb, w, precision)
    assert rc == 0 and st.guard_events == 0
    eps, n = out[0].ravel(), out[4].ravel()
    c = w.nx // 2
    assert abs(eps[c - 16:c + 16].mean() / (3.0 * 529.998) - 1.0) < 1e-3
    assert n.max() < 100.0 and _gamma(out).max() < 15.0


def test_colliding_slabs_default_parameters_fail(rlb):
    w = W.colliding_slabs_1d(precision=W.FP64)
    rc, st, _ = _run(rlb, w, W.FP64)
    assert rc == rlb.RLB_E_INADMISSIBLE and 0 < st.first_bad_step < w.steps
    assert st.guard_events > 0


@pytest.mark.parametrize("precision", [W.FP64, W.MIXED])
def test_strong_shock_cloud_3d_stabilised_full_length(rlb, precision):
    w = W.stabilised(W.shock_cloud_3d(regime="strong", precision=precision))
    assert w.steps == 2000
    rc, st, out = _run(rlb, w, precision, chunk=500)
    assert rc == 0 and st.guard_events == 0
    assert _gamma(out).max() < 3.0 and np.isfinite(out[0]).all() and out[0].max() < 3000.0


def test_blast_wave_192_stabilised_full_length(rlb):
    w = W.stabilised(W.blast_wave_3d(n=192, radius=16.0, precision=W.MIXED))
    assert w.steps == 4000
    rc, st, out = _run(rlb, w, W.MIXED, chunk=500)
    assert rc == 0 and st.guard_events == 0
    assert out[0].max() < 3000.0 and out[4].max() < 10.0 and _gamma(out).max() < 3.0
