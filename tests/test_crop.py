"""The dependency-cone crop used by the full-size GPU parity tests (CPU):
sampled oracle values computed from crops equal the full-domain run."""
import numpy as np

from paper_1302_1125_amd import workloads as W
from tests._helpers import oracle_for, sampled_oracle_fields


def _check(w, cells, steps):
    o = oracle_for(w)
    assert o.step(steps) == 0
    full = o.fields()
    ref = sampled_oracle_fields(w, cells, steps)
    for row, c in zip(ref, cells):
        np.testing.assert_allclose(row, [a[c] for a in full], rtol=1e-13, atol=1e-15)


def test_crop_shock_cloud():
    w = W.shock_cloud_2d(nx=96, ny=48, precision=W.FP64)
    _check(w, [(0, 0, 0), (0, 47, 95), (0, 24, 5), (0, 10, 40), (0, 30, 60), (0, 1, 94)], 3)


def test_crop_blast_periodic_3d():
    w = W.blast_wave_3d(n=24, precision=W.FP64)
    _check(w, [(0, 0, 0), (23, 23, 23), (12, 12, 12), (12, 3, 20), (1, 22, 11)], 3)


def test_crop_shock_cloud_3d():
    # inlet at x = 0, outflow on the other five faces, a spherical obstacle
    w = W.shock_cloud_3d(nx=40, ny=20, nz=20, regime="strong", precision=W.FP64)
    _check(w, [(0, 0, 0), (19, 19, 39), (10, 10, 20), (10, 10, 13), (10, 12, 22), (3, 17, 1),
               (19, 0, 38)], 3)


def test_crop_basic_model_3d():
    # basic model: diagonal links read edge ghosts; inlet, outflow faces, obstacle
    w = W.as_basic(W.shock_cloud_3d(nx=40, ny=20, nz=20, regime="weak", viscous=True,
                                    precision=W.FP64))
    _check(w, [(0, 0, 0), (19, 19, 39), (10, 10, 20), (10, 10, 13), (10, 12, 22), (3, 17, 1),
               (19, 0, 38)], 3)
