"""Host-side logic of bench.py (no GPU): the one-GPU guard, the algorithmic
bytes per cell-update, and the traffic bookkeeping from rocprofv3 counters
(scaled by the copy calibration, keyed by the kernel source hash)."""
import json
import os
import subprocess
import sys
import types

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


@pytest.mark.parametrize("args,expected", [
    ((1, True, 0, 0), 384),    # mixed, density, implicit: 2*19*4 * 2 + 2*5*8
    ((0, True, 0, 0), 688),    # FP64 with density
    ((1, False, 0, 0), 216),   # mixed, no density: 152 + 2*4*8
    ((0, False, 0, 0), 368),   # FP64, no density
    ((1, True, 1, 0), 304),    # Euler mode: no previous fields
    ((1, False, 0, 1), 152),   # basic model: f only, no previous fields
    ((0, False, 0, 1), 304),   # basic model, FP64
])
def test_algorithmic_bytes_per_cell(args, expected):
    """The per-cell figures of the measurement plan (384 / 216 / 688 / 368 B)."""
    assert bench.algorithmic_bytes_per_cell(*args) == expected


@pytest.mark.parametrize("args,expected", [
    ((1, True, 0, False, 0), 384),   # mixed 1D, density, implicit: FP64 previous fields
    ((0, True, 0, False, 0), 688),   # FP64
    ((1, False, 0, False, 0), 232),  # mixed, no density: 152 + 80
    ((1, True, 1, True, 0), 305),    # Euler mode (no previous fields) + obstacle mask
    ((1, False, 0, True, 1), 153),   # basic model: f only, no previous fields, obstacle
    ((0, False, 0, False, 1), 304),  # basic model, FP64
    ((1, True, 0, False, 0, True), 344),   # mixed 2D/3D: previous fields in FP32
    ((0, True, 0, False, 0, True), 688),   # FP64 2D/3D: unchanged
    ((1, True, 1, True, 0, True), 305),    # Euler mode: no previous fields
])
def test_stored_bytes_per_cell(args, expected):
    assert bench.stored_bytes_per_cell(*args) == expected


def _csv(path, counter, rows):
    with open(path, "w") as f:
        f.write("Kernel_Name,Counter_Name,Counter_Value\n")
        for k, v in rows:
            f.write(f'"{k}",{counter},{v}\n')


def test_record_traffic_scales_by_the_copy_probe(tmp_path, monkeypatch):
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(tmp_path / "traffic.json"))
    step = "void rlb::k_step<float, 7, true, false, false>(float const*)"
    _csv(tmp_path / "sf.csv", "FETCH_SIZE", [(step, 1000.0), (step, 1200.0), ("other", 5.0)])
    _csv(tmp_path / "sw.csv", "WRITE_SIZE", [(step, 2048.0)])
    # a 1 MiB copy read as 512 KiB by FETCH_SIZE and 1024 KiB by WRITE_SIZE
    _csv(tmp_path / "cf.csv", "FETCH_SIZE", [("MulFunctor", 512.0)])
    _csv(tmp_path / "cw.csv", "WRITE_SIZE", [("MulFunctor", 1024.0)])
    args = types.SimpleNamespace(
        record_traffic=[str(tmp_path / n) for n in ("sf.csv", "sw.csv", "cf.csv", "cw.csv")],
        copy_probe_gib=1.0 / 1024, workload="blast_wave_3d", precision="mixed", lattice="extended")
    bench.record_traffic(args)
    d = json.load(open(bench.TRAFFIC_FILE))
    e = d["blast_wave_3d:mixed"]
    assert e["fetch_scale"] == 2.0 and e["write_scale"] == 1.0
    assert e["fetch_bytes"] == round(1100.0 * 1024 * 2.0)
    assert e["write_bytes"] == 2048 * 1024
    assert e["kernel_hash"] == bench.kernel_hash()
    assert bench.traffic_entry("blast_wave_3d", "mixed") == e["bytes_per_launch"]
    # a counter record of another kernel source is not used
    e["kernel_hash"] = "0" * 16
    json.dump(d, open(bench.TRAFFIC_FILE, "w"))
    assert bench.traffic_entry("blast_wave_3d", "mixed") is None

