#!/usr/bin/env python3
"""Throughput of the ultra-relativistic lattice Boltzmann update on one MI355X.

One step = one fused update of every cell of the workload (moments, FP64
recovery, equilibria, limited streaming, bulk term, implicit collision,
guard), launched through the C ABI (rlb_step_async) on torch's current
stream.  Default workload: the 3D relativistic blast wave, 384^3 cells,
mixed precision (FP32 populations, FP64 recovery), density distribution on.

Prints one JSON line: MLUPS (cell updates per second / 1e6), the roofline of
the step kernel (algorithmic HBM bytes per launch / measured launch time
against 8 TB/s) and the FP64 CPU oracle timed on a bounded sample.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
KERNEL_SOURCES = ["paper_1302_1125_amd/csrc/rlb_kernels.hip", "paper_1302_1125_amd/csrc/rlb_internal.h"]
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_counters.json")


def kernel_hash() -> str:
    h = hashlib.sha256()
    for p in KERNEL_SOURCES:
        with open(os.path.join(ROOT, p), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def algorithmic_bytes_per_cell(precision: int, with_density: bool, collision: int, obstacle: bool) -> int:
    """Each population read once and written once; previous-step fields read
    and written once (implicit mode); obstacle mask read once."""
    e = 8 if precision == 0 else 4
    b = 2 * 19 * e
    if with_density:
        b += 2 * 19 * e
    if collision == 0:
        b += 2 * 5 * 8
    if obstacle:
        b += 1
    return b


def make_workload(name: str, precision: int):
    from paper_1302_1125_amd import workloads as W
    if name == "blast_wave_3d":
        w = W.blast_wave_3d(precision=precision)
    elif name == "shock_cloud_2d":
        w = W.shock_cloud_2d(precision=precision)
    elif name == "colliding_slabs_1d":
        w = W.colliding_slabs_1d(precision=precision)
    elif name == "shock_tube_1d":
        w = W.shock_tube_1d(precision=precision)
    else:
        raise SystemExit(f"unknown workload {name}")
    return w


def traffic_entry(workload: str, precision: str):
    """HBM bytes per launch from committed rocprofv3 FETCH_SIZE/WRITE_SIZE
    counters, if they were taken on the current kernel source."""
    try:
        with open(TRAFFIC_FILE) as f:
            d = json.load(f)
    except (OSError, ValueError):
        return None
    e = d.get(f"{workload}:{precision}")
    if not e or e.get("kernel_hash") != kernel_hash():
        return None
    return e.get("bytes_per_launch")


def cpu_baseline(workload: str, precision: int, budget_s: float):
    """FP64 CPU oracle on a bounded sample of the same workload recipe."""
    from oracle import oracle as O
    from paper_1302_1125_amd import workloads as W
    if workload == "blast_wave_3d":
        w = W.blast_wave_3d(n=96, precision=precision)
        sample = "blast_wave_3d recipe at 96^3 (same radius fraction, seed, parameters)"
    elif workload == "shock_cloud_2d":
        w = W.shock_cloud_2d(nx=512, ny=256, precision=precision)
        sample = "shock_cloud_2d recipe at 512x256"
    else:
        w = make_workload(workload, precision)
        sample = f"{workload} full grid"
    cfg = O.Config(nx=w.nx, ny=w.ny, nz=w.nz, nu=w.nu, dt=w.dt, euler=(w.collision == 1),
                   tau_mode=w.tau_mode, tau=w.tau, eta_over_s=w.eta_over_s, alpha=w.alpha,
                   with_h=bool(w.with_density), bc=w.bc, face=w.face_states,
                   guard_umax=w.guard_umax, guard_efloor=w.guard_efloor)
    o = O.Oracle(cfg)
    o.init(w.eps, w.ux, w.uy, w.uz, w.n if w.with_density else None, w.obstacle)
    t0 = time.perf_counter()
    o.step(1)
    t1 = time.perf_counter()
    per = max(t1 - t0, 1e-6)
    k = max(1, min(200, int(budget_s / per)))
    t0 = time.perf_counter()
    o.step(k)
    dt = time.perf_counter() - t0
    steps = k + 1
    total = dt + per
    return {"value": round(w.ncell * steps / total / 1e6, 4), "unit": "MLUPS", "cores": O.num_threads(),
            "kind": "oracle", "sample": f"{sample}, {steps} steps, {total:.1f} s, FP64"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="blast_wave_3d",
                    choices=["blast_wave_3d", "shock_cloud_2d", "colliding_slabs_1d", "shock_tube_1d"])
    ap.add_argument("--precision", default="mixed", choices=["mixed", "fp64"])
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-probe-gib", type=float, default=0.0,
                    help="only run a plain device copy of this many GiB (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(domain decomposition is described in DESIGN.md, not implemented).", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1302_1125_amd import rlb

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    if args.copy_probe_gib > 0:
        # plain copy of known size: rocprofv3 FETCH_SIZE / WRITE_SIZE of this
        # kernel calibrate the counters used for the step kernel's traffic
        n = int(args.copy_probe_gib * (1 << 30)) // 4
        a = torch.ones(n, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            torch.mul(a, 1.0, out=b)  # an elementwise shader kernel (copy_ may use a blit)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes_read": n * 4, "copy_probe_bytes_written": n * 4}))
        return
    precision = rlb.RLB_MIXED if args.precision == "mixed" else rlb.RLB_FP64
    w = make_workload(args.workload, precision)
    # a dedicated stream (default priority): the library launches on it and
    # the timing events are recorded on it
    stream = torch.cuda.Stream()
    print(f"[bench] workload {w.name} {w.nx}x{w.ny}x{w.nz} {args.precision} h={w.with_density} "
          f"steps={args.steps} warmup={args.warmup}", file=sys.stderr, flush=True)
    ctx = rlb.context_for_workload(w, precision=precision, stream=stream.cuda_stream)
    ctx.rlb_step(args.warmup)

    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev0.record(stream)
    ctx.rlb_step_async(args.steps)
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ctx.rlb_sync()
    stats = ctx.rlb_stats_get()
    ctx.close()
    kern_ms = ev0.elapsed_time(ev1) / args.steps
    ms_per_step = wall * 1e3 / args.steps
    mlups = w.ncell * args.steps / wall / 1e6
    bpc = algorithmic_bytes_per_cell(precision, w.with_density, w.collision, w.obstacle is not None)
    bytes_launch = bpc * w.ncell
    achieved = bytes_launch / (kern_ms * 1e-3) / 1e9
    traffic = traffic_entry(w.name, args.precision)
    print(f"[bench] {mlups:.1f} MLUPS, kernel {kern_ms:.3f} ms/launch, {achieved:.0f} GB/s, "
          f"guard events {stats.guard_events}", file=sys.stderr, flush=True)

    cpu = None
    if not args.no_cpu_baseline:
        print("[bench] CPU oracle baseline ...", file=sys.stderr, flush=True)
        cpu = cpu_baseline(w.name, precision, args.cpu_seconds)

    out = {
        "metric": "cell-updates/s (MLUPS) & % HBM roofline",
        "value": round(mlups, 2),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32-storage/f64-recovery" if precision == rlb.RLB_MIXED else "f64",
        "data": "synthetic",
        "config": {"workload": w.name, "grid": [w.nx, w.ny, w.nz], "cells": w.ncell,
                   "precision": args.precision, "density_distribution": bool(w.with_density),
                   "guard_umax": w.guard_umax, "dt_over_dx": w.dt, "nu": w.nu,
                   "eta_over_s": w.eta_over_s, "alpha": w.alpha, "guard_events": stats.guard_events,
                   "bytes_per_cell_update": bpc},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                     "kernel_ms": round(kern_ms, 4), "algorithmic_bytes_per_launch": bytes_launch},
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
