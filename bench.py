#!/usr/bin/env python3
"""Benchmark of the PIC particle step on one MI355X.

Metric: particle pushes per second (one push = gather + Boris push + advance +
charge-conserving deposit of one particle), whole step included (the Yee
field solve and the rebin checks run inside the timed region), inputs already
resident in HBM.  Workload (default): the 2D3V laser-wakefield case, 1024x256
cells, 2,097,152 electrons, quadratic shape.  Prints one JSON line.

  python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload lwfa2d|thermal2d|beam3d|cubic3d]
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def make_workload(name):
    from paper_1503_00276_amd import workloads as W

    if name == "lwfa2d":
        return W.workload2()
    if name == "thermal2d":
        return W.workload1()
    if name == "beam3d":
        return W.workload3()
    if name == "cubic3d":
        return W.workload5()
    if name == "cubic3d_sub":
        return W.workload5_sub()
    if name == "thermal2d_lwfa_grid":
        # same grid, cell size, time step and particle count as lwfa2d, thermal random loading
        return W.thermal((1024, 256), (0.05, 0.2), W.courant_dt((0.05, 0.2), 0.95), 2, 8, 0.05,
                         0.01, seed_k=6, steps=2000, name="2d3v_thermal_1024x256_quadratic")
    raise SystemExit(f"unknown workload {name}")


def bytes_per_push(wl):
    """Algorithmic HBM bytes per push: particle state read (cell, offsets, u, w)
    and written (cell, offsets, u), plus E,B read once (24 B/cell) and J written
    once (12 B/cell) shared by the particles of a cell."""
    d = wl.ndim
    particle = (4 + 4 * d + 12 + 4) + (4 + 4 * d + 12)
    ppc = wl.n / wl.ncell
    return particle + 36.0 / ppc


def cpu_baseline(wl, max_particles):
    """Time the FP64 oracle (single thread, as it stands) on one full step of a
    bounded sample of the workload's particles."""
    import numpy as np
    import oracle

    oracle.build(force=False)
    g = oracle.Grid(dim=wl.ndim, nx=wl.nx, dx=wl.dx, dt=wl.dt, order=wl.order)
    n = min(wl.n, max_particles)
    idx = np.arange(wl.n) if n == wl.n else np.random.default_rng(0).choice(wl.n, n, replace=False)
    E = wl.E if wl.E is not None else np.zeros((3, wl.ncell))
    B = wl.B if wl.B is not None else np.zeros((3, wl.ncell))
    t0 = time.perf_counter()
    oracle.step(g, wl.x[idx], wl.u[idx], wl.w[idx], 1.0 / wl.rqm, E, B)
    t = time.perf_counter() - t0
    what = "all" if n == wl.n else "a random sample of"
    return {
        "value": n / t,
        "unit": "particle pushes/s",
        "cores": 1,
        "kind": "oracle",
        "sample": f"one FP64 oracle step (gather, push, deposit, field solve) of {what} {n} particles "
                  f"of the workload, single thread, {t:.1f} s",
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", default="lwfa2d")
    ap.add_argument("--profile-steps", type=int, default=50)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample", type=int, default=2_097_152)
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="also run a plain device copy of this many MiB (counter calibration)")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on exactly one GPU: this build has no multi-GPU path "
              "(the sharding design is described in DESIGN.md); use --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_1503_00276_amd import pic

    assert torch.cuda.is_available(), "no GPU visible"
    torch.cuda.set_device(0)
    stream = torch.cuda.Stream()  # a non-default stream so the library can capture graphs on it

    log(f"generating workload {args.workload}")
    wl = make_workload(args.workload)
    cfg = pic.Config(ndim=wl.ndim, nx=wl.nx, dx=wl.dx, dt=wl.dt, shape_order=wl.order,
                     ion_density=wl.ion_density)
    sim = pic.Pic(cfg, stream=stream)
    log(f"loading {wl.n} particles")
    sim.load_particles(wl.x, wl.u, wl.w, rqm=wl.rqm)
    if wl.E is not None:
        sim.load_fields(wl.E, wl.B)
    info = sim.info()

    log(f"warmup {args.warmup} steps")
    sim.step(args.warmup)
    sim.sync()

    log(f"timing {args.steps} steps")
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev0.record(stream)
    sim.step(args.steps)
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    gpu_ms = ev0.elapsed_time(ev1)
    sim.sync()
    elapsed = max(wall, gpu_ms / 1000.0)
    value = wl.n * args.steps / elapsed

    # per-kernel times: the same steps launched one by one with HIP events
    log(f"profiling {args.profile_steps} steps")
    sim.profile(2)
    sim.step(args.profile_steps)
    kt = sim.kernel_times()
    sim.profile(0)
    sim.sync()
    gpd_ms, gpd_n = kt["particle"]
    gpd_avg_s = gpd_ms / max(gpd_n, 1) / 1000.0
    bpp = bytes_per_push(wl)
    achieved = wl.n * bpp / gpd_avg_s / 1e9
    counts = sim.counts()

    if args.calib_copy_mib > 0:
        n = args.calib_copy_mib * 1024 * 1024 // 4
        a = torch.ones(n, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        del a, b

    cpu = None
    if not args.no_cpu_baseline:
        log("timing the CPU oracle baseline")
        cpu = cpu_baseline(wl, args.cpu_sample)

    out = {
        "metric": "particle pushes/sec (gather+push+deposit), whole step, 1 GPU",
        "value": value,
        "unit": "particle pushes/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed * 1000.0 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": wl.name,
            "cells": list(wl.nx),
            "particles": wl.n,
            "shape_order": wl.order,
            "dt": wl.dt,
            "dx": list(wl.dx),
            "tile": list(info.tile)[:wl.ndim],
            "sort_interval": info.sort_interval,
            "slack": info.slack,
            "rebins_done": int(counts[2]),
            "rebin_checks": int(counts[3]),
        },
        "roofline": {
            "bound": "hbm",
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": None,
            "kernel": "gpd_kernel (fused gather+push+deposit)",
            "bytes_per_push": bpp,
            "kernel_avg_us": gpd_avg_s * 1e6,
            "kernel_pushes_per_s": wl.n / gpd_avg_s,
        },
        "kernel_times_ms_per_step": {k: v[0] / max(v[1], 1) for k, v in kt.items()},
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)
    sim.close()


if __name__ == "__main__":
    main()
