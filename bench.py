#!/usr/bin/env python3
"""Benchmark of the PIC particle step on one MI355X.

Metric: particle pushes per second (one push = gather + Boris push + advance +
charge-conserving deposit of one particle), whole step included (the Yee
field solve and the rebin checks run inside the timed region), inputs already
resident in HBM.  Workload (default): the 2D3V laser-wakefield case, 1024x256
cells, 2,097,152 electrons, quadratic shape, with the layout the autotuner
picks.  A second leg times the batched scan (64 independent 2D thermal
instances of uneven grids and particle counts advanced by the batched step)
against the same instances run plain one after another.  Prints one JSON line.

  python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload lwfa2d|thermal2d|beam3d|cubic3d]
                  [--no-batched] [--no-cpu-baseline] [--tune-steps T]
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


def cpu_baseline(wl, max_particles, min_seconds=10.0, max_steps=20):
    """Time the FP64 oracle (single thread, as it stands) on consecutive full
    steps of a bounded sample of the workload's particles, until about
    min_seconds of CPU work."""
    import numpy as np
    import oracle

    oracle.build(force=False)
    g = oracle.Grid(dim=wl.ndim, nx=wl.nx, dx=wl.dx, dt=wl.dt, order=wl.order)
    n = min(wl.n, max_particles)
    idx = np.arange(wl.n) if n == wl.n else np.random.default_rng(0).choice(wl.n, n, replace=False)
    x, u, w = wl.x[idx], wl.u[idx], wl.w[idx]
    E = wl.E if wl.E is not None else np.zeros((3, wl.ncell))
    B = wl.B if wl.B is not None else np.zeros((3, wl.ncell))
    t = 0.0
    steps = 0
    while steps < max_steps and (steps == 0 or t < min_seconds):
        t0 = time.perf_counter()
        r = oracle.step(g, x, u, w, 1.0 / wl.rqm, E, B)
        t += time.perf_counter() - t0
        x, u, E, B = r.x, r.u, r.E, r.B
        steps += 1
    what = "all" if n == wl.n else "a random sample of"
    return {
        "value": n * steps / t,
        "unit": "particle pushes/s",
        "cores": 1,
        "kind": "oracle",
        "sample": f"{steps} consecutive FP64 oracle steps (gather, push, deposit, field solve) of {what} {n} "
                  f"particles of the workload, single thread, {t:.1f} s",
    }


def measured_traffic(wl, info, kernel_avg_s):
    """HBM traffic of the particle kernel in GB/s from the committed counter
    record (rocprofv3 FETCH_SIZE and WRITE_SIZE per dispatch, each scaled by
    what the same counter reads for a plain device copy of known size), or
    None when no record matches this workload and layout or the kernel's
    source changed since the counters were taken."""
    import hashlib

    path = os.path.join(ROOT, "profiles", "gpd_lwfa2d_1024x256_counters.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    h = hashlib.sha256()
    for f in ["gpd.hip", "pic_dev.h"]:
        with open(os.path.join(ROOT, "paper_1503_00276_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    if rec.get("source_sha256") != h.hexdigest() or rec.get("workload_name") != wl.name:
        return None
    for e in rec.get("layouts", []):
        if (list(e["tile"]) == list(info.tile)[:wl.ndim] and e["sort_interval"] == info.sort_interval
                and e["chunk"] == info.chunk):
            kib = e["fetch_kib_per_dispatch"] * rec["fetch_scale"] + e["write_kib_per_dispatch"] * rec["write_scale"]
            return kib * 1024.0 / kernel_avg_s / 1e9
    return None


def algorithmic_bytes(n, ndim, ncell):
    """Algorithmic HBM bytes of one step's particle kernel for n particles on
    ncell cells (see bytes_per_push)."""
    particle = (4 + 4 * ndim + 12 + 4) + (4 + 4 * ndim + 12)
    return n * particle + 36.0 * ncell


def timed_steps(sim, stream, steps):
    """Seconds for 'steps' steps: max of the wall clock and HIP events on the stream."""
    import torch

    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev0.record(stream)
    sim.step(steps)
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    sim.sync()
    return max(wall, ev0.elapsed_time(ev1) / 1000.0)


def run_batched(args, pic, stream):
    """The batched scan against the same instances run plain one after another,
    each plain run with the layout the batch's autotuner gave that instance."""
    from paper_1503_00276_amd import workloads as W

    log(f"batched leg: generating {args.batch_instances} instances")
    wls = W.workload4(ninst=args.batch_instances, steps=args.batch_steps)
    cfgs = [pic.Config(ndim=2, nx=wl.nx, dx=wl.dx, dt=wl.dt, shape_order=wl.order, ion_density=wl.ion_density)
            for wl in wls]
    ntot = sum(wl.n for wl in wls)
    batch = pic.PicBatch(cfgs, stream=stream)
    log(f"batched leg: loading {ntot} particles")
    for k, wl in enumerate(wls):
        batch.load_particles(k, wl.x, wl.u, wl.w, rqm=wl.rqm)
    batch.step(args.warmup)
    batch.sync()
    tune = None
    if args.tune_steps > 0:
        log("batched leg: autotune")
        tune = batch.autotune(trial_steps=args.tune_steps)
        batch.step(args.warmup)
        batch.sync()
    K = args.batch_steps
    log(f"batched leg: timing {K} steps")
    t_batch = timed_steps(batch, stream, K)
    batch.profile(2)
    batch.step(args.profile_steps)
    kt = batch.kernel_times()
    batch.profile(0)
    batch.sync()
    gpd_avg_s = kt["particle"][0] / max(kt["particle"][1], 1) / 1000.0
    infos = [batch.info(k) for k in range(len(wls))]
    batch.close()
    abytes = sum(algorithmic_bytes(wl.n, 2, wl.ncell) for wl in wls)

    log("batched leg: the same instances plain, one after another")
    t_plain = 0.0
    for k, wl in enumerate(wls):
        inf = infos[k]
        cfg = pic.Config(ndim=2, nx=wl.nx, dx=wl.dx, dt=wl.dt, shape_order=wl.order, ion_density=wl.ion_density,
                         tile=tuple(inf.tile), sort_interval=inf.sort_interval, chunk=inf.chunk)
        sim = pic.Pic(cfg, stream=stream)
        sim.load_particles(wl.x, wl.u, wl.w, rqm=wl.rqm)
        sim.step(args.warmup)
        sim.sync()
        t_plain += timed_steps(sim, stream, K)
        sim.close()
    v_batch = ntot * K / t_batch
    v_plain = ntot * K / t_plain
    return {
        "workload": f"2d3v_thermal_scan_{len(wls)}_instances",
        "instances": len(wls),
        "particles": ntot,
        "steps": K,
        "value": v_batch,
        "unit": "particle pushes/s",
        "ms_per_step": t_batch * 1000.0 / K,
        "plain_value": v_plain,
        "plain_ms_per_step": t_plain * 1000.0 / K,
        "batched_over_plain": v_batch / v_plain,
        "autotune": tune,
        "sort_interval": int(infos[0].sort_interval),
        "roofline": {
            "bound": "hbm",
            "achieved": abytes / gpd_avg_s / 1e9,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": abytes / gpd_avg_s / 1e9 / HBM_PEAK_GBS,
            "traffic": None,
            "kernel": "gpd_kernel, all instances in one launch per shape order",
            "kernel_avg_us": gpd_avg_s * 1e6,
            "kernel_pushes_per_s": ntot / gpd_avg_s,
        },
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", default="lwfa2d")
    ap.add_argument("--profile-steps", type=int, default=48)  # whole cycles of every sort interval searched
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample", type=int, default=2_097_152)
    ap.add_argument("--tune-steps", type=int, default=24,
                    help="steps the autotuner times per candidate layout, rounded up to whole sort "
                         "cycles (0: no autotune); 24 holds whole cycles of every interval searched")
    ap.add_argument("--tune-after", type=int, default=100,
                    help="untimed steps run before the autotuner, so it tunes the developed state")
    ap.add_argument("--tile", type=int, nargs="+", default=None, help="tile extents (default: automatic)")
    ap.add_argument("--chunk", type=int, default=0)
    ap.add_argument("--sort-interval", type=int, default=0)
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--only-batched", action="store_true",
                    help="run only the batched leg and print its record (for profiling)")
    ap.add_argument("--batch-instances", type=int, default=64)
    ap.add_argument("--batch-steps", type=int, default=200)
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="also run a plain device copy of this many MiB (counter calibration)")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on exactly one GPU: the library has no multi-GPU path; use --gpus 1",
              file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_1503_00276_amd import pic

    assert torch.cuda.is_available(), "no GPU visible"
    torch.cuda.set_device(0)
    stream = torch.cuda.Stream()  # a non-default stream so the library can capture graphs on it
    if args.only_batched:
        print(json.dumps(run_batched(args, pic, stream)), flush=True)
        return

    log(f"generating workload {args.workload}")
    wl = make_workload(args.workload)
    cfg = pic.Config(ndim=wl.ndim, nx=wl.nx, dx=wl.dx, dt=wl.dt, shape_order=wl.order,
                     ion_density=wl.ion_density, tile=tuple((args.tile or []) + [0] * (3 - len(args.tile or []))),
                     chunk=args.chunk, sort_interval=args.sort_interval)
    sim = pic.Pic(cfg, stream=stream)
    log(f"loading {wl.n} particles")
    sim.load_particles(wl.x, wl.u, wl.w, rqm=wl.rqm)
    if wl.E is not None:
        sim.load_fields(wl.E, wl.B)
    log(f"warmup {args.warmup} steps")
    sim.step(args.warmup)
    sim.sync()
    tune = None
    if args.tune_steps > 0:
        # tuned on a developed state (the loaded state of a driven plasma is
        # quieter than the run it starts: the wake, its density spikes and the
        # face crossings come later)
        sim.step(args.tune_after)
        log("autotune")
        tune = sim.autotune(trial_steps=args.tune_steps)
        sim.step(args.warmup)
        sim.sync()
    info = sim.info()

    log(f"timing {args.steps} steps")
    elapsed = timed_steps(sim, stream, args.steps)
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

    sim.close()
    batched = None
    if not args.no_batched:
        batched = run_batched(args, pic, stream)

    cpu = None
    if not args.no_cpu_baseline:
        log("timing the CPU oracle baseline")
        cpu = cpu_baseline(wl, args.cpu_sample)

    out = {
        "metric": "particle pushes/sec (gather+push+deposit) and % HBM roofline, plain vs batched, 1 GPU",
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
            "chunk": info.chunk,
            "slack": info.slack,
            "autotune": tune,
            "rebins_done": int(counts[2]),
            "rebin_checks": int(counts[3]),
        },
        "roofline": {
            "bound": "hbm",
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": measured_traffic(wl, info, gpd_avg_s),
            "kernel": "gpd_kernel (fused gather+push+deposit)",
            "bytes_per_push": bpp,
            "kernel_avg_us": gpd_avg_s * 1e6,
            "kernel_pushes_per_s": wl.n / gpd_avg_s,
        },
        "kernel_times_ms_per_step": {k: v[0] / max(v[1], 1) for k, v in kt.items()},
        "batched": batched,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
