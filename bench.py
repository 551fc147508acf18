#!/usr/bin/env python3
"""Benchmark of the PIC particle step on one MI355X.

Metric: particle pushes per second (one push = gather + Boris push + advance +
charge-conserving deposit of one particle), whole step included (the Yee
field solve and the rebin checks run inside the timed region), inputs already
resident in HBM.  Headline workload (default): the 3D3V uniform thermal
plasma of 512x256x256 cells, 134,217,728 electrons, cubic shape, timed after
100 untimed steps in the layout a tile sweep of that developed state found
fastest (8x4x4 tiles, sort interval 1, chunk 768).  Further legs: the 2D3V laser wakefield
(1024x256 cells, 2,097,152 electrons, quadratic, 32x8 tiles, sort interval
12, chunk 1024: the fastest of a sweep of the developed wake, fixed so that
the parity tests and the counter records cover exactly the timed layout;
--workload lwfa2d --tune-headline autotunes it in the run), the batched scan (64 independent 2D thermal instances
of uneven grids and particle counts advanced by the batched step) against the
same instances run plain one after another, and the FP64 CPU oracle on the
host's cores.  Prints one JSON line.

  python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload cubic3d|lwfa2d|thermal2d|beam3d]
                  [--no-lwfa] [--no-batched] [--no-cpu-baseline] [--tune-steps T] [--tune-headline]
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


def _host_cpu():
    """Host CPU model and core counts as the OS reports them."""
    model = ""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:
        usable = os.cpu_count() or 1
    return {"model": model, "nproc": os.cpu_count() or 1, "usable": usable}


def _oracle_steps(job):
    """One worker of the CPU baseline: the FP64 oracle as it stands, stepped on
    its own share of the particles over its own copy of the grid; returns
    (particles, steps, seconds spent inside the oracle's step)."""
    import numpy as np
    import oracle

    dim, nx, dx, dt, order, x, u, w, qm, steps = job
    g = oracle.Grid(dim=dim, nx=nx, dx=dx, dt=dt, order=order)
    E = np.zeros((3, g.ncell))
    B = np.zeros((3, g.ncell))
    t = 0.0
    for _ in range(steps):
        t0 = time.perf_counter()
        r = oracle.step(g, x, u, w, qm, E, B)
        t += time.perf_counter() - t0
        x, u, E, B = r.x, r.u, r.E, r.B
    return len(w), steps, t


def cpu_baseline(wl, target_s=10.0, max_workers=16):
    """The FP64 oracle (as it stands, no tuning) on a bounded random sample of
    the workload's particles, on its own grid: first one thread, then one
    process per usable host core (at most max_workers), each stepping its own
    disjoint sample.  Each leg is sized to about target_s of work."""
    import multiprocessing as mp

    import numpy as np
    import oracle

    oracle.build(force=False)
    rng = np.random.default_rng(0)
    qm = 1.0 / wl.rqm
    spec = (wl.ndim, wl.nx, wl.dx, wl.dt, wl.order)

    def sample(n):
        return np.sort(rng.choice(wl.n, n, replace=False))

    # calibrate the cost per particle-step on a small sample
    n0 = min(wl.n, 4096)
    idx = sample(n0)
    _, _, t0 = _oracle_steps(spec + (wl.x[idx], wl.u[idx], wl.w[idx], qm, 1))
    per = max(t0 / n0, 1e-9)
    n1 = int(min(wl.n, max(n0, target_s / per)))
    idx = sample(n1)
    n, k, t1 = _oracle_steps(spec + (wl.x[idx], wl.u[idx], wl.w[idx], qm, 1))
    single = n * k / t1

    host = _host_cpu()
    P = max(1, min(max_workers, host["usable"]))
    share = int(min(n1, wl.n // P))
    perm = rng.permutation(wl.n)[: share * P]
    jobs = []
    for j in range(P):
        ix = np.sort(perm[j * share:(j + 1) * share])
        jobs.append(spec + (wl.x[ix], wl.u[ix], wl.w[ix], qm, 1))
    ctx = mp.get_context("spawn")  # fresh interpreters: no GPU state is inherited
    with ctx.Pool(P) as pool:
        res = pool.map(_oracle_steps, jobs, chunksize=1)
    tmax = max(r[2] for r in res)
    multi = sum(r[0] * r[1] for r in res) / tmax
    return {
        "value": multi,
        "unit": "particle pushes/s",
        "cores": P,
        "kind": "oracle",
        "sample": f"FP64 oracle step (gather, push, deposit, field solve on the {'x'.join(map(str, wl.nx))} grid) "
                  f"of random particle samples of the workload: {P} processes, each stepping its own "
                  f"{share} particles once ({tmax:.1f} s for the slowest); single thread: {n1} particles, "
                  f"{t1:.1f} s",
        "single_thread_value": single,
        "host": host,
    }


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


def _source_sha256():
    import hashlib

    h = hashlib.sha256()
    for f in ["gpd.hip", "pic_dev.h"]:
        with open(os.path.join(ROOT, "paper_1503_00276_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def batched_traffic(ninst, infos, step_s):
    """Counter-measured HBM traffic (GB/s) of the batched particle launches,
    from the committed record of the same source and the same autotuned
    layout (every instance's tile and the sort interval), else None."""
    path = os.path.join(ROOT, "profiles", f"gpd_2d3v_thermal_scan_{ninst}_instances_counters.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    layout = {"sort_interval": int(infos[0].sort_interval), "tiles": [list(i.tile)[:2] for i in infos],
              "chunks": [int(i.chunk) for i in infos]}
    if rec.get("source_sha256") != _source_sha256() or rec.get("layout") != layout:
        return None
    kib = rec["fetch_kib_per_step"] * rec["fetch_scale"] + rec["write_kib_per_step"] * rec["write_scale"]
    return kib * 1024.0 / step_s / 1e9


# Layout of the batched leg unless --batch-tune: the library's tile for each
# instance, with the chunk the batch autotuner picked for this scan and the
# fastest sort interval of a sweep of 3-12 (fixed so that runs, parity tests
# and the counter record agree).
BATCH_LAYOUT = {"sort_interval": 4, "chunk": 2048}


def run_batched(args, pic, stream):
    """The batched scan against the same instances run plain one after another,
    each plain run with the layout the batch gave that instance."""
    from paper_1503_00276_amd import workloads as W

    log(f"batched leg: generating {args.batch_instances} instances")
    wls = W.workload4(ninst=args.batch_instances, steps=args.batch_steps)
    lay = {} if args.batch_tune else BATCH_LAYOUT
    cfgs = [pic.Config(ndim=2, nx=wl.nx, dx=wl.dx, dt=wl.dt, shape_order=wl.order, ion_density=wl.ion_density,
                       sort_interval=lay.get("sort_interval", 0), chunk=lay.get("chunk", 0))
            for wl in wls]
    ntot = sum(wl.n for wl in wls)
    batch = pic.PicBatch(cfgs, stream=stream)
    log(f"batched leg: loading {ntot} particles")
    for k, wl in enumerate(wls):
        batch.load_particles(k, wl.x, wl.u, wl.w, rqm=wl.rqm)
    batch.step(args.warmup)
    batch.sync()
    tune = None
    if args.batch_tune and args.tune_steps > 0:
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
    # one launch per shape order and step; the profiling events bracket all
    # of a step's particle launches together, so gpd_avg_s is per step
    nlaunch = len({wl.order for wl in wls})
    traffic = batched_traffic(len(wls), infos, gpd_avg_s)
    if args.batch_layout_out:
        with open(args.batch_layout_out, "w") as f:
            json.dump({"sort_interval": int(infos[0].sort_interval), "tiles": [list(i.tile)[:2] for i in infos],
                       "chunks": [int(i.chunk) for i in infos]}, f)

    log("batched leg: the same instances plain, one after another")
    t_plain = 0.0
    for k, wl in enumerate(wls if not args.batch_no_plain else []):
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
    v_plain = ntot * K / t_plain if t_plain > 0 else float("nan")
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
        "layout_from": "autotuned in this run" if tune else "fixed: library tiles, sort interval 4, chunk 2048",
        "sort_interval": int(infos[0].sort_interval),
        "roofline": {
            "bound": "hbm",
            "achieved": abytes / gpd_avg_s / 1e9,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": abytes / gpd_avg_s / 1e9 / HBM_PEAK_GBS,
            "traffic": traffic,
            "kernel": "gpd_kernel, all instances in one launch per shape order",
            "launches_per_step": nlaunch,
            "kernel_avg_us": gpd_avg_s * 1e6,
            "kernel_avg_covers": "all particle launches of a step",
            "kernel_pushes_per_s": ntot / gpd_avg_s,
        },
    }


# Layouts timed when the benchmark does not tune them.  The headline's is the
# fastest of a tile sweep of its developed state (a search over 134 M
# particles re-bins them on the host for every candidate and takes minutes;
# --tune-headline runs it instead); the laser wakefield's is the fastest of a
# sweep of tiles and sort intervals of its developed wake.
DEFAULT_LAYOUT = {
    "cubic3d": {"tile": [8, 4, 4], "sort_interval": 1, "chunk": 768},
    "lwfa2d": {"tile": [32, 8], "sort_interval": 12, "chunk": 1024},
}


def counter_record(wl, info):
    """The committed rocprofv3 counter record of the particle kernel for this
    workload and layout (FETCH_SIZE, WRITE_SIZE and SQ_INSTS_VALU per
    dispatch), or None when there is none or the kernel's source changed
    since the counters were taken."""
    path = os.path.join(ROOT, "profiles", f"gpd_{wl.name}_counters.json")
    if not os.path.exists(path):
        return None, None
    rec = json.load(open(path))
    if rec.get("source_sha256") != _source_sha256() or rec.get("workload_name") != wl.name:
        return rec, None
    for e in rec.get("layouts", []):
        if (list(e["tile"]) == list(info.tile)[:wl.ndim] and e["sort_interval"] == info.sort_interval
                and e["chunk"] == info.chunk):
            return rec, e
    return rec, None


def roofline(wl, info, gpd_avg_s):
    """HBM roofline of the particle kernel (algorithmic bytes over its average
    launch time) with the counter-measured traffic and, for the kernels whose
    arithmetic bounds them, the VALU issue fraction: measured VALU wave
    instructions per launch against one wave instruction per cycle per CU
    (256 CUs at 2.4 GHz; packed FP32 is not used, so this is 78.6 TFLOP/s of
    FMA).  Where the record holds the LDS counters, also the share of the
    launch the LDS is active (SQ_LDS_IDX_ACTIVE cycles per CU over the
    launch's cycles) and the share of those cycles lost to bank conflicts."""
    bpp = bytes_per_push(wl)
    achieved = wl.n * bpp / gpd_avg_s / 1e9
    rec, e = counter_record(wl, info)
    traffic = valu = lds = None
    if e is not None:
        kib = e["fetch_kib_per_dispatch"] * rec["fetch_scale"] + e["write_kib_per_dispatch"] * rec["write_scale"]
        traffic = kib * 1024.0 / gpd_avg_s / 1e9
        if "valu_insts_per_dispatch" in e:
            issue = e["valu_insts_per_dispatch"] / gpd_avg_s
            peak = 256 * 2.4e9
            valu = {"insts_per_launch": e["valu_insts_per_dispatch"], "achieved_insts_per_s": issue,
                    "peak_insts_per_s": peak, "frac": issue / peak,
                    "insts_per_push": e["valu_insts_per_dispatch"] * 64.0 / wl.n}
        if "lds_active_cycles_per_dispatch" in e:
            cyc = 256 * 2.4e9 * gpd_avg_s
            lds = {"active_cycles_per_launch": e["lds_active_cycles_per_dispatch"],
                   "active_frac": e["lds_active_cycles_per_dispatch"] / cyc,
                   "bank_conflict_frac": e["lds_bank_conflict_cycles_per_dispatch"] / e["lds_active_cycles_per_dispatch"]}
    return {
        "bound": "hbm",
        "achieved": achieved,
        "peak": HBM_PEAK_GBS,
        "unit": "GB/s",
        "frac": achieved / HBM_PEAK_GBS,
        "traffic": traffic,
        "kernel": "gpd_kernel (fused gather+push+deposit)",
        "bytes_per_push": bpp,
        "kernel_avg_us": gpd_avg_s * 1e6,
        "kernel_pushes_per_s": wl.n / gpd_avg_s,
        "valu": valu,
        "lds": lds,
    }


def plain_leg(args, pic, stream, name, steps, layout=None, tune=True):
    """One workload on the plain single-instance path: load, untimed steps,
    optionally the autotuner, then 'steps' timed steps and a profiled run."""
    log(f"[{name}] generating")
    wl = make_workload(name)
    lay = layout or {}
    tile = list(lay.get("tile", []))
    cfg = pic.Config(ndim=wl.ndim, nx=wl.nx, dx=wl.dx, dt=wl.dt, shape_order=wl.order,
                     ion_density=wl.ion_density, tile=tuple(tile + [0] * (3 - len(tile))),
                     chunk=lay.get("chunk", 0), sort_interval=lay.get("sort_interval", 0))
    sim = pic.Pic(cfg, stream=stream)
    log(f"[{name}] loading {wl.n} particles")
    sim.load_particles(wl.x, wl.u, wl.w, rqm=wl.rqm)
    if wl.E is not None:
        sim.load_fields(wl.E, wl.B)
    sim.step(args.warmup)
    sim.sync()
    # tuned (and timed) on a developed state: the loaded state is quieter than
    # the run it starts (the wake, its density spikes, particles strayed from
    # their tiles)
    sim.step(args.tune_after)
    sim.sync()
    tuned = None
    if tune and args.tune_steps > 0:
        log(f"[{name}] autotune")
        tuned = sim.autotune(trial_steps=args.tune_steps)
        sim.step(args.warmup)
        sim.sync()
    info = sim.info()
    log(f"[{name}] timing {steps} steps")
    elapsed = timed_steps(sim, stream, steps)
    log(f"[{name}] profiling {args.profile_steps} steps")
    sim.profile(2)
    sim.step(args.profile_steps)
    kt = sim.kernel_times()
    sim.profile(0)
    sim.sync()
    gpd_avg_s = kt["particle"][0] / max(kt["particle"][1], 1) / 1000.0
    counts = sim.counts()
    # charge conservation of the benched layout, from the GPU's FP64
    # diagnostics: max|C| dt / max|rho_e| over one step
    sim.rho_snapshot()
    rho_e = sim.rho() - wl.ion_density
    sim.step(1)
    C = sim.charge_residual()
    import numpy as np

    charge_rel = float(np.abs(C).max() * wl.dt / max(np.abs(rho_e).max(), 1e-300))
    sim.close()
    rec = {
        "value": wl.n * steps / elapsed,
        "unit": "particle pushes/s",
        "ms_per_step": elapsed * 1000.0 / steps,
        "steps": steps,
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
            "lds_bytes": int(info.lds_bytes),
            "autotune": tuned,
            "layout_from": "autotuned in this run" if tuned else (
                "fixed: the fastest layout of a tile sweep of the developed state" if layout else "library defaults"),
            "rebins_done": int(counts[2]),
            "rebin_checks": int(counts[3]),
        },
        "roofline": roofline(wl, info, gpd_avg_s),
        "kernel_times_ms_per_step": {k: v[0] / max(v[1], 1) for k, v in kt.items()},
        "charge_residual_rel": charge_rel,
    }
    return rec


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--workload", default="cubic3d")
    ap.add_argument("--profile-steps", type=int, default=24)  # whole cycles of every sort interval searched
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--tune-steps", type=int, default=24,
                    help="steps the autotuner times per candidate layout, rounded up to whole sort "
                         "cycles (0: no autotune); 24 holds whole cycles of every interval searched")
    ap.add_argument("--tune-after", type=int, default=100,
                    help="untimed steps run before the autotuner (and the timing), so it tunes the "
                         "developed state")
    ap.add_argument("--tune-headline", action="store_true",
                    help="run the autotuner on the headline workload too (slow on 134 M particles)")
    ap.add_argument("--tile", type=int, nargs="+", default=None, help="headline tile extents")
    ap.add_argument("--chunk", type=int, default=0)
    ap.add_argument("--sort-interval", type=int, default=0)
    ap.add_argument("--no-lwfa", action="store_true", help="skip the 2D laser-wakefield leg")
    ap.add_argument("--lwfa-steps", type=int, default=200)
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--only-batched", action="store_true",
                    help="run only the batched leg and print its record (for profiling)")
    ap.add_argument("--batch-instances", type=int, default=64)
    ap.add_argument("--batch-steps", type=int, default=200)
    ap.add_argument("--batch-tune", action="store_true",
                    help="run the batch autotuner instead of the fixed batched layout")
    ap.add_argument("--batch-no-plain", action="store_true",
                    help="skip the plain one-after-another runs of the batched leg (counter passes)")
    ap.add_argument("--batch-layout-out", default="",
                    help="write the batched leg's autotuned layout (JSON) to this file (counter records)")
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
    if args.calib_copy_mib > 0:
        # a plain device copy of known size: the counters' calibration
        n = args.calib_copy_mib * 1024 * 1024 // 4
        a = torch.ones(n, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        del a, b
    if args.only_batched:
        print(json.dumps(run_batched(args, pic, stream)), flush=True)
        return

    layout = None
    if args.tile or args.chunk or args.sort_interval:
        layout = {"tile": args.tile or [], "chunk": args.chunk, "sort_interval": args.sort_interval}
    elif not args.tune_headline:
        layout = DEFAULT_LAYOUT.get(args.workload)
    head = plain_leg(args, pic, stream, args.workload, args.steps, layout,
                     tune=args.tune_headline or (layout is None and args.workload not in DEFAULT_LAYOUT))

    lwfa = None
    if not args.no_lwfa and args.workload != "lwfa2d":
        lwfa = plain_leg(args, pic, stream, "lwfa2d", args.lwfa_steps, DEFAULT_LAYOUT["lwfa2d"], tune=False)
    batched = None
    if not args.no_batched:
        batched = run_batched(args, pic, stream)

    cpu = None
    if not args.no_cpu_baseline:
        log("timing the CPU oracle baseline")
        cwl = make_workload("cubic3d_sub" if args.workload == "cubic3d" else args.workload)
        cpu = cpu_baseline(cwl)
        if args.workload == "cubic3d":
            cpu["sample"] += " (the 64^3 sub-run of the workload: same density, shape, cell and time step)"

    out = {
        "metric": "particle pushes/sec (gather+push+deposit) and % HBM roofline, plain vs batched, 1 GPU",
        "value": head["value"],
        "unit": "particle pushes/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": head["config"],
        "roofline": head["roofline"],
        "kernel_times_ms_per_step": head["kernel_times_ms_per_step"],
        "charge_residual_rel": head["charge_residual_rel"],
        "lwfa2d": lwfa,
        "batched": batched,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
