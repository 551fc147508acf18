"""Helpers shared by the GPU parity tests: one GPU step against one oracle step.

The GPU state is exported (FP32 values promoted to FP64), the oracle takes
one FP64 step from exactly that state, the GPU takes its own step, and the
results are compared element by element with the stated tolerances:
  position   |dx| / dx_d <= 1e-5 per particle (periodic distance)
  momentum   |du| <= 1e-5 * max(|u_p|, u_rms)
  current    max |dJ| <= 1e-5 * max |J|
  fields     max |dF| <= 1e-5 * max |F|   (E, B after the step)
"""
from __future__ import annotations

import numpy as np

POS_TOL = 1e-5
MOM_TOL = 1e-5
J_TOL = 1e-5
F_TOL = 1e-5


def oracle_grid(orc, cfg):
    return orc.Grid(dim=cfg.ndim, nx=tuple(cfg.nx[:cfg.ndim]), dx=tuple(cfg.dx[:cfg.ndim]), dt=cfg.dt,
                    order=cfg.shape_order, xmin=tuple(cfg.xmin), e0=tuple(cfg.e0), b0=tuple(cfg.b0),
                    deposit=getattr(cfg, "deposit", 0), smooth=tuple(tuple(p) for p in getattr(cfg, "smooth", ())),
                    window=getattr(cfg, "move_window", 0), inject_ppc=tuple(getattr(cfg, "inject_ppc", (1, 1, 1))),
                    inject_w=getattr(cfg, "inject_w", 0.0), inject_uth=getattr(cfg, "inject_uth", 0.0),
                    inject_seed=getattr(cfg, "inject_seed", 0), cyl=int(getattr(cfg, "geometry", 0) == 1))


def periodic_dx(a, b, L):
    d = a - b
    return d - L * np.round(d / L)


def compare_state(cfg, x_gpu, u_gpu, x_ref, u_ref):
    L = np.asarray(cfg.nx[:cfg.ndim]) * np.asarray(cfg.dx[:cfg.ndim])
    dx = np.asarray(cfg.dx[:cfg.ndim])
    ex = np.abs(periodic_dx(x_gpu, x_ref, L)) / dx
    urms = np.sqrt(np.mean(np.sum(u_ref ** 2, axis=1))) if len(u_ref) else 0.0
    scale = np.maximum(np.linalg.norm(u_ref, axis=1), urms)
    scale = np.where(scale > 0, scale, 1.0)
    eu = np.linalg.norm(u_gpu - u_ref, axis=1) / scale
    return (ex.max() if ex.size else 0.0), (eu.max() if eu.size else 0.0)


def rel_max(a, ref):
    m = np.abs(ref).max()
    if m == 0:
        return np.abs(a).max()
    return np.abs(a - ref).max() / m


def step_parity(orc, sim, cfg, qm=-1.0):
    """Take one step on both sides from the GPU's current state; return the errors."""
    x0, u0, w0 = sim.state()
    E0, B0 = sim.fields()
    g = oracle_grid(orc, cfg)
    ref = orc.step(g, x0, u0, w0, qm, E0, B0)
    sim.step(1)
    x1, u1, _ = sim.state()
    E1, B1 = sim.fields()
    J1 = sim.current()
    ex, eu = compare_state(cfg, x1, u1, ref.x, ref.u)
    return {
        "pos": ex,
        "mom": eu,
        "J": rel_max(J1, ref.J),
        "E": rel_max(E1, ref.E),
        "B": rel_max(B1, ref.B),
        "Jmax": np.abs(ref.J).max(),
    }


def sampled_step_parity(orc, sim, cfg, nsample, box_lo, box_hi, qm=-1.0, seed=0, margin=4):
    """Per-step parity at sizes the oracle cannot step whole: positions and
    momenta of a random sample of particles, and current and fields inside a
    sub-box (cells box_lo..box_hi, FP64 oracle fed every particle within
    'margin' cells of it, so the box interior sees all its contributions)."""
    x0, u0, w0 = sim.state()
    E0, B0 = sim.fields()
    g = oracle_grid(orc, cfg)
    d = cfg.ndim
    dx = np.asarray(cfg.dx[:d])
    nxa = np.asarray(cfg.nx[:d])
    rng = np.random.default_rng(seed)
    idx = rng.choice(len(w0), size=min(nsample, len(w0)), replace=False)
    ref_s = orc.step(g, x0[idx], u0[idx], w0[idx], qm, E0, B0)
    cell = np.floor(x0 / dx).astype(np.int64)
    lo = np.asarray(box_lo) - margin
    hi = np.asarray(box_hi) + margin
    rel = (cell - lo) % nxa
    inside = np.all(rel < (hi - lo), axis=1)
    sel = np.nonzero(inside)[0]
    ref_b = orc.step(g, x0[sel], u0[sel], w0[sel], qm, E0, B0)
    sim.step(1)
    x1, u1, _ = sim.state()
    E1, B1 = sim.fields()
    J1 = sim.current()
    ex, eu = compare_state(cfg, x1[idx], u1[idx], ref_s.x, ref_s.u)
    # interior of the box (the Yee update reaches 2 cells, the deposit 3)
    grids = np.meshgrid(*[np.arange(a + 2, b - 2) % n for a, b, n in zip(box_lo, box_hi, nxa)], indexing="ij")
    flat = np.zeros_like(grids[0])
    mul = 1
    for k in range(d):
        flat = flat + grids[k] * mul
        mul *= int(nxa[k])
    flat = flat.ravel()
    Jr = ref_b.J[:, flat]
    Jg = J1[:, flat]
    Er, Br = ref_b.E[:, flat], ref_b.B[:, flat]
    scaleJ = max(np.abs(Jr).max(), np.abs(J1).max())
    return {
        "pos": ex,
        "mom": eu,
        "J": np.abs(Jg - Jr).max() / scaleJ if scaleJ > 0 else np.abs(Jg).max(),
        "E": rel_max(E1[:, flat], Er),
        "B": rel_max(B1[:, flat], Br),
        "nbox": len(sel),
    }
