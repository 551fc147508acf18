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
                    order=cfg.shape_order, xmin=tuple(cfg.xmin), e0=tuple(cfg.e0), b0=tuple(cfg.b0))


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
