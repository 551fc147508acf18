"""GPU parity of the moving window (Sec. 4.5, dynamic simulation spaces): each
step of the HIP path against one step of the FP64 oracle's window step from
the same (GPU-exported) state, across steps that shift the window, remove
particles and inject the plasma of the new front column (cold, or thermal
with momenta drawn from the injected particles' ids).  Positions are
compared in window coordinates (lab x1 minus the window's travel), particles
by identity (survivors in load order, then the injected ones in injection
order), grid arrays in window order."""
import dataclasses

import numpy as np
import pytest

from parity import POS_TOL, MOM_TOL, J_TOL, F_TOL, compare_state, oracle_grid, rel_max

pytestmark = pytest.mark.gpu


def _pic():
    from paper_1503_00276_amd import pic

    return pic


def _plasma(ndim, nx, dx, ppc, uth, seed):
    rng = np.random.default_rng(seed)
    ncell = int(np.prod(nx))
    cells = np.repeat(np.arange(ncell), ppc)
    idx = np.stack(np.unravel_index(cells, tuple(reversed(nx)))[::-1], axis=1)
    x = (idx + rng.random((len(cells), ndim))) * np.asarray(dx)
    u = rng.normal(0, uth, size=(len(cells), 3))
    w = np.full(len(cells), -1.0 / ppc)
    return x, u, w


def _to_window(cfg, x_lab, shifts):
    x = x_lab - np.asarray(cfg.xmin[:cfg.ndim])
    x[:, 0] -= shifts * cfg.dx[0]
    return x


def window_step_parity(orc, sim, cfg, n, qm=-1.0, nload=0):
    """Step n -> n+1 on both sides from the GPU's state; return the errors.
    nload: particles loaded before the first step (the injected ids follow
    them, one per lattice point of every new column)."""
    g = dataclasses.replace(oracle_grid(orc, cfg), xmin=(0.0, 0.0, 0.0))
    x0, u0, w0 = sim.state()
    E0, B0 = sim.fields()
    s0 = orc.window_shifts(g, n)
    per_shift = int(np.prod(cfg.inject_ppc[:cfg.ndim])) * (int(np.prod(cfg.nx[:cfg.ndim])) // cfg.nx[0])
    ref, wref, keep = orc.step_window(g, n, _to_window(cfg, x0, s0), u0, w0, qm, E0, B0,
                                      id0=nload + s0 * per_shift)
    sim.step(1)
    x1, u1, w1 = sim.state()
    E1, B1 = sim.fields()
    J1 = sim.current()
    s1 = orc.window_shifts(g, n + 1)
    assert len(x1) == len(ref.x), (n, len(x1), len(ref.x))
    xw = _to_window(cfg, x1, s1)
    ex, eu = compare_state(cfg, xw, u1, ref.x, ref.u)
    return {
        "pos": ex,
        "mom": eu,
        "w": float(np.abs(w1 - wref).max()) if len(w1) else 0.0,
        "J": rel_max(J1, ref.J),
        "E": rel_max(E1, ref.E),
        "B": rel_max(B1, ref.B),
        "np": len(x1),
        "shift": s1 - s0,
        "removed": len(x0) - len(keep),
        "inside": bool(np.all((xw[:, 0] >= 0) & (xw[:, 0] < cfg.nx[0] * cfg.dx[0]))),
    }


CASES = [
    # ndim, nx, dx, dt, order, tile, ppc, inject_ppc, extra config
    (2, (32, 16), (0.2, 0.25), 0.1, 2, (8, 8), 4, (2, 2), {}),
    (2, (36, 20), (0.2, 0.2), 0.1, 1, (16, 8), 3, (3, 1), {}),                      # ragged tiles
    (2, (32, 16), (0.2, 0.25), 0.1, 3, (8, 8), 3, (2, 2), {"accumulator": 2}),      # int64 fold
    (2, (40, 16), (0.2, 0.2), 0.1, 1, (8, 8), 3, (2, 2), {"deposit": 1}),           # TRISTAN
    (2, (32, 16), (0.2, 0.25), 0.1, 2, (8, 8), 3, (1, 2),
     {"smooth": ((0.25, 0.5, 0.25), (-0.25, 1.5, -0.25))}),                          # smoothed current
    (3, (16, 8, 8), (0.2, 0.2, 0.2), 0.08, 1, (8, 4, 4), 2, (1, 2, 1), {}),
    (3, (12, 10, 8), (0.2, 0.2, 0.25), 0.08, 2, (4, 5, 4), 2, (2, 1, 1), {}),
    # thermal injection (Sec. 4.5: the new region initialised thermal)
    (2, (32, 16), (0.2, 0.25), 0.1, 2, (8, 8), 3, (2, 2), {"inject_uth": 0.05, "inject_seed": 150300276}),
    (3, (16, 8, 8), (0.2, 0.2, 0.2), 0.08, 3, (8, 4, 4), 2, (1, 2, 1), {"inject_uth": 0.2, "inject_seed": 7}),
]


def _ident(c):
    tag = "x".join(map(str, c[1]))
    extra = "_".join(f"{k}" for k in c[8])
    return f"{c[0]}d_o{c[4]}_{tag}" + (f"_{extra}" if extra else "")


@pytest.mark.parametrize("case", CASES, ids=_ident)
def test_window_step_parity(orc, case):
    pic = _pic()
    ndim, nx, dx, dt, order, tile, ppc, ippc, extra = case
    x, u, w = _plasma(ndim, nx, dx, ppc, 0.3, 31 + order + 10 * ndim)
    xmin = (1.0, -0.5, 0.25)[:ndim] + (0.0,) * (3 - ndim)
    kw = dict(extra)
    smooth = kw.pop("smooth", ())
    if smooth:
        kw["smooth"] = tuple(smooth if a == 0 else () for a in range(ndim))
    cfg = pic.Config(ndim=ndim, nx=nx, dx=dx, dt=dt, shape_order=order, tile=tile, sort_interval=1,
                     xmin=xmin, ion_density=1.0, move_window=1, inject_ppc=ippc + (1,) * (3 - len(ippc)),
                     inject_w=-1.0 / int(np.prod(ippc)), **kw)
    sim = pic.Pic(cfg)
    sim.load_particles(x + np.asarray(xmin[:ndim]), u, w, rqm=-1.0)
    rng = np.random.default_rng(9)
    ncell = int(np.prod(nx))
    E = rng.normal(0, 0.05, (3, ncell))
    B = rng.normal(0, 0.05, (3, ncell))
    sim.load_fields(E, B)
    print(f"case {_ident(case)}", flush=True)
    shifts = removed = 0
    for n in range(7):  # several window shifts (c dt / dx1 = 0.4 or 0.5)
        err = window_step_parity(orc, sim, cfg, n, nload=len(x))
        print(n, err, flush=True)
        assert err["inside"]
        assert err["pos"] <= POS_TOL
        assert err["mom"] <= MOM_TOL
        assert err["w"] <= 1e-7
        assert err["J"] <= J_TOL
        assert err["E"] <= F_TOL and err["B"] <= F_TOL
        shifts += err["shift"]
        removed += err["removed"]
    assert shifts >= 2 and removed > 0


@pytest.mark.parametrize("ndim", [2, 3])
def test_window_resting_plasma_stays_on_its_lab_lattice(ndim):
    """A cold plasma at rest with no fields, loaded on the injection lattice:
    over many shifts the count never changes, no field or current appears,
    and every particle stays on the lattice in the lab frame."""
    pic = _pic()
    nx = (24, 8) if ndim == 2 else (16, 8, 4)
    dx = (0.2, 0.25, 0.25)[:ndim]
    ippc = (2, 2, 1)[:ndim]
    tile = (8, 8) if ndim == 2 else (8, 4, 4)
    grids = np.meshgrid(*[np.arange(nx[d] * ippc[d]) for d in range(ndim)], indexing="ij")
    x = np.stack([(gd.ravel() + 0.5) * dx[d] / ippc[d] for d, gd in enumerate(grids)], axis=1)
    wq = -1.0 / int(np.prod(ippc))
    cfg = pic.Config(ndim=ndim, nx=nx, dx=dx, dt=0.15 if ndim == 2 else 0.1, shape_order=2, tile=tile,
                     sort_interval=1, move_window=1, inject_ppc=tuple(ippc) + (1,) * (3 - ndim), inject_w=wq,
                     ion_density=1.0)
    sim = pic.Pic(cfg)
    sim.load_particles(x, np.zeros((len(x), 3)), np.full(len(x), wq), rqm=-1.0)
    n0 = len(x)
    nsteps = 61  # n c dt / dx1 is not a whole number here
    sim.step(nsteps)
    sim.sync()
    xs, us, ws = sim.state()
    E, B = sim.fields()
    assert len(xs) == n0
    assert np.abs(E).max() == 0 and np.abs(B).max() == 0 and np.abs(sim.current()).max() == 0
    assert np.abs(us).max() == 0 and np.all(ws == np.float32(wq))
    shifts = int(np.floor(nsteps * (cfg.dt / dx[0])))  # floor(n c dt / dx1)
    assert shifts > 20
    lo = shifts * dx[0]
    assert np.all((xs[:, 0] >= lo) & (xs[:, 0] < lo + nx[0] * dx[0]))
    for d in range(ndim):
        k = xs[:, d] / (dx[d] / ippc[d]) - 0.5
        assert np.abs(k - np.round(k)).max() < 1e-4
    # every lattice point of the current window is occupied exactly once
    k0 = np.round(xs[:, 0] / (dx[0] / ippc[0]) - 0.5).astype(np.int64)
    assert k0.min() == shifts * ippc[0] and k0.max() == (shifts + nx[0]) * ippc[0] - 1
    assert len(np.unique(np.stack([np.round(xs[:, d] / (dx[d] / ippc[d]) - 0.5) for d in range(ndim)], 1),
                         axis=0)) == n0


def test_window_rejects_autotune():
    pic = _pic()
    cfg = pic.Config(ndim=2, nx=(16, 8), dx=(0.2, 0.2), dt=0.1, shape_order=1, tile=(8, 8), sort_interval=1,
                     move_window=1, inject_ppc=(1, 1, 1), inject_w=-1.0)
    sim = pic.Pic(cfg)
    x, u, w = _plasma(2, (16, 8), (0.2, 0.2), 1, 0.0, 3)
    sim.load_particles(x, u, w, rqm=-1.0)
    with pytest.raises(pic.PicError):
        sim.autotune(trial_steps=2)
