"""GPU parity: one step of the HIP path against one step of the FP64 oracle,
element by element, from the same (GPU-exported) state.  All calls go
through the C ABI of libpic.so."""
import numpy as np
import pytest

from parity import POS_TOL, MOM_TOL, J_TOL, F_TOL, step_parity

pytestmark = pytest.mark.gpu


def _pic():
    from paper_1503_00276_amd import pic

    return pic


def _thermal(ndim, nx, dx, ppc, uth, seed):
    rng = np.random.default_rng(seed)
    ncell = int(np.prod(nx))
    cells = np.repeat(np.arange(ncell), ppc)
    idx = np.stack(np.unravel_index(cells, tuple(reversed(nx)))[::-1], axis=1)
    x = (idx + rng.random((len(cells), ndim))) * np.asarray(dx)
    u = rng.normal(0, uth, size=(len(cells), 3))
    w = np.full(len(cells), -1.0 / ppc)
    return x, u, w


CASES = [
    # ndim, nx, dx, dt, order, ppc, uth, tile
    (2, (32, 24), (0.2, 0.25), 0.1, 1, 4, 0.05, (8, 8)),
    (2, (36, 20), (0.2, 0.2), 0.1, 2, 3, 0.3, (16, 8)),     # ragged tiles
    (2, (24, 24), (0.2, 0.2), 0.1, 3, 3, 0.5, (8, 8)),
    (3, (16, 12, 10), (0.2, 0.2, 0.25), 0.08, 1, 2, 0.2, (8, 6, 5)),
    (3, (12, 12, 12), (0.2, 0.2, 0.2), 0.08, 2, 2, 0.3, (4, 4, 4)),
    (3, (12, 10, 12), (0.2, 0.2, 0.2), 0.08, 3, 2, 0.3, (4, 5, 4)),
]


# 2D boxes take the two-phase kernel with the library's chunk, the one-phase
# kernel with work items of more than 1024 particles (chunk 2048)
STEP_CASES = [(c, 0) for c in CASES] + [(c, 2048) for c in CASES if c[0] == 2]


@pytest.mark.parametrize("case,chunk", STEP_CASES,
                         ids=lambda c: f"{c[0]}d_o{c[4]}_{'x'.join(map(str, c[1]))}" if isinstance(c, tuple) else f"chunk{c}")
def test_step_parity(orc, case, chunk):
    pic = _pic()
    ndim, nx, dx, dt, order, ppc, uth, tile = case
    x, u, w = _thermal(ndim, nx, dx, ppc, uth, 11 + order + 10 * ndim)
    cfg = pic.Config(ndim=ndim, nx=nx, dx=dx, dt=dt, shape_order=order, tile=tile, sort_interval=2,
                     ion_density=1.0, chunk=chunk)
    sim = pic.Pic(cfg)
    sim.load_particles(x, u, w, rqm=-1.0)
    rng = np.random.default_rng(5)
    ncell = int(np.prod(nx))
    sim.load_fields(rng.normal(0, 0.05, (3, ncell)), rng.normal(0, 0.05, (3, ncell)))
    print(f"case {case}", flush=True)
    for k in range(3):  # several steps, crossing a rebin check
        err = step_parity(orc, sim, cfg)
        print(k, err, flush=True)
        assert err["pos"] <= POS_TOL
        assert err["mom"] <= MOM_TOL
        assert err["J"] <= J_TOL
        assert err["E"] <= F_TOL and err["B"] <= F_TOL
    sim.sync()


@pytest.mark.parametrize("ndim,order", [(2, 2), (3, 1)])
def test_fixed64_parity_and_bitwise_determinism(orc, ndim, order):
    """The int64 fold gives the same parity and bitwise identical results on
    a re-run from the same state (order-independent current)."""
    pic = _pic()
    nx = (24, 16) if ndim == 2 else (12, 10, 8)
    dx = (0.2,) * ndim
    tile = (8, 8) if ndim == 2 else (6, 5, 4)
    x, u, w = _thermal(ndim, nx, dx, 3, 0.2, 77 + ndim)
    outs = []
    for rep in range(2):
        cfg = pic.Config(ndim=ndim, nx=nx, dx=dx, dt=0.08, shape_order=order, tile=tile, sort_interval=2,
                         accumulator=pic.PIC_ACC_FIXED64, ion_density=1.0)
        sim = pic.Pic(cfg)
        sim.load_particles(x, u, w, rqm=-1.0)
        if rep == 0:
            err = step_parity(orc, sim, cfg)
            assert err["pos"] <= POS_TOL and err["mom"] <= MOM_TOL and err["J"] <= J_TOL, err
            sim.step(5)
        else:
            sim.step(6)
        xs, us, _ = sim.state()
        outs.append((xs, us, sim.current(), sim.fields()[0]))
        sim.close()
    for a, b in zip(outs[0], outs[1]):
        assert np.array_equal(a, b)


@pytest.mark.parametrize("ndim,nx,tile", [(2, (40, 24), (8, 8)), (3, (16, 12, 10), (8, 6, 5))])
def test_tristan_step_parity(orc, ndim, nx, tile):
    """The TRISTAN (Villasenor-Buneman) deposit, linear shape: hot particles
    cross faces every step; per-step parity against the oracle's path cut."""
    pic = _pic()
    dx = (0.2, 0.25, 0.2)[:ndim]
    x, u, w = _thermal(ndim, nx, dx, 3, 0.6, 5 + ndim)
    cfg = pic.Config(ndim=ndim, nx=nx, dx=dx, dt=0.08, shape_order=1, tile=tile, sort_interval=2,
                     ion_density=1.0, deposit=pic.PIC_DEPOSIT_TRISTAN)
    sim = pic.Pic(cfg)
    sim.load_particles(x, u, w, rqm=-1.0)
    rng = np.random.default_rng(8)
    ncell = int(np.prod(nx))
    sim.load_fields(rng.normal(0, 0.05, (3, ncell)), rng.normal(0, 0.05, (3, ncell)))
    for k in range(3):
        err = step_parity(orc, sim, cfg)
        print(k, err, flush=True)
        assert err["pos"] <= POS_TOL and err["mom"] <= MOM_TOL
        assert err["J"] <= J_TOL
        assert err["E"] <= F_TOL and err["B"] <= F_TOL
    # charge conservation measured on the GPU (FP64 residual of the FP32 step)
    rho_e = sim.rho() - 1.0
    sim.rho_snapshot()
    sim.step(1)
    C = sim.charge_residual()
    assert np.abs(C).max() * cfg.dt <= 1e-6 * np.abs(rho_e).max()
    sim.close()


@pytest.mark.parametrize("ndim,order,acc", [(2, 2, 0), (2, 1, 2), (3, 1, 0)])
def test_smoothed_current_step_parity(orc, ndim, order, acc):
    """Current smoothing between the deposit and the field solve: binomial
    and compensator passes per axis, on the FP32 and the int64 accumulator;
    the smoothed current, E and B against the oracle."""
    pic = _pic()
    nx = (36, 20) if ndim == 2 else (16, 12, 10)
    tile = (12, 10) if ndim == 2 else (8, 6, 5)
    dx = (0.2, 0.25, 0.2)[:ndim]
    smooth = [[(1, 2, 1), (1, 2, 1), (-1, 6, -1)], [(1, 2, 1)], [(1, 2, 1), (1, 2, 1)]][:ndim]
    x, u, w = _thermal(ndim, nx, dx, 3, 0.3, 17 + ndim)
    cfg = pic.Config(ndim=ndim, nx=nx, dx=dx, dt=0.08, shape_order=order, tile=tile, sort_interval=2,
                     ion_density=1.0, accumulator=acc, smooth=smooth)
    sim = pic.Pic(cfg)
    sim.load_particles(x, u, w, rqm=-1.0)
    for k in range(3):
        err = step_parity(orc, sim, cfg)
        print(k, err, flush=True)
        assert err["pos"] <= POS_TOL and err["mom"] <= MOM_TOL
        assert err["J"] <= J_TOL
        assert err["E"] <= F_TOL and err["B"] <= F_TOL
    sim.close()


@pytest.mark.parametrize("order", [1, 2, 3])
def test_dense_item_current_parity(orc, order):
    """A work item near the largest size the two-phase 3D kernel takes (764
    particles of one 4x4x4 tile, chunk 768), 700 of them in one cell moving
    together at 0.9 c: nodes of the item's 32-bit current tile sum hundreds
    of near-maximal contributions of one sign, the case its fixed-point
    range is sized for.  Every cell also holds one background particle.
    The step matches the oracle within the stated tolerances, three steps
    in a row."""
    pic = _pic()
    nx, dx, dt = (8, 8, 8), (0.2, 0.2, 0.2), 0.08
    rng = np.random.default_rng(40 + order)
    ncell = 512
    idx = np.stack(np.unravel_index(np.arange(ncell), (8, 8, 8))[::-1], axis=1)
    xb = (idx + rng.random((ncell, 3))) * 0.2
    ub = rng.normal(0, 0.1, size=(ncell, 3))
    xd = (np.array([1, 2, 1]) + 0.3 + 0.4 * rng.random((700, 3))) * 0.2
    ud = np.tile([1.6, 1.2, 0.8], (700, 1)) * (1 + 1e-3 * rng.standard_normal((700, 1)))
    x = np.concatenate([xb, xd])
    u = np.concatenate([ub, ud])
    w = np.full(len(x), -1.0 / 4)
    cfg = pic.Config(ndim=3, nx=nx, dx=dx, dt=dt, shape_order=order, tile=(4, 4, 4), sort_interval=1,
                     chunk=768, ion_density=1.0)
    sim = pic.Pic(cfg)
    sim.load_particles(x, u, w, rqm=-1.0)
    print(f"dense item, order {order}", flush=True)
    for k in range(3):
        err = step_parity(orc, sim, cfg)
        print(k, err, flush=True)
        assert err["pos"] <= POS_TOL
        assert err["mom"] <= MOM_TOL
        assert err["J"] <= J_TOL
        assert err["E"] <= F_TOL and err["B"] <= F_TOL
    sim.sync()


@pytest.mark.parametrize("order", [1, 2, 3])
def test_dense_item_current_parity_2d(orc, order):
    """The two-phase 2D kernel at its largest work item (1024 particles of
    one 8x8 tile): 960 particles in one cell moving together at 0.9 c with
    out-of-plane motion, plus one background particle per cell, so that
    nodes of the item's 32-bit current tile sum hundreds of near-maximal
    contributions of one sign in all three components.  The step matches
    the oracle within the stated tolerances, three steps in a row."""
    pic = _pic()
    nx, dx, dt = (16, 16), (0.2, 0.2), 0.08
    rng = np.random.default_rng(60 + order)
    ncell = 256
    idx = np.stack(np.unravel_index(np.arange(ncell), (16, 16))[::-1], axis=1)
    xb = (idx + rng.random((ncell, 2))) * 0.2
    ub = rng.normal(0, 0.1, size=(ncell, 3))
    xd = (np.array([2, 3]) + 0.3 + 0.4 * rng.random((960, 2))) * 0.2
    ud = np.tile([1.6, 1.0, 0.8], (960, 1)) * (1 + 1e-3 * rng.standard_normal((960, 1)))
    x = np.concatenate([xb, xd])
    u = np.concatenate([ub, ud])
    w = np.full(len(x), -1.0 / 4)
    cfg = pic.Config(ndim=2, nx=nx, dx=dx, dt=dt, shape_order=order, tile=(8, 8), sort_interval=1,
                     ion_density=1.0)
    sim = pic.Pic(cfg)
    sim.load_particles(x, u, w, rqm=-1.0)
    assert sim.info().chunk == 1024
    print(f"dense 2D item, order {order}", flush=True)
    for k in range(3):
        err = step_parity(orc, sim, cfg)
        print(k, err, flush=True)
        assert err["pos"] <= POS_TOL
        assert err["mom"] <= MOM_TOL
        assert err["J"] <= J_TOL
        assert err["E"] <= F_TOL and err["B"] <= F_TOL
    sim.sync()
