"""The autotuner (pic_autotune / pic_batch_autotune) through the C ABI: the
measured search leaves the simulation state untouched and changes only the
layout, so a tuned run continues bitwise like an untuned one (int64 current
fold), and the tuned layout still matches the FP64 oracle."""
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


def _snapshot(sim):
    x, u, w = sim.state()
    E, B = sim.fields()
    return [x, u, w, E, B, sim.current()]


def test_autotune_keeps_state_and_continues_bitwise():
    pic = _pic()
    nx, dx = (64, 48), (0.2, 0.2)
    cfg = pic.Config(ndim=2, nx=nx, dx=dx, dt=0.1, shape_order=2, accumulator=pic.PIC_ACC_FIXED64,
                     ion_density=1.0)
    x, u, w = _thermal(2, nx, dx, 8, 0.2, 3)
    a = pic.Pic(cfg)
    b = pic.Pic(cfg)
    for s in (a, b):
        s.load_particles(x, u, w, rqm=-1.0)
        s.step(3)
    before = _snapshot(a)
    res = a.autotune(trial_steps=4)
    print("autotune", res, "tile", list(a.info().tile), flush=True)
    assert res["candidates"] >= 3
    assert 0 < res["ms_after"] <= res["ms_before"]
    assert a.info().sort_interval == res["sort_interval"]
    assert a.info().chunk == res["chunk"]
    after = _snapshot(a)
    for p, q in zip(before, after):
        assert np.array_equal(p, q)
    assert a.counts()[0] == 3  # step count restored
    a.step(5)
    b.step(5)
    for p, q in zip(_snapshot(a), _snapshot(b)):
        assert np.array_equal(p, q)
    a.close()
    b.close()


def test_batch_autotune_keeps_results_bitwise():
    pic = _pic()
    specs = [((64, 64), 4, 1, 0.05), ((128, 64), 12, 2, 0.02), ((32, 96), 24, 2, 0.04)]
    cfgs, parts = [], []
    for k, (nx, ppc, order, uth) in enumerate(specs):
        cfgs.append(pic.Config(ndim=2, nx=nx, dx=(0.2, 0.2), dt=0.1, shape_order=order,
                               accumulator=pic.PIC_ACC_FIXED64, ion_density=1.0))
        parts.append(_thermal(2, nx, (0.2, 0.2), ppc, uth, 60 + k))
    batch = pic.PicBatch(cfgs)
    for k, p in enumerate(parts):
        batch.load_particles(k, *p, rqm=-1.0)
    res = batch.autotune(trial_steps=4)
    print("batch autotune", res, [list(batch.info(k).tile) for k in range(3)], flush=True)
    assert res["ms_after"] <= res["ms_before"]
    batch.step(7)
    for k, cfg in enumerate(cfgs):
        sim = pic.Pic(cfg)
        sim.load_particles(*parts[k], rqm=-1.0)
        sim.step(7)
        xb, ub, _ = batch.state(k)
        xs, us, _ = sim.state()
        assert np.array_equal(xb, xs) and np.array_equal(ub, us), k
        assert np.array_equal(batch.current(k), sim.current()), k
        sim.close()
    batch.close()


@pytest.mark.parametrize("ndim,order", [(2, 3), (3, 2)])
def test_tuned_layout_matches_oracle(orc, ndim, order):
    pic = _pic()
    nx = (48, 40) if ndim == 2 else (16, 16, 12)
    dx = (0.2,) * ndim
    cfg = pic.Config(ndim=ndim, nx=nx, dx=dx, dt=0.08, shape_order=order, ion_density=1.0)
    sim = pic.Pic(cfg)
    sim.load_particles(*_thermal(ndim, nx, dx, 4, 0.3, 90 + ndim), rqm=-1.0)
    rng = np.random.default_rng(9)
    n = cfg.ncell
    sim.load_fields(rng.normal(0, 0.05, (3, n)), rng.normal(0, 0.05, (3, n)))
    res = sim.autotune(trial_steps=2)
    print("tuned", res, list(sim.info().tile), flush=True)
    for _ in range(3):
        err = step_parity(orc, sim, cfg)
        assert err["pos"] <= POS_TOL and err["mom"] <= MOM_TOL and err["J"] <= J_TOL, err
        assert err["E"] <= F_TOL and err["B"] <= F_TOL, err
    sim.close()


def test_autotune_errors():
    pic = _pic()
    cfg = pic.Config(ndim=2, nx=(16, 16), dx=(0.2, 0.2), dt=0.1)
    sim = pic.Pic(cfg)
    with pytest.raises(pic.PicError) as e:
        sim.autotune(trial_steps=2)  # no particles
    assert e.value.code == pic.PIC_E_STATE
    sim.load_particles(*_thermal(2, (16, 16), (0.2, 0.2), 2, 0.1, 1), rqm=-1.0)
    with pytest.raises(pic.PicError) as e:
        sim.autotune(trial_steps=0)
    assert e.value.code == pic.PIC_E_INVALID
    sim.close()
