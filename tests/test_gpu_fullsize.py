"""Parity at the full sizes of the five workloads, in the launch
configuration the benchmark uses (autotuned layout where the benchmark tunes),
through the C ABI.

Where the oracle can step every particle (workloads 1, 2 and the 64^3
sub-run) every particle, current and field value is compared; at the 3D full
sizes a random sample of particles is stepped one by one and the current and
fields are compared inside a sub-box whose particles the oracle steps in full
(tests/parity.py: sampled_step_parity)."""
import numpy as np
import pytest

from parity import POS_TOL, MOM_TOL, J_TOL, F_TOL, oracle_grid, sampled_step_parity, step_parity

pytestmark = pytest.mark.gpu


def _pic():
    from paper_1503_00276_amd import pic

    return pic


def _sim(pic, wl, **kw):
    cfg = pic.Config(ndim=wl.ndim, nx=wl.nx, dx=wl.dx, dt=wl.dt, shape_order=wl.order,
                     ion_density=wl.ion_density, **kw)
    sim = pic.Pic(cfg)
    sim.load_particles(wl.x, wl.u, wl.w, rqm=wl.rqm)
    if wl.E is not None:
        sim.load_fields(wl.E, wl.B)
    return cfg, sim


def _check(err, what):
    print(what, {k: float(v) for k, v in err.items()}, flush=True)
    assert err["pos"] <= POS_TOL and err["mom"] <= MOM_TOL, (what, err)
    assert err["J"] <= J_TOL, (what, err)
    assert err["E"] <= F_TOL and err["B"] <= F_TOL, (what, err)


@pytest.mark.parametrize("ndim,nx,dx,dt", [(2, (4096, 2048), (0.05, 0.2), 0.04), (3, (512, 256, 256), (0.05,) * 3, 0.02)])
def test_yee_full_grid_parity_large(orc, ndim, nx, dx, dt):
    """The field step alone on grids far larger than the workgroups the GPU
    holds at once (tens of thousands of Yee tiles): every E and B value
    against the oracle's FP64 solve.  A tile that read a halo node already
    advanced by a neighbouring workgroup would show here."""
    pic = _pic()
    cfg = pic.Config(ndim=ndim, nx=nx, dx=dx, dt=dt, shape_order=1)
    sim = pic.Pic(cfg)
    rng = np.random.default_rng(11)
    n = cfg.ncell
    E0 = rng.normal(0, 1, (3, n))
    B0 = rng.normal(0, 1, (3, n))
    sim.load_fields(E0, B0)
    g = oracle_grid(orc, cfg)
    E, B = sim.fields()  # FP32-rounded start, as the GPU holds it
    for k in range(2):
        Bh = orc.yee_b(g, E, B, 0.5 * dt)
        En = orc.yee_e(g, E, Bh, np.zeros((3, n)), dt)
        Bn = orc.yee_b(g, En, Bh, 0.5 * dt)
        sim.step(1)
        Eg, Bg = sim.fields()
        eE = np.abs(Eg - En).max() / np.abs(En).max()
        eB = np.abs(Bg - Bn).max() / np.abs(Bn).max()
        print("yee", ndim, k, eE, eB, flush=True)
        assert eE <= F_TOL and eB <= F_TOL, (k, eE, eB)
        E, B = Eg, Bg
    sim.close()


def test_thermal_64x64_full_parity_and_energy_history(orc):
    """Workload 1 (65,536 electrons, CIC): every particle per step, and the
    energy history of 100 steps against the oracle's FP64 run (statistical:
    FP32 and FP64 trajectories part ways, the field and kinetic energies do
    not, within 1%)."""
    from paper_1503_00276_amd import workloads as W

    pic = _pic()
    wl = W.workload1()
    cfg, sim = _sim(pic, wl)
    for k in range(2):
        _check(step_parity(orc, sim, cfg), f"cfg1 step {k}")
    sim.close()
    cfg, sim = _sim(pic, wl)
    g = oracle_grid(orc, cfg)
    x, u, w = wl.x, wl.u, wl.w
    E = np.zeros((3, wl.ncell))
    B = np.zeros((3, wl.ncell))
    ref, gpu = [], []
    for n in range(100):
        r = orc.step(g, x, u, w, -1.0, E, B)
        x, u, E, B = r.x, r.u, r.E, r.B
        fe = orc.field_energy(g, E, B)
        ke = orc.particle_moments(g, u, w, -1.0)[0]
        ref.append((fe[0] + fe[1], ke))
        sim.step(1)
        en = sim.energy()
        gpu.append((en[0] + en[1], en[2]))
    ref, gpu = np.array(ref), np.array(gpu)
    scale = ref[:, 1].max()
    assert np.abs(gpu[:, 1] - ref[:, 1]).max() <= 1e-2 * scale
    assert np.abs(gpu[:, 0] - ref[:, 0]).max() <= 1e-2 * max(ref[:, 0].max(), 1e-3 * scale)
    sim.close()


@pytest.mark.parametrize("layout", [None, (32, 8, 8, 1024, 45), (32, 8, 6, 1024, 112), (32, 8, 12, 1024, 118)],
                         ids=["autotuned", "32x8_si8_chunk1024", "32x8_si6_chunk1024", "bench_32x8_si12_chunk1024"])
def test_lwfa_full_size_parity_in_bench_layout(orc, layout):
    """Workload 2 (2,097,152 electrons, quadratic, laser): the autotuned
    layout, fixed 32x8 layouts with sort intervals 8 and 6, and the
    benchmark's layout (32x8 tiles, sort interval 12, chunk 1024) at the
    benchmark's state (it times from step 111 on; the steps compared are
    the last two of a sort cycle, where the staged halo is widest: 113-114
    at interval 6, 119-120 at interval 12); then every particle, current
    and field value for two steps."""
    from paper_1503_00276_amd import workloads as W

    pic = _pic()
    wl = W.workload2()
    if layout is None:
        cfg, sim = _sim(pic, wl)
        tune = sim.autotune(trial_steps=4)
        nsteps = 40
    else:
        cfg, sim = _sim(pic, wl, tile=layout[:2], sort_interval=layout[2], chunk=layout[3])
        tune = None
        nsteps = layout[4]
    info = sim.info()
    print("layout", list(info.tile), info.sort_interval, info.chunk, tune, flush=True)
    sim.step(nsteps)
    for k in range(2):
        _check(step_parity(orc, sim, cfg), f"cfg2 step {nsteps + 1 + k}")
    assert sim.counts()[2] > 0  # rebins happened
    sim.close()


def test_beam3d_full_size_sampled_parity(orc):
    """Workload 3 (34,603,008 particles, 256x128x128, quadratic): sampled
    particles, and current and fields in a sub-box around the beam."""
    from paper_1503_00276_amd import workloads as W

    pic = _pic()
    wl = W.workload3()
    cfg, sim = _sim(pic, wl)
    sim.step(2)
    c = (60, 64, 64)  # beam centre in cells
    err = sampled_step_parity(orc, sim, cfg, 20000, (c[0] - 24, c[1] - 8, c[2] - 8), (c[0] + 24, c[1] + 8, c[2] + 8))
    _check(err, "cfg3")
    assert err["nbox"] > 100000
    sim.close()


def test_cubic3d_subrun_full_parity(orc):
    """Workload 5's 64^3 sub-run (1,048,576 electrons, cubic): every particle
    of a 20,000 sample, and current and fields of a 16^3 sub-box."""
    from paper_1503_00276_amd import workloads as W

    pic = _pic()
    wl = W.workload5_sub()
    cfg, sim = _sim(pic, wl)
    sim.step(3)
    _check(sampled_step_parity(orc, sim, cfg, 20000, (8, 8, 8), (24, 24, 24)), "cfg5 sub-run")
    sim.close()


def _golden_energy():
    import os

    path = os.path.join(os.path.dirname(__file__), "golden", "cubic3d_64_energy.txt")
    rows = [line.split() for line in open(path) if line.strip() and not line.startswith("#")]
    return np.array([[float(v) for v in r[1:]] for r in rows])


@pytest.mark.parametrize("layout", [(8, 4, 4, 1, 768), (4, 4, 4, 1, 512)],
                         ids=["bench_8x4x4_si1_chunk768", "4x4x4_si1_chunk512"])
def test_cubic3d_subrun_energy_history_in_bench_layout(layout):
    """Workload 5's 64^3 sub-run in the benchmark's layout of the full
    workload (8x4x4 tiles, sort interval 1, chunk 768; and 4x4x4 tiles, the
    fixed-stride variant of the kernel): the field and
    kinetic energies of 100 FP32 steps against the FP64 oracle's history
    (tests/golden/cubic3d_64_energy.txt, written by make_cubic_sub_energy.py
    from the oracle alone).  W_E and W_B grow from the thermal noise and
    are compared within 1 % of their own value from step 5 on; W_K moves by
    about 1 % over the run, and its change is compared within 1 %."""
    from paper_1503_00276_amd import workloads as W

    pic = _pic()
    ref = _golden_energy()
    assert ref.shape == (100, 3)
    wl = W.workload5_sub()
    cfg, sim = _sim(pic, wl, tile=layout[:3], sort_interval=layout[3], chunk=layout[4])
    gpu = []
    for n in range(100):
        sim.step(1)
        en = sim.energy()
        gpu.append((en[0], en[1], en[2]))
    gpu = np.array(gpu)
    print("W_E", gpu[[4, 49, 99], 0], ref[[4, 49, 99], 0], flush=True)
    print("W_B", gpu[[4, 49, 99], 1], ref[[4, 49, 99], 1], flush=True)
    print("W_K", gpu[[4, 49, 99], 2], ref[[4, 49, 99], 2], flush=True)
    assert np.abs(gpu[4:, 0] / ref[4:, 0] - 1).max() <= 1e-2
    assert np.abs(gpu[4:, 1] / ref[4:, 1] - 1).max() <= 1e-2
    dk = np.abs(ref[:, 2] - ref[0, 2]).max()
    assert np.abs(gpu[:, 2] - ref[:, 2]).max() <= 1e-2 * dk + 1e-6 * ref[:, 2].max()
    assert sim.counts()[0] == 100
    sim.close()


@pytest.mark.parametrize("layout", [None, (8, 4, 4, 1, 768), (4, 4, 4, 1, 512)],
                         ids=["defaults", "bench_8x4x4_si1_chunk768", "4x4x4_si1_chunk512"])
def test_cubic3d_full_size_sampled_parity(orc, layout):
    """Workload 5 at full size (134,217,728 electrons, 512x256x256, cubic):
    with the library's defaults two steps in, and in the benchmark's layout
    (8x4x4 tiles, sort interval 1, chunk 768; also 4x4x4 tiles, the
    fixed-stride variant) at the benchmark's state (it
    times from step 111 on, after the work items have been re-interleaved
    and particles have strayed from their tiles for a hundred steps)."""
    from paper_1503_00276_amd import workloads as W

    pic = _pic()
    wl = W.workload5()
    if layout is None:
        cfg, sim = _sim(pic, wl)
        nsteps = 2
    else:
        cfg, sim = _sim(pic, wl, tile=layout[:3], sort_interval=layout[3], chunk=layout[4])
        nsteps = 111
    del wl
    sim.step(nsteps)
    print("layout", list(sim.info().tile), sim.info().sort_interval, sim.info().chunk, flush=True)
    _check(sampled_step_parity(orc, sim, cfg, 20000, (200, 100, 100), (216, 116, 116)), f"cfg5 full, step {nsteps + 1}")
    sim.close()


@pytest.mark.parametrize("tuned", [False, True], ids=["bench_layout", "autotuned"])
def test_batched_scan_parity(tuned):
    """Workload 4 (64 instances, 62 M particles) in the benchmark's batched
    layout (the library's tiles, sort interval 4, chunk 2048) at the state it
    times from (after 10 steps), and autotuned: every particle of the four
    smallest instances and a sample of two large ones, one step each,
    against the oracle."""
    import oracle as orc
    from paper_1503_00276_amd import workloads as W

    pic = _pic()
    wls = W.workload4()
    lay = {} if tuned else {"sort_interval": 4, "chunk": 2048}
    cfgs = [pic.Config(ndim=2, nx=wl.nx, dx=wl.dx, dt=wl.dt, shape_order=wl.order, ion_density=wl.ion_density, **lay)
            for wl in wls]
    batch = pic.PicBatch(cfgs)
    for k, wl in enumerate(wls):
        batch.load_particles(k, wl.x, wl.u, wl.w, rqm=wl.rqm)
    if tuned:
        batch.autotune(trial_steps=4)
        batch.step(5)
    else:
        batch.step(10)
    sizes = np.array([wl.n for wl in wls])
    pick = list(np.argsort(sizes)[:4]) + list(np.argsort(sizes)[-2:])
    states = {}
    for k in pick:
        x, u, w = batch.state(k)
        E, B = batch.fields(k)
        states[k] = (x, u, w, E, B)
    batch.step(1)
    rng = np.random.default_rng(3)
    for k in pick:
        x, u, w, E, B = states[k]
        g = oracle_grid(orc, cfgs[k])
        sel = np.arange(len(w)) if len(w) <= 100000 else rng.choice(len(w), 20000, replace=False)
        ref = orc.step(g, x[sel], u[sel], w[sel], -1.0, E, B)
        x1, u1, _ = batch.state(k)
        from parity import compare_state

        ex, eu = compare_state(cfgs[k], x1[sel], u1[sel], ref.x, ref.u)
        print("instance", k, wls[k].nx, len(w), ex, eu, flush=True)
        assert ex <= POS_TOL and eu <= MOM_TOL, (k, ex, eu)
        if len(sel) == len(w):
            J = batch.current(k)
            assert np.abs(J - ref.J).max() <= J_TOL * np.abs(ref.J).max(), k
    batch.close()
