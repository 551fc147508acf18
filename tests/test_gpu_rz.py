"""GPU parity of the 2D cylindrically symmetric r-z geometry (Sec. 3.3): each
step of the HIP path against one step of the FP64 oracle from the same
(GPU-exported) state, with ring particles near the axis (shapes reaching the
mirror rows) and near the conducting wall (removed when they reach it).
Particles are compared by identity (load order without the removed ones),
grid arrays element by element."""
import numpy as np
import pytest

from parity import POS_TOL, MOM_TOL, J_TOL, F_TOL, compare_state, oracle_grid, rel_max

pytestmark = pytest.mark.gpu


def _pic():
    from paper_1503_00276_amd import pic

    return pic


def _ring_plasma(nz, nr, dz, dr, ppc, uth, seed, density=1.0):
    """ppc ring particles per cell, uniform in the cell, weights for a
    uniform density (w = n (r/dr) / ppc), a few placed near the axis and a
    few near the wall moving out."""
    rng = np.random.default_rng(seed)
    n = nz * (nr - 1) * ppc
    z = rng.random(n) * nz * dz
    r = rng.random(n) * (nr - 1) * dr
    r[: n // 10] = rng.random(n // 10) * 1.5 * dr  # near the axis
    u = rng.normal(0, uth, (n, 3))
    wall = (nr - 0.5) * dr
    k = max(4, n // 50)
    r[-k:] = wall - rng.random(k) * 0.3 * dr       # near the wall, moving out
    u[-k:, 1] = np.abs(u[-k:, 1]) + 2.0
    w = -density * (r / dr) / ppc
    return np.stack([z, r], 1), u, w


def _rz_fields(nz, nr, seed, scale=0.05):
    """Random E, B with the axis structure: E_r, B_theta zero on the axis."""
    rng = np.random.default_rng(seed)
    E = rng.normal(0, scale, (3, nr, nz))
    B = rng.normal(0, scale, (3, nr, nz))
    E[1, 0] = 0.0
    B[2, 0] = 0.0
    return E.reshape(3, -1), B.reshape(3, -1)


def rz_step_parity(orc, sim, cfg, qm=-1.0):
    g = oracle_grid(orc, cfg)
    x0, u0, w0 = sim.state()
    E0, B0 = sim.fields()
    ref, wref, keep = orc.step_cyl(g, x0, u0, w0, qm, E0, B0)
    sim.step(1)
    x1, u1, w1 = sim.state()
    E1, B1 = sim.fields()
    J1 = sim.current()
    assert len(x1) == len(ref.x), (len(x1), len(ref.x))
    ex, eu = compare_state(cfg, x1, u1, ref.x, ref.u)
    return {
        "pos": ex,
        "mom": eu,
        "w": float(np.abs(w1 - wref).max()) if len(w1) else 0.0,
        "J": rel_max(J1, ref.J),
        "E": rel_max(E1, ref.E),
        "B": rel_max(B1, ref.B),
        "removed": len(x0) - len(keep),
        "rmin": float(x1[:, 1].min()) if len(x1) else 0.0,
    }


CASES = [
    # nx (z, r), dx (dz, dr), dt, order, tile, ppc, deposit, accumulator
    ((32, 24), (0.2, 0.2), 0.1, 1, (8, 8), 4, 0, 0),
    ((32, 20), (0.2, 0.25), 0.1, 2, (16, 8), 3, 0, 0),   # ragged tiles in r
    ((24, 24), (0.2, 0.2), 0.1, 3, (8, 8), 3, 0, 2),     # cubic, int64 fold
    ((32, 24), (0.2, 0.2), 0.1, 1, (8, 8), 3, 1, 0),     # TRISTAN
]


@pytest.mark.parametrize("case", CASES, ids=lambda c: f"o{c[3]}_{c[0][0]}x{c[0][1]}_dep{c[6]}_acc{c[7]}")
def test_rz_step_parity(orc, case):
    pic = _pic()
    nx, dx, dt, order, tile, ppc, dep, acc = case
    x, u, w = _ring_plasma(nx[0], nx[1], dx[0], dx[1], ppc, 0.3, 41 + order + 7 * dep)
    cfg = pic.Config(ndim=2, nx=nx, dx=dx, dt=dt, shape_order=order, tile=tile, sort_interval=1,
                     geometry=pic.PIC_GEOM_RZ, deposit=dep, accumulator=acc, ion_density=1.0)
    sim = pic.Pic(cfg)
    sim.load_particles(x, u, w, rqm=-1.0)
    E, B = _rz_fields(nx[0], nx[1], 13)
    sim.load_fields(E, B)
    print(f"case {case}", flush=True)
    removed = 0
    for k in range(5):
        err = rz_step_parity(orc, sim, cfg)
        print(k, err, flush=True)
        assert err["pos"] <= POS_TOL
        assert err["mom"] <= MOM_TOL
        assert err["w"] == 0.0
        assert err["J"] <= J_TOL
        assert err["E"] <= F_TOL and err["B"] <= F_TOL
        assert err["rmin"] >= 0.0
        removed += err["removed"]
    assert removed > 0  # the wall removed the outgoing particles


SMOOTH_CASES = [
    # order, accumulator, passes along z, passes along r
    (2, 0, ((1, 2, 1),), ((1, 2, 1), (-1, 6, -1))),     # both axes, compensated along r
    (1, 2, (), ((0.25, 0.5, 0.25),)),                    # r only (first pass along r), int64 fold
    (3, 0, ((1, 2, 1), (1, 2, 1)), ()),                  # z only
]


@pytest.mark.parametrize("case", SMOOTH_CASES, ids=lambda c: f"o{c[0]}_acc{c[1]}_z{len(c[2])}_r{len(c[3])}")
def test_rz_smoothed_step_parity(orc, case):
    """Current smoothing in r-z: the filtered current density (mirror
    neighbours below the axis, zero at the wall) and the fields it drives,
    step by step against the oracle, with rings near the axis and the wall."""
    pic = _pic()
    order, acc, sz, sr = case
    nz, nr, dz, dr = 32, 20, 0.2, 0.2
    x, u, w = _ring_plasma(nz, nr, dz, dr, 3, 0.3, 500 + order)
    cfg = pic.Config(ndim=2, nx=(nz, nr), dx=(dz, dr), dt=0.1, shape_order=order, tile=(8, 8), sort_interval=1,
                     geometry=pic.PIC_GEOM_RZ, accumulator=acc, ion_density=1.0, smooth=(sz, sr))
    sim = pic.Pic(cfg)
    sim.load_particles(x, u, w, rqm=-1.0)
    E, B = _rz_fields(nz, nr, 17)
    sim.load_fields(E, B)
    print(f"case {case}", flush=True)
    for k in range(4):
        err = rz_step_parity(orc, sim, cfg)
        print(k, err, flush=True)
        assert err["pos"] <= POS_TOL and err["mom"] <= MOM_TOL
        assert err["w"] == 0.0
        assert err["J"] <= J_TOL
        assert err["E"] <= F_TOL and err["B"] <= F_TOL
    J = sim.current().reshape(3, nr, nz)
    assert np.abs(J[1, 0]).max() == 0.0  # J_r on the axis


def test_rz_pillbox_fields_match_the_oracle_over_many_steps(orc):
    """The vacuum TM010 pillbox mode for 200 steps: the FP32 r-z field solve
    against the FP64 oracle (no particles)."""
    special = pytest.importorskip("scipy.special")
    pic = _pic()
    nz, nr, dr = 8, 40, 0.1
    cfg = pic.Config(ndim=2, nx=(nz, nr), dx=(0.1, dr), dt=0.05, shape_order=1, tile=(8, 8), sort_interval=1,
                     geometry=pic.PIC_GEOM_RZ)
    g = oracle_grid(orc, cfg)
    R = (nr - 0.5) * dr
    k = special.jn_zeros(0, 1)[0] / R
    r = (np.arange(nr) - 0.5) * dr
    E = np.zeros((3, nr, nz))
    E[0] = special.j0(k * np.abs(r))[:, None]
    E = E.reshape(3, -1)
    B = np.zeros((3, nz * nr))
    sim = pic.Pic(cfg)
    sim.load_fields(E, B)
    sim.step(200)
    Eg, Bg = sim.fields()
    J = np.zeros((3, nz * nr))
    for _ in range(200):
        B = orc.yee_b(g, E, B, g.dt / 2)
        E = orc.yee_e(g, E, B, J, g.dt)
        B = orc.yee_b(g, E, B, g.dt / 2)
    # FP32 error growth over 200 steps stays far below the field scale
    assert rel_max(Eg, E) < 2e-5 and rel_max(Bg, B) < 2e-5


def test_rz_free_rings_follow_their_3d_lines():
    """Zero-weight rings in zero fields, 30 steps on the GPU: radius and
    local-frame momenta of the straight 3D line (closed form)."""
    pic = _pic()
    cfg = pic.Config(ndim=2, nx=(16, 64), dx=(0.2, 0.2), dt=0.1, shape_order=2, tile=(8, 8), sort_interval=1,
                     geometry=pic.PIC_GEOM_RZ)
    rng = np.random.default_rng(5)
    n = 200
    x0 = np.stack([rng.random(n) * 3.2, 0.02 + rng.random(n) * 6.0], 1)
    u0 = rng.normal(0, 0.6, (n, 3))
    sim = pic.Pic(cfg)
    sim.load_particles(x0, u0, np.zeros(n), rqm=-1.0)
    nsteps = 30
    sim.step(nsteps)
    x, u, _ = sim.state()
    t = nsteps * cfg.dt
    gam = np.sqrt(1 + (u0.astype(np.float32).astype(np.float64) ** 2).sum(1))
    px = x0[:, 1] + t * u0[:, 1] / gam
    py = t * u0[:, 2] / gam
    rr = np.hypot(px, py)
    inside = rr < (64 - 0.5) * 0.2
    assert inside.sum() == len(x)  # the ones that reached the wall are gone
    np.testing.assert_allclose(x[:, 1], rr[inside], atol=2e-4)
    np.testing.assert_allclose(u[:, 1], ((u0[:, 1] * px + u0[:, 2] * py) / rr)[inside], atol=2e-5)
    np.testing.assert_allclose(u[:, 2], ((-u0[:, 1] * py + u0[:, 2] * px) / rr)[inside], atol=2e-5)


def test_rz_rejects_unsupported_combinations():
    pic = _pic()
    base = dict(ndim=2, nx=(16, 16), dx=(0.2, 0.2), dt=0.1, shape_order=1, tile=(8, 8), geometry=pic.PIC_GEOM_RZ)
    for extra in ({"xmin": (0.0, 1.0, 0.0)}, {"sort_interval": 2}):
        with pytest.raises(pic.PicError):
            pic.Pic(pic.Config(**{**base, **extra}))
    sim = pic.Pic(pic.Config(**base))
    x = np.array([[0.5, 0.3]])
    sim.load_particles(x, np.zeros((1, 3)), np.array([-0.1]), rqm=-1.0)
    with pytest.raises(pic.PicError):
        sim.load_particles(np.array([[0.5, -0.1]]), np.zeros((1, 3)), np.array([-0.1]), rqm=-1.0)
    with pytest.raises(pic.PicError):
        sim.load_particles(np.array([[0.5, 3.11]]), np.zeros((1, 3)), np.array([-0.1]), rqm=-1.0)


@pytest.mark.parametrize("order", [1, 2, 3])
def test_rz_fp64_diagnostics_match_the_oracle(orc, order):
    """rho with the axis fold and ring volumes, the Gauss residual with the
    cylindrical divergence, energies with ring volumes and the moments
    (axial momentum, angular momentum) against the oracle; then the charge
    residual after one GPU step vanishes (cylindrical continuity) on every
    row the wall does not touch."""
    pic = _pic()
    nz, nr, dz, dr = 24, 20, 0.2, 0.2
    rng = np.random.default_rng(200 + order)
    n = nz * 12 * 3
    x = np.stack([rng.random(n) * nz * dz, rng.random(n) * 12 * dr], 1)  # away from the wall
    x[: n // 5, 1] = rng.random(n // 5) * 1.2 * dr
    u = rng.normal(0, 0.2, (n, 3))
    w = -(x[:, 1] / dr) / 3
    cfg = pic.Config(ndim=2, nx=(nz, nr), dx=(dz, dr), dt=0.1, shape_order=order, tile=(8, 10), sort_interval=1,
                     geometry=pic.PIC_GEOM_RZ, ion_density=0.7)
    sim = pic.Pic(cfg)
    sim.load_particles(x, u, w, rqm=-1.0)
    E, B = _rz_fields(nz, nr, 21)
    sim.load_fields(E, B)
    g = oracle_grid(orc, cfg)
    xs, us, ws = sim.state()
    Eg, Bg = sim.fields()
    rho_ref = orc.rho(g, xs, ws) + 0.7
    rho = sim.rho()
    np.testing.assert_allclose(rho, rho_ref, rtol=0, atol=1e-12 * np.abs(rho_ref).max())
    G = sim.gauss_residual()
    G_ref = orc.gauss_residual(g, Eg, rho_ref)
    np.testing.assert_allclose(G, G_ref, rtol=0, atol=1e-9 * np.abs(G_ref).max())
    en = sim.energy()
    fe = orc.field_energy(g, Eg, Bg)
    pm = orc.particle_moments(g, us, ws, -1.0, x=xs)
    np.testing.assert_allclose(en[:3], [fe[0], fe[1], pm[0]], rtol=1e-10)
    mo = sim.momentum()
    np.testing.assert_allclose(mo, [pm[1], pm[2], pm[3]], rtol=1e-10, atol=1e-12)
    # continuity after one step, rows 1 .. nr - 4 (the particles stay below row 14)
    sim.rho_snapshot()
    r0 = sim.rho()
    sim.step(1)
    C = sim.charge_residual().reshape(nr, nz)
    scale = np.abs(r0 - 0.7).max() / cfg.dt
    assert np.abs(C[1:nr - 4]).max() <= 1e-6 * scale


@pytest.mark.parametrize("order,ippc_r,acc,smooth,uth", [(1, 1, 0, (), 0.0), (2, 2, 0, (), 0.0), (3, 3, 2, (), 0.0),
                                                         (2, 2, 0, (((1, 2, 1),), ((1, 2, 1),)), 0.0),
                                                         (2, 3, 0, (), 0.1)])
def test_rz_window_step_parity(orc, order, ippc_r, acc, smooth, uth):
    """r-z with a moving window along z: each step against the oracle's
    window step in the r-z geometry across shifts, with rings near the axis,
    rings leaving through the wall and the back, and the ring lattice the
    window injects (weights proportional to the radius); one case with the
    current smoothed along z (zero beyond the window's ends) and r, one with
    thermally injected rings."""
    from test_gpu_window import window_step_parity

    pic = _pic()
    nz, nr, dz, dr = 32, 16, 0.2, 0.25
    x, u, w = _ring_plasma(nz, nr, dz, dr, 3, 0.3, 300 + order)
    cfg = pic.Config(ndim=2, nx=(nz, nr), dx=(dz, dr), dt=0.1, shape_order=order, tile=(8, 8), sort_interval=1,
                     geometry=pic.PIC_GEOM_RZ, move_window=1, inject_ppc=(2, ippc_r, 1), inject_w=-0.2,
                     accumulator=acc, xmin=(0.5, 0.0, 0.0), smooth=smooth, inject_uth=uth, inject_seed=99)
    sim = pic.Pic(cfg)
    sim.load_particles(x + np.array([0.5, 0.0]), u, w, rqm=-1.0)
    E, B = _rz_fields(nz, nr, 23)
    sim.load_fields(E, B)
    shifts = removed = 0
    for n in range(7):
        err = window_step_parity(orc, sim, cfg, n, nload=len(x))
        print(n, err, flush=True)
        assert err["inside"]
        assert err["pos"] <= POS_TOL and err["mom"] <= MOM_TOL
        assert err["w"] <= 1e-6
        assert err["J"] <= J_TOL
        assert err["E"] <= F_TOL and err["B"] <= F_TOL
        shifts += err["shift"]
        removed += err["removed"]
    assert shifts >= 3 and removed > 0
