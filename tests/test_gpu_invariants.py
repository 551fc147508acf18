"""Invariants of the method measured on the GPU's FP32 path, through the C ABI.

* A slow, cold, coherently drifting plasma (1e-4 and 1e-3 c): the current
  of a step against the oracle's FP64 deposit of the same moves, at the
  current tolerance (no bias from the current's fixed point).
* A zero-weight particle gyrating in a uniform external B for 10^4 steps
  (Sec. 3.2, Eq. momentum-update: the Boris rotation keeps |u| and gamma
  exactly, FP32 up to a random walk of its rounding; its positions lie on
  the polygon of the closed-form radius).
* A cold plasma oscillation (Sec. 3.1 loop): the leapfrog plasma frequency
  (2/dt) asin(w_p dt / 2).
"""
import math
import os

import numpy as np
import pytest

from parity import J_TOL, POS_TOL, oracle_grid, periodic_dx

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))


def _closed_forms():
    cf = {}
    with open(os.path.join(HERE, "golden", "closed_forms.txt")) as f:
        for line in f:
            line = line.strip()
            if line and not line.startswith("#"):
                k, v = line.split()
                cf[k] = float(v)
    return cf


def _pic():
    from paper_1503_00276_amd import pic

    return pic


@pytest.mark.parametrize("speed", [1e-4, 1e-3])
@pytest.mark.parametrize("ndim,order", [(2, 1), (2, 2), (2, 3), (3, 1), (3, 2), (3, 3)])
def test_slow_coherent_drift_current(orc, ndim, order, speed):
    """Every particle moves with the same small velocity, so all contributions
    to a node share their sign and any bias of the current's rounding unit
    adds up.  The GPU's current is compared with the oracle's FP64 deposit of
    the very moves the GPU made (its exported positions before and after the
    step): the current follows the FP32 positions exactly, as charge
    conservation demands, so this isolates the deposit's own arithmetic and
    rounding from the FP32 rounding of the position update (about 2^-25 of a
    cell per step, which at 1e-4 c is a part in 10^3 of the displacement)."""
    pic = _pic()
    nx = (32, 24) if ndim == 2 else (12, 12, 12)
    dx = (0.2,) * ndim
    ppc = 4 if ndim == 2 else 2
    rng = np.random.default_rng(100 * ndim + order)
    ncell = int(np.prod(nx))
    cells = np.repeat(np.arange(ncell), ppc)
    idx = np.stack(np.unravel_index(cells, tuple(reversed(nx)))[::-1], axis=1)
    x = (idx + rng.random((len(cells), ndim))) * np.asarray(dx)
    d = np.array([1.0, 0.6, 0.3])
    u = np.tile(speed * d / np.linalg.norm(d), (len(cells), 1))
    w = np.full(len(cells), -1.0 / ppc)
    cfg = pic.Config(ndim=ndim, nx=nx, dx=dx, dt=0.08, shape_order=order, tile=(4,) * ndim, ion_density=1.0)
    sim = pic.Pic(cfg)
    sim.load_particles(x, u, w, rqm=-1.0)
    g = oracle_grid(orc, cfg)
    L = np.asarray(nx) * np.asarray(dx)
    print(f"drift {speed} ndim {ndim} order {order}", flush=True)
    for k in range(2):
        x0, _, w0 = sim.state()
        sim.step(1)
        x1, u1, _ = sim.state()
        J = sim.current()
        a = x0 / np.asarray(dx)
        b = a + periodic_dx(x1, x0, L) / np.asarray(dx)
        v3 = u1[:, 2] / np.sqrt(1.0 + (u1 ** 2).sum(axis=1))
        ref = orc.deposit_cells(g, a, b, w0, v3)
        err = np.abs(J - ref).max() / np.abs(ref).max()
        # the displacement itself: the velocity times dt up to the FP32
        # rounding of the offsets
        mv = periodic_dx(x1, x0, L) - (u1[:, :ndim] / np.sqrt(1.0 + (u1 ** 2).sum(axis=1))[:, None]) * cfg.dt
        print(k, "J", err, "move", np.abs(mv / np.asarray(dx)).max(), flush=True)
        assert err <= J_TOL
        assert np.abs(mv / np.asarray(dx)).max() <= POS_TOL
    sim.close()


@pytest.mark.parametrize("ndim", [2, 3])
def test_uniform_b_gyration_keeps_u_and_radius_fp32(ndim):
    """q/m = -1, B = z (external), E = 0, dt = 0.1, u = (0.1, 0, 0): over
    10^4 FP32 steps |u| and gamma stay within the FP32 random-walk bound, and
    the positions stay on the circle of the closed-form radius."""
    pic = _pic()
    cf = _closed_forms()
    nx = (16, 16) if ndim == 2 else (8, 8, 8)
    dx = (0.2,) * ndim
    cfg = pic.Config(ndim=ndim, nx=nx, dx=dx, dt=0.1, shape_order=2, b0=(0.0, 0.0, 1.0), ion_density=0.0)
    sim = pic.Pic(cfg)
    x0 = np.array([[1.55, 1.45, 0.85][:ndim]])
    u0 = np.array([[0.1, 0.0, 0.0]])
    sim.load_particles(x0, u0, np.zeros(1), rqm=-1.0)
    pos, mom = [], []
    nsteps, every = 10000, 10
    for n in range(0, nsteps, every):
        sim.step(every)
        x, u, _ = sim.state()
        pos.append(x[0, :2].copy())
        mom.append(u[0].copy())
    pos, mom = np.array(pos), np.array(mom)
    umag = np.linalg.norm(mom, axis=1)
    gam = np.sqrt(1.0 + umag ** 2)
    # exact in exact arithmetic; in FP32 each rotation changes |u| by a few
    # units of 2^-24 in either direction, a random walk of about 2^-24 sqrt(N)
    # after N steps: allowed twice that (1.2e-5 at N = 10^4)
    tol = 2.0 * 2.0 ** -24 * math.sqrt(nsteps)
    drift = np.abs(umag / 0.1 - 1).max()
    print("|u| drift", drift, "tolerance", tol, flush=True)
    assert drift <= tol
    assert np.abs(gam / cf["boris_gamma"] - 1).max() <= tol
    assert np.abs(mom[:, 2]).max() == 0.0
    # the positions are the vertices of a regular polygon on a circle of the
    # closed-form radius: fit the centre by least squares (the periodic box is
    # far larger than the orbit: unwrap about the start)
    r = cf["boris_radius"]
    L = np.asarray(nx[:2]) * np.asarray(dx[:2])
    p = pos - L * np.round((pos - x0[0, :2]) / L)
    A = np.column_stack([2 * p, np.ones(len(p))])
    sol, *_ = np.linalg.lstsq(A, (p ** 2).sum(axis=1), rcond=None)
    centre = sol[:2]
    rad = np.linalg.norm(p - centre, axis=1)
    print("radius", rad.mean(), rad.min(), rad.max(), "closed form", r, flush=True)
    assert abs(rad.mean() / r - 1) <= 1e-5
    assert np.abs(rad / r - 1).max() <= 1e-4
    sim.close()


def test_cold_plasma_oscillation_frequency():
    """A cold plasma displaced by a long-wavelength sinusoid (unit density,
    q/m = -1, so w_p = 1) oscillates at (2/dt) asin(w_p dt / 2) on the GPU."""
    pic = _pic()
    cf = _closed_forms()
    nx, ppc_x = (256, 2), 2
    dx, dt = (0.2, 0.2), 0.1
    cfg = pic.Config(ndim=2, nx=nx, dx=dx, dt=dt, shape_order=1, ion_density=1.0)
    L = nx[0] * dx[0]
    ii, jj = np.meshgrid(np.arange(nx[0] * ppc_x), np.arange(nx[1] * ppc_x), indexing="ij")
    x = np.stack([(ii.ravel() + 0.5) * dx[0] / ppc_x, (jj.ravel() + 0.5) * dx[1] / ppc_x], axis=1)
    k = 2 * math.pi / L
    x[:, 0] += 1e-3 * np.sin(k * x[:, 0])
    w = np.full(len(x), -1.0 / (ppc_x * ppc_x))
    sim = pic.Pic(cfg)
    sim.load_particles(x, np.zeros((len(x), 3)), w, rqm=-1.0)
    # consistent initial E1 from Gauss's law along x1 (the GPU's FP64 charge)
    rho = sim.rho().reshape(nx[1], nx[0])
    e1 = np.cumsum(rho.mean(axis=0)) * dx[0]
    e1 -= e1.mean()
    E = np.zeros((3, nx[0] * nx[1]))
    E[0] = np.tile(e1, nx[1])
    sim.load_fields(E, np.zeros_like(E))
    proj = np.sin(k * (np.arange(nx[0]) + 0.5) * dx[0])
    sig = []
    for _ in range(330):
        sim.step(1)
        Ef, _ = sim.fields()
        sig.append(Ef[0].reshape(nx[1], nx[0]).mean(axis=0) @ proj)
    sig = np.array(sig)
    zc = [i + sig[i] / (sig[i] - sig[i + 1]) for i in range(len(sig) - 1) if sig[i] * sig[i + 1] < 0]
    omega = math.pi / (np.mean(np.diff(zc)) * dt)
    print("omega", omega, "leapfrog", cf["plasma_omega"], flush=True)
    assert len(zc) >= 8
    assert abs(omega / cf["plasma_omega"] - 1) < 1e-4, omega
    sim.close()
