"""pic_diag_noalloc (the diagnostics entry point that allocates nothing)
against pic_diag, through the C ABI: two calls in a row on the device's
shared scratch, the second on a smaller grid."""
import ctypes as C

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _sim(pic, nx, ppc, seed, order):
    rng = np.random.default_rng(seed)
    ndim = len(nx)
    ncell = int(np.prod(nx))
    cells = np.repeat(np.arange(ncell), ppc)
    idx = np.stack(np.unravel_index(cells, tuple(reversed(nx)))[::-1], axis=1)
    dx = (0.2,) * ndim
    x = (idx + rng.random((len(cells), ndim))) * np.asarray(dx)
    u = rng.normal(0, 0.2, (len(cells), 3))
    w = np.full(len(cells), -1.0 / ppc)
    cfg = pic.Config(ndim=ndim, nx=nx, dx=dx, dt=0.08, shape_order=order, ion_density=1.0)
    sim = pic.Pic(cfg)
    sim.load_particles(x, u, w, rqm=-1.0)
    sim.load_fields(rng.normal(0, 0.05, (3, ncell)), rng.normal(0, 0.05, (3, ncell)))
    return cfg, sim


def _close(a, b, scale):
    return np.abs(a - b).max() <= 1e-12 * scale


@pytest.mark.parametrize("nx,order", [((40, 36, 24), 3), ((24, 20, 12), 2)])
def test_noalloc_diagnostics_equal_pic_diag(nx, order):
    import torch

    from paper_1503_00276_amd import pic

    print(f"grid {nx} order {order}", flush=True)
    cfg, sim = _sim(pic, nx, 2, 7 + order, order)
    ncell = int(np.prod(nx))
    out = torch.full((ncell,), float("nan"), dtype=torch.float64, device="cuda")
    sim.step(2)
    sim.rho_snapshot()
    sim.step(1)
    rho = sim.rho()
    scale = np.abs(rho).max()
    for kind, ref in [(pic.PIC_DIAG_RHO, rho), (pic.PIC_DIAG_GAUSS_RESIDUAL, sim.gauss_residual()),
                      (pic.PIC_DIAG_CHARGE_RESIDUAL, sim.charge_residual())]:
        for rep in range(2):  # the scratch keeps the last call's contents
            out.fill_(float("nan"))
            assert sim.diag_noalloc(kind, out) == ncell * 8
            got = out.cpu().numpy()
            assert np.isfinite(got).all()
            s = scale / cfg.dt if kind == pic.PIC_DIAG_CHARGE_RESIDUAL else scale / 0.2
            assert _close(got, ref, s), (kind, np.abs(got - ref).max(), s)
    sim.close()


def test_noalloc_rejects_what_it_cannot_do():
    import torch

    from paper_1503_00276_amd import pic

    cfg, sim = _sim(pic, (16, 16, 8), 2, 3, 1)
    sim.step(1)
    ncell = 16 * 16 * 8
    dev = torch.zeros(ncell, dtype=torch.float64, device="cuda")
    host = np.zeros(ncell)
    wr = C.c_size_t(0)
    L = pic.lib()
    # a host buffer is refused before any kernel runs
    assert L.pic_diag_noalloc(sim._h, pic.PIC_DIAG_RHO, C.c_void_p(host.ctypes.data), host.nbytes,
                              C.byref(wr)) == pic.PIC_E_INVALID
    # too small
    assert L.pic_diag_noalloc(sim._h, pic.PIC_DIAG_RHO, C.c_void_p(dev.data_ptr()), 8, C.byref(wr)) == pic.PIC_E_RANGE
    assert wr.value == ncell * 8
    # kinds it does not compute, and a residual without a snapshot
    assert L.pic_diag_noalloc(sim._h, pic.PIC_DIAG_ENERGY, C.c_void_p(dev.data_ptr()), dev.numel() * 8,
                              C.byref(wr)) == pic.PIC_E_UNSUPPORTED
    assert L.pic_diag_noalloc(sim._h, pic.PIC_DIAG_CHARGE_RESIDUAL, C.c_void_p(dev.data_ptr()), dev.numel() * 8,
                              C.byref(wr)) == pic.PIC_E_STATE
    sim.close()
