"""ctypes loader for the FP64 C oracle ``pic_oracle.c``.

TEST INFRASTRUCTURE ONLY: only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may use it.  Most functions here are
argument marshalling around the C routine of the same name, whose arithmetic
lives in ``pic_oracle.c`` (which cites the dissertation's Ch. 3 passages);
the moving window's bookkeeping (``step_window``: removal, shift, injection)
and the generator of thermally injected momenta (``splitmix64``,
``thermal_normal``) are written here in numpy.
"""
from __future__ import annotations

import ctypes as C
import math
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "pic_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (FP64, no FMA contraction)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(
            ["gcc", "-O2", "-ffp-contract=off", "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"]
        )
        os.replace(tmp, _LIB)
    return _LIB


class _Grid(C.Structure):
    _fields_ = [
        ("dim", C.c_int32),
        ("nx", C.c_int32 * 3),
        ("dx", C.c_double * 3),
        ("xmin", C.c_double * 3),
        ("dt", C.c_double),
        ("order", C.c_int32),
        ("e0", C.c_double * 3),
        ("b0", C.c_double * 3),
        ("deposit", C.c_int32),
        ("smooth_level", C.c_int32 * 3),
        ("smooth_w", C.c_double * 72),
        ("window", C.c_int32),
        ("cyl", C.c_int32),
    ]

ISIS = 0
TRISTAN = 1


@dataclass
class Grid:
    """Grid, time step and shape order of one periodic simulation box."""

    dim: int
    nx: tuple
    dx: tuple
    dt: float
    order: int
    xmin: tuple = (0.0, 0.0, 0.0)
    e0: tuple = (0.0, 0.0, 0.0)
    b0: tuple = (0.0, 0.0, 0.0)
    deposit: int = ISIS  # ISIS, or TRISTAN (linear shape only)
    smooth: tuple = ()    # per axis: a list of (a, b, c) weights, one per smoothing pass
    window: int = 0       # 1: moving window along x1 (see step_window)
    inject_ppc: tuple = (1, 1, 1)  # moving window: injected particles per cell, per axis
    inject_w: float = 0.0          # moving window: weight of an injected particle
    inject_uth: float = 0.0        # moving window: thermal spread of the injected momenta (0: at rest)
    inject_seed: int = 0           # moving window: seed of their generator (see thermal_normal)
    cyl: int = 0          # 1: 2D cylindrically symmetric r-z box (x1 = z, x2 = r; see step_cyl)

    def c(self) -> _Grid:
        g = _Grid()
        g.dim = self.dim
        nx = list(self.nx) + [1] * (3 - len(self.nx))
        dx = list(self.dx) + [1.0] * (3 - len(self.dx))
        xm = list(self.xmin) + [0.0] * (3 - len(self.xmin))
        for i in range(3):
            g.nx[i] = int(nx[i]) if i < self.dim else 1
            g.dx[i] = float(dx[i])
            g.xmin[i] = float(xm[i])
            g.e0[i] = float(self.e0[i])
            g.b0[i] = float(self.b0[i])
        g.dt = float(self.dt)
        g.order = int(self.order)
        if self.deposit not in (ISIS, TRISTAN) or (self.deposit == TRISTAN and self.order != 1):
            raise ValueError("TRISTAN deposit is defined for the linear shape only")
        g.deposit = int(self.deposit)
        g.window = int(self.window)
        if self.cyl:
            if self.dim != 2:
                raise ValueError("the r-z geometry is 2D")
            if float(xm[1]) != 0.0:
                raise ValueError("in r-z the second coordinate is the radius (xmin[1] = 0)")
        g.cyl = int(self.cyl)
        for ax, passes in enumerate(self.smooth):
            if len(passes) > 8:
                raise ValueError("at most 8 smoothing passes per axis")
            g.smooth_level[ax] = len(passes)
            for p, wts in enumerate(passes):
                for k in range(3):
                    g.smooth_w[(ax * 8 + p) * 3 + k] = float(wts[k])
        return g

    @property
    def ncell(self) -> int:
        n = 1
        for i in range(self.dim):
            n *= int(self.nx[i])
        return n

    @property
    def shape(self) -> tuple:
        """numpy shape of one grid component, slowest axis first."""
        return tuple(int(self.nx[i]) for i in reversed(range(self.dim)))


_lib = None


def _L():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        lib = C.CDLL(_LIB)
        P = C.POINTER(C.c_double)
        G = C.POINTER(_Grid)
        lib.orc_shape.argtypes = [C.c_int, C.c_double]
        lib.orc_shape.restype = C.c_double
        lib.orc_gather.argtypes = [G, C.c_int64, P, P, P, P, P]
        lib.orc_boris.argtypes = [C.c_int64, P, P, P, P, C.c_double]
        lib.orc_deposit_cells.argtypes = [G, C.c_int64, P, P, P, P, P]
        lib.orc_rho.argtypes = [G, C.c_int64, P, P, P]
        lib.orc_yee_b.argtypes = [G, P, P, C.c_double]
        lib.orc_yee_e.argtypes = [G, P, P, P, C.c_double]
        lib.orc_step.argtypes = [G, C.c_int64, P, P, P, P, P, P, P]
        lib.orc_step.restype = C.c_int
        lib.orc_gauss_residual.argtypes = [G, P, P, P]
        lib.orc_charge_residual.argtypes = [G, P, P, P, P]
        lib.orc_field_energy.argtypes = [G, P, P, P]
        lib.orc_particle_moments.argtypes = [G, C.c_int64, P, P, P, P]
        lib.orc_smooth_current.argtypes = [G, P]
        lib.orc_yee_b_cyl.argtypes = [G, P, P, C.c_double]
        lib.orc_yee_e_cyl.argtypes = [G, P, P, P, C.c_double]
        lib.orc_particle_moments_cyl.argtypes = [G, C.c_int64, P, P, P, P, P]
        _lib = lib
    return _lib


def _p(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"], (a.dtype, a.flags)
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


def shape(order: int, t: float) -> float:
    return _L().orc_shape(int(order), float(t))


def gather(g: Grid, x, E, B):
    """E, B (each [3, ncell]) at absolute positions x[n, dim] -> (Ep, Bp) [n, 3]."""
    x = _f64(x).reshape(-1, g.dim)
    n = x.shape[0]
    E = _f64(E).reshape(3, g.ncell)
    B = _f64(B).reshape(3, g.ncell)
    Ep = np.zeros((n, 3))
    Bp = np.zeros((n, 3))
    gc = g.c()
    _L().orc_gather(C.byref(gc), n, _p(x), _p(E), _p(B), _p(Ep), _p(Bp))
    return Ep, Bp


def boris(u, Ep, Bp, qm, dt):
    """Return u^{n+1/2} from u^{n-1/2} [n, 3] and fields at the particles."""
    u = _f64(u).reshape(-1, 3).copy()
    n = u.shape[0]
    Ep = _f64(Ep).reshape(n, 3)
    Bp = _f64(Bp).reshape(n, 3)
    qm = _f64(np.broadcast_to(qm, (n,)))
    _L().orc_boris(n, _p(u), _p(Ep), _p(Bp), _p(qm), float(dt))
    return u


def deposit_cells(g: Grid, a, b, w, v3=None, J=None):
    """ISIS current of particles moving a -> b (cell units, unwrapped) -> J [3, ncell]."""
    a = _f64(a).reshape(-1, g.dim)
    n = a.shape[0]
    b = _f64(b).reshape(n, g.dim)
    w = _f64(np.broadcast_to(w, (n,)))
    v3 = _f64(np.zeros(n) if v3 is None else np.broadcast_to(v3, (n,)))
    J = np.zeros((3, g.ncell)) if J is None else J
    gc = g.c()
    _L().orc_deposit_cells(C.byref(gc), n, _p(a), _p(b), _p(w), _p(v3), _p(J))
    return J


def rho(g: Grid, x, w, out=None):
    x = _f64(x).reshape(-1, g.dim)
    n = x.shape[0]
    w = _f64(np.broadcast_to(w, (n,)))
    out = np.zeros(g.ncell) if out is None else out
    gc = g.c()
    _L().orc_rho(C.byref(gc), n, _p(x), _p(w), _p(out))
    return out


def yee_b(g: Grid, E, B, h):
    """B - h curl E (returns a new array)."""
    E = _f64(E).reshape(3, g.ncell)
    B = _f64(B).reshape(3, g.ncell).copy()
    gc = g.c()
    (_L().orc_yee_b_cyl if g.cyl else _L().orc_yee_b)(C.byref(gc), _p(E), _p(B), float(h))
    return B


def yee_e(g: Grid, E, B, J, dt):
    """E + dt (curl B - J) (returns a new array)."""
    E = _f64(E).reshape(3, g.ncell).copy()
    B = _f64(B).reshape(3, g.ncell)
    J = _f64(J).reshape(3, g.ncell)
    gc = g.c()
    (_L().orc_yee_e_cyl if g.cyl else _L().orc_yee_e)(C.byref(gc), _p(E), _p(B), _p(J), float(dt))
    return E


def smooth_current(g: Grid, J):
    """The current after the smoothing passes of g (returns a new array)."""
    J = _f64(J).reshape(3, g.ncell).copy()
    gc = g.c()
    _L().orc_smooth_current(C.byref(gc), _p(J))
    return J


@dataclass
class StepResult:
    x: np.ndarray
    u: np.ndarray
    E: np.ndarray
    B: np.ndarray
    J: np.ndarray = field(default=None)


def step(g: Grid, x, u, w, qm, E, B) -> StepResult:
    """One full PIC step; inputs are not modified."""
    x = _f64(x).reshape(-1, g.dim).copy()
    n = x.shape[0]
    u = _f64(u).reshape(n, 3).copy()
    w = _f64(np.broadcast_to(w, (n,)))
    qm = _f64(np.broadcast_to(qm, (n,)))
    E = _f64(E).reshape(3, g.ncell).copy()
    B = _f64(B).reshape(3, g.ncell).copy()
    J = np.zeros((3, g.ncell))
    gc = g.c()
    rc = _L().orc_step(C.byref(gc), n, _p(x), _p(u), _p(w), _p(qm), _p(E), _p(B), _p(J))
    if rc != 0:
        raise MemoryError("oracle step failed to allocate")
    return StepResult(x=x, u=u, E=E, B=B, J=J)


def window_shifts(g: Grid, n: int) -> int:
    """Cell shifts of a window moving along x1 at the speed of light after n
    steps: the window is moved by dx1 whenever the distance c t it should have
    travelled exceeds the distance it has been moved by a whole cell (Sec. 4.5,
    dynamic spaces; c = 1 in the normalised units)."""
    return int(math.floor(n * (g.dt / g.dx[0])))


_GOLDEN = np.uint64(0x9E3779B97F4A7C15)


def splitmix64(seed: int, n) -> np.ndarray:
    """Outputs n (>= 1, array) of the SplitMix64 generator seeded with 'seed'
    (Steele, Lea and Flood, "Fast splittable pseudorandom number generators",
    OOPSLA 2014): state_n = seed + n * 0x9e3779b97f4a7c15 (mod 2^64), output
    the state mixed by two xor-shift-multiply rounds and a final xor-shift."""
    with np.errstate(over="ignore"):
        z = np.uint64(seed) + np.asarray(n, dtype=np.uint64) * _GOLDEN
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
        return z ^ (z >> np.uint64(31))


def thermal_normal(seed: int, ids, c: int) -> np.ndarray:
    """Standard normal deviates for component c of particles 'ids' by the
    Box-Muller transform (1958) of U1 in (0, 1] and U2 in [0, 1), the top 53
    bits of SplitMix64 outputs 8 id + 2c + 1 and 8 id + 2c + 2."""
    ids = np.asarray(ids, dtype=np.uint64)
    n = np.uint64(8) * ids + np.uint64(2 * c)
    u1 = ((splitmix64(seed, n + np.uint64(1)) >> np.uint64(11)).astype(np.float64) + 1.0) * 2.0 ** -53
    u2 = (splitmix64(seed, n + np.uint64(2)) >> np.uint64(11)).astype(np.float64) * 2.0 ** -53
    return np.sqrt(-2.0 * np.log(u1)) * np.cos(2.0 * math.pi * u2)


def step_window(g: Grid, n: int, x, u, w, qm, E, B, id0: int = 0) -> StepResult:
    """One PIC step of a box whose window moves along x1 at c (Sec. 4.5).

    x are positions relative to the window's current lower corner.  The step
    is the ordinary one with x1 not periodic (grid values beyond the x1 ends
    are zero, currents deposited there are dropped); then
      1. particles that left the window through an x1 face are removed;
      2. if the window moves after this step (n -> n+1), every grid array
         moves down by one x1 cell, the new front cell column gets zero E, B
         (and J), particles move by -dx1 and those that fall behind the window
         are removed, and a plasma is initialised in the front column:
         inject_ppc per axis on a regular sub-lattice of each cell, weight
         inject_w, cells in increasing linear index, lattice points with
         axis 1 fastest; the injected particles take ids id0, id0 + 1, ...
         in that order and momenta inject_uth * thermal_normal(inject_seed,
         id, c) per component (u = 0 for inject_uth = 0: a cold plasma).
    Returns x, u, w of the survivors (in input order) followed by the
    injected particles, E, B, J, and 'keep', the survivors' input indices.
    In the r-z geometry (x = (z, r)) particles that reach the wall are
    removed too, and the injected lattice is the same in cell coordinates
    without its points below the axis (cell coordinate < 1/2), each with
    weight inject_w * r / dr (a uniform density)."""
    assert g.window == 1
    r = step(g, x, u, w, qm, E, B)
    w = _f64(np.broadcast_to(w, (len(r.x),))).copy()
    L1 = g.nx[0] * g.dx[0]
    inside = (r.x[:, 0] >= 0.0) & (r.x[:, 0] < L1)
    if g.cyl:
        inside &= r.x[:, 1] < cyl_wall(g)
    keep = np.nonzero(inside)[0]
    x1, u1, w1 = r.x[keep], r.u[keep], w[keep]
    E1, B1, J1 = r.E, r.B, r.J
    if window_shifts(g, n + 1) > window_shifts(g, n):
        shape = g.shape
        def shift(F):
            F = F.reshape((3,) + shape).copy()
            F[..., :-1] = F[..., 1:]
            F[..., -1] = 0.0
            return F.reshape(3, -1)
        E1, B1, J1 = shift(E1), shift(B1), shift(J1)
        x1 = x1.copy()
        x1[:, 0] -= g.dx[0]
        back = np.nonzero(x1[:, 0] >= 0.0)[0]
        keep = keep[back]
        x1, u1, w1 = x1[back], u1[back], w1[back]
        # cold plasma in the new front column
        d = g.dim
        ppc = list(g.inject_ppc)[:d]
        if d == 2:
            offs = np.stack(np.meshgrid((np.arange(ppc[0]) + 0.5) / ppc[0], (np.arange(ppc[1]) + 0.5) / ppc[1],
                                        indexing="xy"), -1).reshape(-1, 2)
        else:
            o = np.meshgrid((np.arange(ppc[0]) + 0.5) / ppc[0], (np.arange(ppc[1]) + 0.5) / ppc[1],
                            (np.arange(ppc[2]) + 0.5) / ppc[2], indexing="ij")
            offs = np.stack([o[0].transpose(2, 1, 0), o[1].transpose(2, 1, 0), o[2].transpose(2, 1, 0)],
                            -1).reshape(-1, 3)
        cells = []
        if d == 2:
            for j in range(g.nx[1]):
                cells.append((g.nx[0] - 1, j))
        else:
            for k in range(g.nx[2]):
                for j in range(g.nx[1]):
                    cells.append((g.nx[0] - 1, j, k))
        newx = np.concatenate([(np.asarray(c, dtype=float) + offs) * np.asarray(g.dx[:d]) for c in cells])
        neww = np.full(len(newx), float(g.inject_w))
        ids = int(id0) + np.arange(len(newx))
        if g.cyl:
            # cell coordinate r/dr + 1/2: drop the points below the axis
            newx[:, 1] -= 0.5 * g.dx[1]
            ok = newx[:, 1] >= 0.0
            newx = newx[ok]
            ids = ids[ok]
            neww = float(g.inject_w) * newx[:, 1] / g.dx[1]
        newu = np.zeros((len(newx), 3))
        if g.inject_uth > 0.0:
            for c in range(3):
                newu[:, c] = g.inject_uth * thermal_normal(g.inject_seed, ids, c)
        x1 = np.concatenate([x1, newx])
        u1 = np.concatenate([u1, newu])
        w1 = np.concatenate([w1, neww])
    return StepResult(x=x1, u=u1, E=E1, B=B1, J=J1), w1, keep


def gauss_residual(g: Grid, E, rho_):
    E = _f64(E).reshape(3, g.ncell)
    rho_ = _f64(rho_).reshape(g.ncell)
    G = np.zeros(g.ncell)
    gc = g.c()
    _L().orc_gauss_residual(C.byref(gc), _p(E), _p(rho_), _p(G))
    return G


def charge_residual(g: Grid, rho0, rho1, J):
    rho0 = _f64(rho0).reshape(g.ncell)
    rho1 = _f64(rho1).reshape(g.ncell)
    J = _f64(J).reshape(3, g.ncell)
    Cc = np.zeros(g.ncell)
    gc = g.c()
    _L().orc_charge_residual(C.byref(gc), _p(rho0), _p(rho1), _p(J), _p(Cc))
    return Cc


def field_energy(g: Grid, E, B):
    E = _f64(E).reshape(3, g.ncell)
    B = _f64(B).reshape(3, g.ncell)
    out = np.zeros(2)
    gc = g.c()
    _L().orc_field_energy(C.byref(gc), _p(E), _p(B), _p(out))
    return out


def particle_moments(g: Grid, u, w, qm, x=None):
    """[kinetic energy, momentum (3)]; in r-z (x = (z, r) needed) [kinetic
    energy, axial momentum, sum of radial momenta, angular momentum]."""
    u = _f64(u).reshape(-1, 3)
    n = u.shape[0]
    w = _f64(np.broadcast_to(w, (n,)))
    qm = _f64(np.broadcast_to(qm, (n,)))
    out = np.zeros(4)
    gc = g.c()
    if g.cyl:
        x = _f64(x).reshape(n, 2)
        _L().orc_particle_moments_cyl(C.byref(gc), n, _p(x), _p(u), _p(w), _p(qm), _p(out))
    else:
        _L().orc_particle_moments(C.byref(gc), n, _p(u), _p(w), _p(qm), _p(out))
    return out


def cyl_wall(g: Grid) -> float:
    """Radius of the conducting wall of an r-z box: (nr - 1/2) dr."""
    return (g.nx[1] - 0.5) * g.dx[1]


def step_cyl(g: Grid, x, u, w, qm, E, B):
    """One PIC step of an r-z box (Sec. 3.3); x = (z, r).  Particles that
    reach the wall at r = (nr - 1/2) dr are removed after depositing their
    current.  Returns (StepResult of the survivors, their w, their input
    indices)."""
    assert g.cyl == 1
    r = step(g, x, u, w, qm, E, B)
    w = _f64(np.broadcast_to(w, (len(r.x),))).copy()
    keep = np.nonzero(r.x[:, 1] < cyl_wall(g))[0]
    return StepResult(x=r.x[keep], u=r.u[keep], E=r.E, B=r.B, J=r.J), w[keep], keep
