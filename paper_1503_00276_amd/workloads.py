"""Seeded synthetic inputs (initial particles and fields) for the PIC workloads.

Shared by the tests, the benchmark and the checker: this module only draws
random numbers and lays out initial conditions; it holds none of the PIC
method's arithmetic.  Generator: numpy PCG64, base seed 150300276; workload k
uses seed + k, batch instance j uses seed + 1000 + j.

Workloads (sizes from the dissertation's run scales; units normalised):
  1  2D3V thermal plasma, 64x64, dx=0.2, dt=0.1, 16 uniform-random particles
     per cell, u_th=0.01, CIC                                  (65,536 e-)
  2  2D3V laser wakefield, 1024x256, dx=(0.05,0.2)/k0, dt=0.95 Courant,
     8 per cell on a (2,4) sub-lattice, n=0.01 n_c with a 20-cell ramp,
     linearly polarised laser a0=2, quadratic shape        (2,097,152 e-)
  3  3D3V beam-driven blowout, 256x128x128, dx=0.05, dt=0.02, 8 per cell
     (2,2,2) background + 2^20 bi-Gaussian beam, quadratic (34,603,008)
  4  64 independent 2D thermal instances (parameter scan), CIC or quadratic
  5  3D3V uniform thermal plasma, 512x256x256, 4 per cell, u_th=0.02, cubic
     (134,217,728 e-), and its 64^3 sub-run
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np

BASE_SEED = 150300276


@dataclass
class Workload:
    name: str
    ndim: int
    nx: tuple
    dx: tuple
    dt: float
    order: int
    steps: int
    x: np.ndarray            # [n, ndim] absolute positions
    u: np.ndarray            # [n, 3]
    w: np.ndarray            # [n]
    rqm: float = -1.0
    ion_density: float = 1.0
    E: Optional[np.ndarray] = None  # [3, ncell] or None (zero)
    B: Optional[np.ndarray] = None
    extra: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return len(self.w)

    @property
    def ncell(self) -> int:
        return int(np.prod(self.nx))


def rng_for(k: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(BASE_SEED + k))


def uniform_in_cells(rng, nx, dx, ppc, dtype=np.float64):
    """ppc positions uniformly at random inside every cell, cell by cell."""
    ndim = len(nx)
    ncell = int(np.prod(nx))
    cells = np.repeat(np.arange(ncell, dtype=np.int64), ppc)
    idx = np.stack(np.unravel_index(cells, tuple(reversed(nx)))[::-1], axis=1)
    x = (idx + rng.random((len(cells), ndim))) * np.asarray(dx)
    return x.astype(dtype)


def lattice_in_cells(nx, dx, per_axis):
    """Regular sub-lattice of prod(per_axis) positions per cell (num_par_x)."""
    ndim = len(nx)
    offs = np.stack(np.meshgrid(*[(np.arange(k) + 0.5) / k for k in per_axis], indexing="ij"), -1).reshape(-1, ndim)
    grids = np.stack(np.meshgrid(*[np.arange(n) for n in nx], indexing="ij"), -1).reshape(-1, ndim)
    pos = (grids[:, None, :] + offs[None, :, :]).reshape(-1, ndim)
    return pos * np.asarray(dx)


def thermal(nx, dx, dt, order, ppc, uth, density=1.0, seed_k=1, steps=100, name="thermal") -> Workload:
    rng = rng_for(seed_k)
    x = uniform_in_cells(rng, nx, dx, ppc)
    u = rng.normal(0.0, uth, size=(len(x), 3))
    w = np.full(len(x), -density / ppc)
    return Workload(name, len(nx), tuple(nx), tuple(dx), dt, order, steps, x, u, w, ion_density=density)


def workload1() -> Workload:
    return thermal((64, 64), (0.2, 0.2), 0.1, 1, 16, 0.01, 1.0, seed_k=1, steps=100,
                   name="2d3v_thermal_64x64_cic")


def courant_dt(dx, frac):
    return frac / math.sqrt(sum(1.0 / d ** 2 for d in dx))


def _poly_ramp(s):
    s = np.clip(s, 0.0, 1.0)
    return 10 * s ** 3 - 15 * s ** 4 + 6 * s ** 5


def laser_fields(nx, dx, a0=2.0, k0=1.0, x_start=5.0, length=30.0, w0=2 * math.pi * 10, center2=None):
    """Linearly polarised (E2, B3) pulse moving along +x1: E2 = B3 = a0 env sin(k0 x1),
    polynomial rise and fall (10s^3 - 15s^4 + 6s^5) over half the length each and a
    Gaussian transverse profile; sampled at the staggered E2 (i, j+1/2) and
    B3 (i+1/2, j+1/2) locations of the grid layout."""
    n1, n2 = nx
    L2 = n2 * dx[1]
    c2 = L2 / 2 if center2 is None else center2
    half = length / 2

    def env(x1):
        xi = x1 - x_start
        return np.where(xi < half, _poly_ramp(xi / half), _poly_ramp((length - xi) / half)) * ((xi >= 0) & (xi <= length))

    i = np.arange(n1)
    j = np.arange(n2)
    E = np.zeros((3, n2, n1))
    B = np.zeros((3, n2, n1))
    x1e = i * dx[0]
    x1b = (i + 0.5) * dx[0]
    x2 = (j + 0.5) * dx[1]
    trans = np.exp(-((x2 - c2) ** 2) / w0 ** 2)
    E[1] = a0 * trans[:, None] * (env(x1e) * np.sin(k0 * x1e))[None, :]
    B[2] = a0 * trans[:, None] * (env(x1b) * np.sin(k0 * x1b))[None, :]
    return E.reshape(3, -1), B.reshape(3, -1)


def workload2(nx=(1024, 256)) -> Workload:
    dx = (0.05, 0.2)
    dt = courant_dt(dx, 0.95)
    x = lattice_in_cells(nx, dx, (2, 4))
    n_plasma = 0.01
    ramp_cells = 20
    ramp = np.minimum(1.0, (np.floor(x[:, 0] / dx[0]) + 0.5) / ramp_cells)
    w = -n_plasma * ramp / 8.0
    u = np.zeros((len(x), 3))
    E, B = laser_fields(nx, dx)
    return Workload("2d3v_lwfa_1024x256_quadratic", 2, tuple(nx), dx, dt, 2, 2000, x, u, w,
                    ion_density=n_plasma, E=E, B=B, extra={"ramp_cells": ramp_cells})


def workload3(nx=(256, 128, 128), nbeam=2 ** 20) -> Workload:
    rng = rng_for(3)
    dx = (0.05, 0.05, 0.05)
    dt = 0.02
    xb = lattice_in_cells(nx, dx, (2, 2, 2))
    wb = np.full(len(xb), -1.0 / 8)
    L = np.asarray(nx) * np.asarray(dx)
    sz, sr, nb_peak = 0.5, 0.1, 4.0
    centre = np.array([3.0, L[1] / 2, L[2] / 2])
    beam = rng.normal(0.0, 1.0, size=(nbeam, 3)) * np.array([sz, sr, sr]) + centre
    gam = rng.normal(2.0e4, 20.0, size=nbeam)
    ub = np.zeros((nbeam, 3))
    ub[:, 0] = np.sqrt(gam ** 2 - 1.0)
    V = float(np.prod(dx))
    w_beam = -nb_peak * (2 * math.pi) ** 1.5 * sz * sr * sr / (nbeam * V)
    x = np.concatenate([xb, beam])
    u = np.concatenate([np.zeros((len(xb), 3)), ub])
    w = np.concatenate([wb, np.full(nbeam, w_beam)])
    return Workload("3d3v_beam_blowout_256x128x128_quadratic", 3, tuple(nx), dx, dt, 2, 500, x, u, w,
                    ion_density=1.0, extra={"nbeam": nbeam, "w_beam": w_beam})


def workload4(ninst=64, steps=200) -> List[Workload]:
    grids = [(64, 64), (128, 128), (256, 128), (512, 256)]
    out = []
    for j in range(ninst):
        rng = rng_for(1000 + j)
        nx = grids[int(rng.integers(0, 4))]
        ppc = int(rng.integers(4, 33))
        dens = float(rng.uniform(0.5, 2.0))
        uth = float(rng.uniform(0.005, 0.05))
        order = int(rng.integers(1, 3))
        x = uniform_in_cells(rng, nx, (0.2, 0.2), ppc)
        u = rng.normal(0.0, uth, size=(len(x), 3))
        w = np.full(len(x), -dens / ppc)
        out.append(Workload(f"scan_{j}", 2, nx, (0.2, 0.2), 0.1, order, steps, x, u, w, ion_density=dens,
                            extra={"ppc": ppc, "uth": uth}))
    return out


def workload5(nx=(512, 256, 256)) -> Workload:
    wl = thermal(nx, (0.05, 0.05, 0.05), 0.02, 3, 4, 0.02, 1.0, seed_k=5, steps=100,
                 name="3d3v_uniform_%dx%dx%d_cubic" % tuple(nx))
    return wl


def workload5_sub() -> Workload:
    return workload5((64, 64, 64))
