"""Write cubic3d_64_energy.txt: the FP64 oracle's energy history over 100
steps of the 64^3 sub-run of the uniform cubic-shape 3D plasma (4 particles
per cell, u_th = 0.02, dx = 0.05, dt = 0.02, seeded as in workloads.py).
Calls only the oracle; single thread, about an hour and a half.

  python tests/golden/make_cubic_sub_energy.py
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_1503_00276_amd import workloads as W  # noqa: E402


def main(steps=100):
    oracle.build(force=False)
    wl = W.workload5_sub()
    g = oracle.Grid(dim=3, nx=wl.nx, dx=wl.dx, dt=wl.dt, order=wl.order)
    x, u, w = wl.x, wl.u, wl.w
    E = np.zeros((3, wl.ncell))
    B = np.zeros((3, wl.ncell))
    rows = []
    t0 = time.time()
    for n in range(steps):
        r = oracle.step(g, x, u, w, 1.0 / wl.rqm, E, B)
        x, u, E, B = r.x, r.u, r.E, r.B
        fe = oracle.field_energy(g, E, B)
        ke = oracle.particle_moments(g, u, w, 1.0 / wl.rqm)[0]
        rows.append((n + 1, fe[0], fe[1], ke))
        print(f"step {n + 1}: W_E {fe[0]:.12e} W_B {fe[1]:.12e} W_K {ke:.12e} ({time.time() - t0:.0f} s)", flush=True)
    out = os.path.join(HERE, "cubic3d_64_energy.txt")
    with open(out, "w") as f:
        f.write("# FP64 oracle energy history of the 64^3 sub-run of the uniform cubic-shape 3D plasma\n")
        f.write("# (tests/golden/make_cubic_sub_energy.py): after step n, field energies (V/2) sum |E|^2 and\n")
        f.write("# (V/2) sum |B|^2, kinetic energy V sum_p w rqm (gamma - 1) at u^{n+1/2}\n")
        f.write("# step W_E W_B W_K\n")
        for r in rows:
            f.write(f"{r[0]} {r[1]:.15e} {r[2]:.15e} {r[3]:.15e}\n")
    print("wrote", out)


if __name__ == "__main__":
    main()
