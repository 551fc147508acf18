"""FP64 CPU oracle of the PIC step (test infrastructure only).

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  It shares no code with the HIP library.
"""
from .oracle import (  # noqa: F401
    Grid,
    ISIS,
    TRISTAN,
    build,
    shape,
    gather,
    boris,
    deposit_cells,
    rho,
    yee_b,
    yee_e,
    step,
    gauss_residual,
    charge_residual,
    field_energy,
    particle_moments,
    smooth_current,
    step_window,
    window_shifts,
    splitmix64,
    thermal_normal,
    step_cyl,
    cyl_wall,
)
