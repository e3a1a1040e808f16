"""Seeded synthetic inputs for the PSATD field step.

This module is shared by the oracle tests, the GPU parity tests and the
benchmark.  It only produces arrays (fields, source profiles, time factors);
it holds none of the PSATD update itself.  The spectral projections used to
make the inputs physically consistent (transverse B, Gauss-consistent E,
charge from the continuity equation) are written here on their own, with
numpy's FFT as the only library primitive.

Units are normalized: c = eps0 = mu0 = 1, lambda0 = 1, so T0 = 1 and
omega0 = 2*pi.  Arrays are indexed [z][x] in 2D (the (x, z) plane of the
paper's simulations, Sec. II.B and Sec. V) and [z][y][x] in 3D, x fastest.
"""

from .fields import (  # noqa: F401
    LAMBDA0,
    lattice_k,
    spectral_div,
    spectral_grad,
    project_transverse,
    laser_2d,
    laser_3d,
    plane_wave_list,
    plane_wave_packets_3d,
    current_factors,
    current_profile,
    source_time_factors,
    SourceSchedule,
)
from .workloads import (  # noqa: F401
    Workload,
    Patch,
    workload,
    lattice_plane_wave,
    CONFIG_NAMES,
)
