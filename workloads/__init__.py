"""Seeded synthetic inputs for the DDA solve: voxelised scatterers and incident waves.

This package only describes *what* is scattered and *how it is lit*: voxel masks,
permittivity arrays, grid spacing, wavenumber and incident directions /
polarisations.  It contains none of the method's arithmetic (no polarisability,
no Green tensor, no incident-field evaluation), so both the CPU oracle side of
the tests and the HIP path can be fed from it without sharing any of the
computation they are checked on.
"""

from .geometry import (  # noqa: F401
    Scatterer,
    hex_prism_grid,
    hex_prism_fit,
    sphere_grid,
    cuboid_grid,
    random_mask,
)
from .incidence import (  # noqa: F401
    plane_wave_z,
    random_directions,
    batch_directions,
)
from .configs import (  # noqa: F401
    config_c1,
    config_c2,
    config_c3,
    config_c4,
    config_c5,
    config_c5_dense,
    plate_case,
    plate_fit_rounding,
    smooth7,
    PLATE_MU,
    PLATE_X,
)
