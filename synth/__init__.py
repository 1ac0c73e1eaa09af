"""Seeded synthetic inputs for the 2-D TE scattering solver.

This package only *generates inputs*: grids, relative-permittivity maps and
sampled incident plane waves.  It contains none of the solver's arithmetic
(no Green tensor, no operator, no Krylov method), so both the CPU oracle and
the GPU path may draw their inputs from it without sharing any computation.
"""

from .objects import (  # noqa: F401
    Grid,
    centred_grid,
    cell_centres,
    cylinder,
    square,
    layered_square,
    ellipse_mask,
    plane_wave,
    plane_wave_te3,
    plane_wave_tm,
    gaussian_random_field,
    random_field_object,
    inclusion_object,
    sinusoid_object,
)
from .workloads import workload, WORKLOADS  # noqa: F401
