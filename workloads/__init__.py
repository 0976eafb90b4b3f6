"""Seeded synthetic inputs shared by the oracle tests and the GPU path.

This package generates inputs only: lattice shape masks, Drude permittivity
tables, electron trajectories, energy grids and the named workload recipes.
It contains none of the method's arithmetic (no fields, no polarizabilities,
no interaction, no solves, no losses), so that the oracle and the HIP path
stay independent of each other and of it.
"""

from .shapes import (
    sphere_mask,
    capped_rod_mask,
    ellipsoid_mask,
    box_mask,
    random_mask,
    lattice_coordinate,
)
from .materials import drude_eps, uniform_eps
from .configs import (
    Workload,
    c1_single_solve,
    c2_nanorod_spectrum,
    c3_cherenkov,
    c4_impact_map,
    c5_request_stream,
    scaled_down,
)

__all__ = [
    "sphere_mask",
    "capped_rod_mask",
    "ellipsoid_mask",
    "box_mask",
    "random_mask",
    "lattice_coordinate",
    "drude_eps",
    "uniform_eps",
    "Workload",
    "c1_single_solve",
    "c2_nanorod_spectrum",
    "c3_cherenkov",
    "c4_impact_map",
    "c5_request_stream",
    "scaled_down",
]
