"""Dipole centres of the cubic lattice.

Cell (i, j, l) of an nx x ny x nz lattice with cell size d has its centre at
d * (i - nx/2 + 1/2, j - ny/2 + 1/2, l - nz/2 + 1/2): the lattice is centred
on the origin.  Occupied cells are listed in increasing linear index
l*ny*nx + j*nx + i (x fastest), the order every per-dipole array follows.
"""

from __future__ import annotations

import numpy as np


def occupied_indices(mask: np.ndarray) -> np.ndarray:
    """Linear indices (x fastest) of the occupied cells of mask[nz][ny][nx]."""
    return np.flatnonzero(np.asarray(mask).ravel() != 0).astype(np.int64)


def dipole_centres(mask: np.ndarray, d: float) -> np.ndarray:
    """Centres (nm) of the occupied cells, float64 [n_occ][3] as (x, y, z)."""
    m = np.asarray(mask)
    nz, ny, nx = m.shape
    lin = occupied_indices(m)
    l, rem = np.divmod(lin, ny * nx)
    j, i = np.divmod(rem, nx)
    c = np.empty((lin.size, 3), dtype=np.float64)
    c[:, 0] = d * (i - nx / 2.0 + 0.5)
    c[:, 1] = d * (j - ny / 2.0 + 0.5)
    c[:, 2] = d * (l - nz / 2.0 + 0.5)
    return c
