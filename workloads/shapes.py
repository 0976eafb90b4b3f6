"""Lattice shape masks (uint8, shape [nz][ny][nx], x fastest).

A cubic lattice of n cells along an axis, cell size d, is centred on the
origin: cell i has its centre at d*(i - n/2 + 1/2).  A cell is occupied when
its centre lies inside (or on the boundary of) the shape.  The particle models
follow the shapes the paper simulates: spheres (section 3.2), a hemispherically
capped cylinder (section 3.4) and, for synthetic variety, ellipsoids.
"""

from __future__ import annotations

import numpy as np


def lattice_coordinate(n: int, d: float) -> np.ndarray:
    """Cell-centre coordinates along one axis of an n-cell lattice, in nm."""
    return d * (np.arange(n, dtype=np.float64) - n / 2.0 + 0.5)


def _grids(nx: int, ny: int, nz: int, d: float):
    x = lattice_coordinate(nx, d)
    y = lattice_coordinate(ny, d)
    z = lattice_coordinate(nz, d)
    return np.meshgrid(z, y, x, indexing="ij")  # Z, Y, X each [nz][ny][nx]


def sphere_mask(n: int, d: float, radius: float) -> np.ndarray:
    """Sphere of the given radius (nm) centred on an n^3 lattice."""
    Z, Y, X = _grids(n, n, n, d)
    return (X * X + Y * Y + Z * Z <= radius * radius).astype(np.uint8)


def ellipsoid_mask(nx: int, ny: int, nz: int, d: float, a: float, b: float, c: float) -> np.ndarray:
    """Axis-aligned ellipsoid with semi-axes a, b, c (nm) along x, y, z."""
    Z, Y, X = _grids(nx, ny, nz, d)
    return ((X / a) ** 2 + (Y / b) ** 2 + (Z / c) ** 2 <= 1.0).astype(np.uint8)


def capped_rod_mask(nx: int, ny: int, nz: int, d: float, radius: float, length: float,
                    axis: str = "x") -> np.ndarray:
    """Cylinder with hemispherical caps; total tip-to-tip length `length` (nm).

    The rod axis lies along `axis` through the lattice centre.  The straight
    part has length `length - 2*radius`.
    """
    Z, Y, X = _grids(nx, ny, nz, d)
    if axis == "x":
        a, r1, r2 = X, Y, Z
    elif axis == "y":
        a, r1, r2 = Y, X, Z
    elif axis == "z":
        a, r1, r2 = Z, X, Y
    else:
        raise ValueError("axis must be 'x', 'y' or 'z'")
    half = length / 2.0 - radius
    ac = np.clip(a, -half, half)  # nearest point on the axis segment
    dist2 = (a - ac) ** 2 + r1 * r1 + r2 * r2
    return (dist2 <= radius * radius).astype(np.uint8)


def box_mask(nx: int, ny: int, nz: int) -> np.ndarray:
    """Every cell occupied."""
    return np.ones((nz, ny, nx), dtype=np.uint8)


def random_mask(nx: int, ny: int, nz: int, fill: float, seed: int) -> np.ndarray:
    """Seeded random occupancy (for ragged, irregular index maps in tests)."""
    rng = np.random.default_rng(seed)
    m = (rng.random((nz, ny, nx)) < fill).astype(np.uint8)
    if m.sum() == 0:
        m.flat[rng.integers(m.size)] = 1
    return m
