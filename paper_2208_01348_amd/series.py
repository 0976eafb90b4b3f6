"""Spectra of one particle on a series of lattices and their Richardson
extrapolation to zero dipole size (section 3.2: a quadratic in d, point
errors taken to scale as d^3, 95 % intervals of twice the standard error).

Orchestration only: every solve and loss sum runs in libdda's kernels, and the
fit is libdda's dda_richardson.
"""

from __future__ import annotations

from typing import Callable, Sequence

import numpy as np

from . import _lib as L
from .solver import DDASolver


def lattice_series(mask_fn: Callable[[int, float], np.ndarray], size_nm: float,
                   n_list: Sequence[int], m_h: complex, beta: float, energies,
                   eps_fn: Callable[[np.ndarray], np.ndarray], r0, precision: str = "mixed",
                   tol: float = 1e-8, solver: str = "cocg", maxit: int = 50000):
    """Solves the spectrum on lattices of n_x = n cells across size_nm
    (d = size_nm / n), with mask_fn(n, d) giving each lattice's mask.
    Returns (d [n_lat], P [n_lat][rhs][4], extrapolated [rhs][4], ci95
    [rhs][4], infos per lattice); rhs = energy-major over the trajectories."""
    E = np.atleast_1d(np.asarray(energies, dtype=np.float64))
    R = np.asarray(r0, dtype=np.float64).reshape(-1, 3)
    ds, Ps, infos = [], [], []
    for n in n_list:
        d = size_nm / n
        mask = mask_fn(n, d)
        s = DDASolver(mask, d, m_h, precision=precision, tol=tol, maxit=maxit, solver=solver)
        eps = np.repeat(np.asarray(eps_fn(E))[:, None], s.n_occ, axis=1)
        P, info = s.spectrum(E, beta, eps, R)
        s.close()
        ds.append(d)
        Ps.append(np.asarray(P))
        infos.append(info)
    P_all = np.stack(Ps)
    ext = np.empty(P_all.shape[1:])
    ci = np.empty(P_all.shape[1:])
    for r in range(P_all.shape[1]):
        for q in range(P_all.shape[2]):
            ext[r, q], ci[r, q] = L.dda_richardson(ds, P_all[:, r, q])
    return np.asarray(ds), P_all, ext, ci, infos
