"""The whole DDA EELS/CL path for one (energy, trajectory), in plain FP64.

Steps in the order the method takes them: lattice -> polarizabilities ->
electron field (eq. 25) -> solve A p = e -> reductions (eqs. 37, 48, 18, 42).
"""

from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from . import cdense
from .electron import auxiliary_field, incident_field, k0_of
from .lattice import dipole_centres
from .losses import p_abs, p_cl, p_eels, p_ext
from .polarizability import polarizability, relative_m2
from .solve import bicgstab, lu_solve

LU_MAX_DIPOLES = 1500


@dataclass
class PointResult:
    p_eels: float
    p_ext: float
    p_abs: float
    p_cl: float
    p_hat: np.ndarray
    e_hat: np.ndarray
    iters: int
    residual: float


def system(mask, d, eps_dipoles, m_h, energy_eV, pol="ldr"):
    """Centres, alpha, host wavenumber k and m^2 for one energy."""
    centres = dipole_centres(mask, d)
    k = complex(m_h) * k0_of(energy_eV)
    eps = np.broadcast_to(np.asarray(eps_dipoles, dtype=np.complex128), (centres.shape[0],))
    alpha = polarizability(pol, eps, m_h, d, k)
    return centres, alpha, k, relative_m2(eps, m_h)


def solve_point(mask, d, eps_dipoles, m_h, beta, r0, energy_eV, pol="ldr", tol=1e-12,
                method="auto", maxit=100000, interaction="point") -> PointResult:
    """interaction: "point" (the point-dipole G_tilde) or "igt" (the cell
    average of G_tilde for near offsets, dense LU only)."""
    centres, alpha, k, m2 = system(mask, d, eps_dipoles, m_h, energy_eV, pol)
    n = centres.shape[0]
    e = incident_field(centres, energy_eV, beta, m_h, r0)
    g = auxiliary_field(centres, energy_eV, beta, m_h, r0)
    if n == 0:
        z = np.zeros((0, 3), dtype=np.complex128)
        return PointResult(0.0, 0.0, 0.0, 0.0, z, z, 0, 0.0)
    if interaction == "igt":
        from .interaction import dense_matrix_igt, interaction_matrix_igt
        A = dense_matrix_igt(centres, alpha, k, d)
        p = np.linalg.solve(A, e.reshape(-1)).reshape(n, 3)
        res = float(np.linalg.norm(e.reshape(-1) - A @ p.reshape(-1)) / np.linalg.norm(e))
        Gp = (interaction_matrix_igt(centres, k, d) @ p.reshape(-1)).reshape(n, 3)
        return PointResult(
            p_eels=p_eels(g, p, energy_eV, beta, m_h),
            p_ext=p_ext(e, p, energy_eV, beta, m_h),
            p_abs=p_abs(p, alpha, m2, d, energy_eV, beta, m_h),
            p_cl=p_cl(p, Gp, energy_eV, beta, m_h),
            p_hat=p, e_hat=e, iters=0, residual=res,
        )
    if method == "lu" or (method == "auto" and n <= LU_MAX_DIPOLES):
        p = lu_solve(centres, alpha, k, e)
        r = e - cdense.matvec(centres, alpha, k, p)
        it, res = 0, float(np.linalg.norm(r) / np.linalg.norm(e))
    else:
        p, it, res = bicgstab(centres, alpha, k, e, tol=tol, maxit=maxit)
    Gp = cdense.matvec(centres, alpha, k, p, interaction_only=True)
    return PointResult(
        p_eels=p_eels(g, p, energy_eV, beta, m_h),
        p_ext=p_ext(e, p, energy_eV, beta, m_h),
        p_abs=p_abs(p, alpha, m2, d, energy_eV, beta, m_h),
        p_cl=p_cl(p, Gp, energy_eV, beta, m_h),
        p_hat=p, e_hat=e, iters=it, residual=res,
    )
