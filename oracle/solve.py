"""Solving the DDA system A p = e.

* Dense LU (numpy / LAPACK zgesv) on the explicit matrix for small systems.
* BiCGStab (van der Vorst 1992, complex form with the Hermitian inner
  product) with the on-the-fly dense matvec otherwise: x0 = 0, stopping when
  the true relative residual ||e - A p|| / ||e|| of the unscaled system is at
  most `tol` (the stopping threshold of the paper's iterative solver,
  section S5).
"""

from __future__ import annotations

import numpy as np

from . import cdense
from .interaction import dense_matrix


def lu_solve(centres, alpha, k, e):
    A = dense_matrix(centres, alpha, k)
    n = np.asarray(centres).shape[0]
    return np.linalg.solve(A, np.asarray(e, dtype=np.complex128).reshape(3 * n)).reshape(n, 3)


def bicgstab(centres, alpha, k, e, tol=1e-12, maxit=100000, matvec=None):
    """Returns (p [n][3], iterations, true relative residual).

    Each cycle runs BiCGStab from the current iterate until the recursively
    updated residual meets `tol`; the true residual is then recomputed and a
    new cycle starts if it drifted above `tol`.
    """
    if matvec is None:
        def matvec(v):
            return cdense.matvec(centres, alpha, k, v)
    b = np.asarray(e, dtype=np.complex128)
    nb = np.linalg.norm(b)
    x = np.zeros_like(b)
    if nb == 0:
        return x, 0, 0.0
    it = 0
    r = b.copy()
    while True:
        res = np.linalg.norm(r) / nb
        if res <= tol or it >= maxit:
            return x, it, res
        rhat = r.copy()
        rho_old = alpha_s = omega = 1.0 + 0j
        v = np.zeros_like(b)
        p = np.zeros_like(b)
        while it < maxit:
            rho = np.vdot(rhat, r)
            if rho == 0:
                break
            beta = (rho / rho_old) * (alpha_s / omega)
            p = r + beta * (p - omega * v)
            v = matvec(p)
            alpha_s = rho / np.vdot(rhat, v)
            s = r - alpha_s * v
            it += 1
            if np.linalg.norm(s) / nb <= tol:
                x = x + alpha_s * p
                break
            t = matvec(s)
            tt = np.vdot(t, t)
            omega = np.vdot(t, s) / tt if tt != 0 else 0.0
            x = x + alpha_s * p + omega * s
            r = s - omega * t
            rho_old = rho
            if omega == 0 or np.linalg.norm(r) / nb <= tol:
                break
        r = b - matvec(x)
