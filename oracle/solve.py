"""Solving the DDA system A p = e.

* Dense LU (numpy / LAPACK zgesv) on the explicit matrix for small systems.
* BiCGStab (van der Vorst 1992, complex form with the Hermitian inner
  product) with the on-the-fly dense matvec otherwise: x0 = 0, stopping when
  the true relative residual ||e - A p|| / ||e|| of the unscaled system is at
  most `tol` (the stopping threshold of the paper's iterative solver,
  section S5).
* QMR for complex-symmetric matrices (the paper's recommended solver family,
  section S5; Freund 1992): the Lanczos process of the bilinear form x^T y,
  which A = A^T (reciprocity, section 2.4) turns into a three-term
  recurrence, with vectors scaled to unit 2-norm, and the quasi-minimal
  residual solution from Givens rotations of its tridiagonal matrix.
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


def _givens(a: complex, b: float):
    """(c, s, r) with [c s; -conj(s) c] (a, b)^T = (r, 0), c real >= 0, b real."""
    if a == 0:
        return 0.0, 1.0 + 0j, complex(b)
    nu = np.hypot(abs(a), b)
    ph = a / abs(a)
    return abs(a) / nu, ph * b / nu, ph * nu


def qmr_cs(centres, alpha, k, e, tol=1e-12, maxit=100000, matvec=None, callback=None):
    """QMR for the complex-symmetric system A p = e from p0 = 0.  Returns
    (p, iterations, true relative residual).

    Lanczos for the bilinear form: v_1 = r0/||r0||, and for n = 1, 2, ...
        u = A v_n, delta_n = v_n^T v_n, alpha_n = v_n^T u / delta_n,
        beta_n = rho_n delta_n / delta_{n-1} (0 for n = 1),
        w = u - alpha_n v_n - beta_n v_{n-1}, rho_{n+1} = ||w||, v_{n+1} = w/rho_{n+1},
    so that A V_n = V_{n+1} H_n with H_n tridiagonal (column n: beta_n,
    alpha_n, rho_{n+1}).  The iterate minimises ||rho_1 e_1 - H_n y||; the
    rotations that reduce H_n to triangular form also give the update
    directions p_n and the quasi-residual tau_{n+1}; since every v has unit
    norm, ||e - A p_n|| <= sqrt(n + 1) |tau_{n+1}|.  A cycle ends when that
    bound meets tol ||e||; the true residual is then recomputed and a new
    cycle starts from it if it is still above tol.  callback(n, x, tau), if
    given, sees the iterate and the quasi-residual after iteration n of a
    cycle."""
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
        rho = np.linalg.norm(r)
        v = r / rho
        v_prev = np.zeros_like(b)
        delta_prev = 1.0 + 0j
        delta = np.sum(v * v)
        p1 = np.zeros_like(b)   # p_{n-1}
        p2 = np.zeros_like(b)   # p_{n-2}
        c1, s1 = 1.0, 0j        # G_{n-1}
        c2, s2 = 1.0, 0j        # G_{n-2}
        tau = complex(rho)
        n = 0
        while it < maxit:
            n += 1
            it += 1
            if delta == 0:
                break  # Lanczos breakdown: restart from the true residual
            u = matvec(v)
            a = np.sum(v * u) / delta
            beta = rho * delta / delta_prev if n > 1 else 0j
            w = u - a * v - beta * v_prev
            rho_next = np.linalg.norm(w)
            # column n of H through the previous rotations
            eps = s2 * beta
            th = c2 * beta
            d2 = c1 * th + s1 * a
            gam = -np.conj(s1) * th + c1 * a
            c, s, rr = _givens(gam, rho_next)
            if rr == 0:
                break
            p = (v - d2 * p1 - eps * p2) / rr
            x = x + (c * tau) * p
            tau = -np.conj(s) * tau
            if callback is not None:
                callback(n, x, tau)
            p2, p1 = p1, p
            c2, s2, c1, s1 = c1, s1, c, s
            if rho_next == 0 or np.sqrt(n + 1) * abs(tau) <= tol * nb:
                break
            v_prev, v = v, w / rho_next
            rho = rho_next
            delta_prev, delta = delta, np.sum(v * v)
        r = b - matvec(x)
