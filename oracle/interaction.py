"""Dipole-dipole interaction and the dense DDA system matrix.

Discretising eq. (8) over cubic cells gives, for p_tilde = p/(4 pi eps0 m_h^2),
the field of dipole j at dipole i as G_tilde(r_i - r_j) p_tilde_j with

    G_tilde(R) = (k^2 I + grad grad) exp(ikR)/R
               = exp(ikR)/R^3 [ (k^2 R^2 + i k R - 1) I
                                + (3 - 3 i k R - k^2 R^2) R_hat R_hat ],

i.e. 4 pi k^2 times the Green's tensor of eq. (5), with k = m_h k0 the host
wavenumber (complex in an absorbing host).  The DDA system (one 3-block per
occupied cell) is

    (A p)_i = p_i / alpha_i - sum_{j != i} G_tilde(r_i - r_j) p_j = e_i .

G_tilde(R) is a symmetric tensor and even in R, so A = A^T (reciprocity,
section 2.4).
"""

from __future__ import annotations

import numpy as np


def green_tensor(R: np.ndarray, k: complex) -> np.ndarray:
    """G_tilde for separation vectors R[..., 3] (nm); returns [..., 3, 3]."""
    R = np.asarray(R, dtype=np.float64)
    r = np.sqrt(np.sum(R * R, axis=-1))
    if np.any(r == 0):
        raise ZeroDivisionError("G_tilde is singular at R = 0")
    kr = k * r
    e = np.exp(1j * kr) / r ** 3
    a = e * (kr * kr + 1j * kr - 1.0)
    b = e * (3.0 - 3.0j * kr - kr * kr)
    rh = R / r[..., None]
    G = b[..., None, None] * rh[..., :, None] * rh[..., None, :]
    idx = np.arange(3)
    G[..., idx, idx] += a[..., None]
    return G


def interaction_matrix(centres: np.ndarray, k: complex) -> np.ndarray:
    """Sum_{j != i} G_tilde(r_i - r_j) as a 3n x 3n matrix (zero diagonal
    blocks), unknown ordering 3*i + component."""
    c = np.asarray(centres, dtype=np.float64)
    n = c.shape[0]
    G = np.zeros((n, 3, n, 3), dtype=np.complex128)
    if n > 1:
        R = c[:, None, :] - c[None, :, :]
        off = ~np.eye(n, dtype=bool)
        ii, jj = np.nonzero(off)
        G[ii, :, jj, :] = green_tensor(R[off], k)
    return G.reshape(3 * n, 3 * n)


def dense_matrix(centres: np.ndarray, alpha: np.ndarray, k: complex) -> np.ndarray:
    """The full 3n x 3n system matrix A = diag(1/alpha) - G_off."""
    n = np.asarray(centres).shape[0]
    A = -interaction_matrix(centres, k)
    A[np.arange(3 * n), np.arange(3 * n)] = np.repeat(1.0 / np.asarray(alpha, dtype=np.complex128), 3)
    return A
