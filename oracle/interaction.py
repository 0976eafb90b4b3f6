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

Integrated interaction (the option the paper recommends, section S5; the
reading taken here): with the polarization constant over each cubic cell, the
field at the centre of cell i from cell j is the Green's tensor of eq. (5)
integrated over cell j (the volume integral of eqs. 4 and 8).  For a near
offset, |R| <= IGT_RADIUS d, the interaction is that cell average

    G_int(R) = d^-3 int_{cube of side d} G_tilde(R + s) d^3 s,

evaluated here by a tensor Gauss-Legendre rule (the integrand is smooth on
the source cube, whose nearest point is d/2 from the observation point);
beyond it the point value G_tilde(R), which the average approaches as
G_tilde(R) (1 - (kd)^2/24) + O((d/R)^4).  The self term (R = 0) stays with the
polarizability.
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


IGT_RADIUS = 3.0  # near offsets: |R| <= IGT_RADIUS d take the cell average


def integrated_green_tensor(R, k: complex, d: float, n: int = 32) -> np.ndarray:
    """Cell average of G_tilde over the cube of side d centred at R (R != 0,
    |R| >= d): tensor Gauss-Legendre with n nodes per axis (numpy's nodes and
    weights); returns [3, 3]."""
    u, w = np.polynomial.legendre.leggauss(n)
    s = 0.5 * d * u
    S = np.stack(np.meshgrid(s, s, s, indexing="ij"), axis=-1).reshape(-1, 3)
    W = (np.einsum("i,j,k->ijk", w, w, w) / 8.0).reshape(-1)
    G = green_tensor(np.asarray(R, dtype=np.float64)[None, :] + S, k)
    return np.einsum("n,nab->ab", W, G)


def near_offsets(radius: float = IGT_RADIUS):
    """Integer offsets o != 0 with |o| <= radius."""
    r = int(np.floor(radius))
    out = []
    for i in range(-r, r + 1):
        for j in range(-r, r + 1):
            for l in range(-r, r + 1):
                if (i, j, l) != (0, 0, 0) and i * i + j * j + l * l <= radius * radius + 1e-9:
                    out.append((i, j, l))
    return out


def interaction_matrix_igt(centres: np.ndarray, k: complex, d: float,
                           radius: float = IGT_RADIUS) -> np.ndarray:
    """The interaction part with the cell average for near offsets (lattice
    centres on a grid of spacing d)."""
    c = np.asarray(centres, dtype=np.float64)
    n = c.shape[0]
    Gm = interaction_matrix(c, k).reshape(n, 3, n, 3)
    if n < 2:
        return Gm.reshape(3 * n, 3 * n)
    table = {o: integrated_green_tensor(d * np.array(o, dtype=np.float64), k, d)
             for o in near_offsets(radius)}
    off = np.rint((c[:, None, :] - c[None, :, :]) / d).astype(int)
    for (i, j) in zip(*np.nonzero(np.sum(off * off, axis=-1) <= radius * radius + 1e-9)):
        if i != j:
            Gm[i, :, j, :] = table[tuple(off[i, j])]
    return Gm.reshape(3 * n, 3 * n)


def dense_matrix_igt(centres: np.ndarray, alpha: np.ndarray, k: complex, d: float,
                     radius: float = IGT_RADIUS) -> np.ndarray:
    n = np.asarray(centres).shape[0]
    A = -interaction_matrix_igt(centres, k, d, radius)
    A[np.arange(3 * n), np.arange(3 * n)] = np.repeat(1.0 / np.asarray(alpha, dtype=np.complex128), 3)
    return A
