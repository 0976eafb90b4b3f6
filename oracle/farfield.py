"""Far-field radiation of the dipoles and CL resolved over directions (test
infrastructure: only the tests, the smoke check and the benchmark's CPU leg
use this package).

CL is the power scattered by the particle (eq. 42, section 2.6), and the
paper notes that a detector collects it only over some solid angle.  Far from
the particle, the field of the dipoles (p_tilde normalisation of
interaction.py, G_tilde = (k^2 I + grad grad) e^{ikR}/R) in direction n is

    E_sca ~ (e^{ikr}/r) k^2 (I - n n) A(n),   A(n) = sum_j p_j exp(-i k n . r_j),

for a real host wavenumber k = m_h k0.  Since
Im G_tilde(R) = (k^3/4pi) * integral over the sphere of (I - n n) e^{i k n.R},
the quadratic form in P_CL (losses.py) is the angular integral

    Im(p^H G_off p) + (2/3) k^3 ||p||^2 = (k^3/4pi) integral |(I - n n) A(n)|^2 dOmega,

so per unit solid angle

    dP_CL/dOmega(n) = Pi/(m_h^2 |gamma_h|^2) * (k^3/4pi) * |(I - n n) A(n)|^2

and a quadrature (n_q, w_q) with sum w_q = 4pi gives P_CL; over a detector's
directions it gives the collected signal.  Absorbing hosts are excluded: the
far field decays there and the paper calls CL in them qualitative.
"""

from __future__ import annotations

import numpy as np

from .electron import gamma_h, k0_of
from .losses import prefactor


def amplitudes(centres: np.ndarray, p_hat: np.ndarray, k: float, dirs: np.ndarray) -> np.ndarray:
    """A(n_q) = sum_j p_j exp(-i k n_q . r_j): [n_dir][3] for p_hat [n_occ][3]."""
    E = np.exp(-1j * k * (np.asarray(dirs, dtype=np.float64) @ np.asarray(centres).T))
    return E @ np.asarray(p_hat)


def transverse_intensity(A: np.ndarray, dirs: np.ndarray) -> np.ndarray:
    """|(I - n n) A|^2 = |A|^2 - |n . A|^2 per direction."""
    n = np.asarray(dirs, dtype=np.float64)
    nA = np.sum(n * A, axis=-1)
    return np.sum(np.abs(A) ** 2, axis=-1) - np.abs(nA) ** 2


def dp_domega(centres, p_hat, dirs, energy_eV: float, beta: float, m_h) -> np.ndarray:
    mh = complex(m_h)
    if mh.imag != 0.0:
        raise ValueError("far-field CL needs a non-absorbing host")
    k = mh.real * k0_of(energy_eV)
    g = gamma_h(beta, mh)
    A = amplitudes(centres, p_hat, k, dirs)
    scale = prefactor(energy_eV, beta) / (mh.real ** 2 * abs(g) ** 2) * k ** 3 / (4.0 * np.pi)
    return scale * transverse_intensity(A, dirs)


def sphere_rule(n_theta: int, n_phi: int):
    """Product quadrature on the unit sphere: Gauss-Legendre in cos(theta),
    equispaced phi.  Exact for spherical harmonics of degree < min(2 n_theta,
    n_phi).  Returns (dirs [n][3], weights [n]) with sum(weights) = 4 pi."""
    x, wx = np.polynomial.legendre.leggauss(n_theta)
    phi = 2.0 * np.pi * np.arange(n_phi) / n_phi
    st = np.sqrt(1.0 - x * x)
    d = np.stack([np.outer(st, np.cos(phi)), np.outer(st, np.sin(phi)),
                  np.outer(x, np.ones(n_phi))], axis=-1).reshape(-1, 3)
    w = np.outer(wx, np.full(n_phi, 2.0 * np.pi / n_phi)).reshape(-1)
    return d, w
