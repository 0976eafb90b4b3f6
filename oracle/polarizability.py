"""Dipole polarizabilities.

The paper names the polarizability as an option of the DDA code (section S5)
without giving formulas, so these follow the DDA literature, in the
normalisation of eqs. (7)-(8): with p_tilde = p / (4 pi eps0 m_h^2) the dipole
obeys p_tilde = alpha * E_exc, alpha in nm^3, and m = m_p / m_h is the
relative refractive index of eq. (2).

* Clausius-Mossotti: alpha = (3 d^3 / 4 pi) (m^2 - 1)/(m^2 + 2).
* Radiative reaction: alpha_CM / (1 - (2/3) i k^3 alpha_CM).
* Lattice dispersion relation (Draine & Goodman 1993):
  alpha_CM / (1 + (alpha_CM/d^3) [ (b1 + m^2 b2 + m^2 b3 S)(kd)^2
                                   - (2/3) i (kd)^3 ]),
  b1 = -1.8915316, b2 = 0.1648469, b3 = -1.7700004.  S = sum_mu a_mu^2 e_mu^2
  for propagation a and polarisation e; for the electron moving along the
  lattice z axis with its transverse field, S = 0 (the reading taken
  here).  The coefficient values are literature constants: parity unpinned
  for the values themselves.
"""

from __future__ import annotations

import numpy as np

LDR_B1 = -1.8915316
LDR_B2 = 0.1648469
LDR_B3 = -1.7700004


def relative_m2(eps_particle: np.ndarray, m_h: complex) -> np.ndarray:
    """m^2 = eps_p / m_h^2 with eps_p the absolute particle permittivity (eq. 2)."""
    return np.asarray(eps_particle, dtype=np.complex128) / (complex(m_h) ** 2)


def alpha_cm(m2: np.ndarray, d: float) -> np.ndarray:
    return (3.0 * d ** 3 / (4.0 * np.pi)) * (m2 - 1.0) / (m2 + 2.0)


def alpha_rr(m2: np.ndarray, d: float, k: complex) -> np.ndarray:
    a = alpha_cm(m2, d)
    return a / (1.0 - (2.0 / 3.0) * 1j * k ** 3 * a)


def alpha_ldr(m2: np.ndarray, d: float, k: complex, S: float = 0.0) -> np.ndarray:
    a = alpha_cm(m2, d)
    kd = k * d
    corr = (LDR_B1 + m2 * LDR_B2 + m2 * LDR_B3 * S) * kd ** 2 - (2.0 / 3.0) * 1j * kd ** 3
    return a / (1.0 + (a / d ** 3) * corr)


def polarizability(kind: str, eps_particle: np.ndarray, m_h: complex, d: float,
                   k: complex) -> np.ndarray:
    m2 = relative_m2(eps_particle, m_h)
    kind = kind.lower()
    if kind == "cm":
        return alpha_cm(m2, d)
    if kind == "rr":
        return alpha_rr(m2, d, k)
    if kind == "ldr":
        return alpha_ldr(m2, d, k)
    raise ValueError(f"unknown polarizability {kind!r}")
