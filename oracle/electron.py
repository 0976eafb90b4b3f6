"""The fast electron: kinematics and incident/auxiliary fields (section 2.2,
eqs. 20-25; section 2.4, eq. 34; section 2.7, eq. 47).

Fields are returned as dimensionless shapes.  The physical incident field is
E_inc = C * e_hat with C = q omega / (2 pi eps0 m_h^2 v^2 gamma_h) (eq. 25);
C cancels from every loss probability once the prefactor in losses.py is
applied.
"""

from __future__ import annotations

import numpy as np
from scipy import special

from .constants import HBAR_C_EV_NM, ME_C2_KEV


def beta_from_kev(kinetic_keV: float) -> float:
    """v/c of an electron with the given kinetic energy (special relativity)."""
    gamma = 1.0 + kinetic_keV / ME_C2_KEV
    return float(np.sqrt(1.0 - 1.0 / (gamma * gamma)))


def kev_for_host_scaling(kinetic_keV: float, eps_h: float) -> float:
    """Kinetic energy whose speed is m_h times that of `kinetic_keV` (eq. 47).

    eps_h = m_h^2 is the (real) relative permittivity of the host.
    """
    E, E0 = kinetic_keV, ME_C2_KEV
    return float(E0 * ((E + E0) / np.sqrt(E0 * E0 - (eps_h - 1.0) * E * (2.0 * E0 + E)) - 1.0))


def beta_h(beta: float, m_h: complex) -> complex:
    """beta_h = (v/c) m_h (eq. 24)."""
    return complex(beta) * complex(m_h)


def gamma_h(beta: float, m_h: complex) -> complex:
    """gamma_h = (1 - beta_h^2)^(-1/2) on the branch of eq. (24).

    The branch is the one continuous in eps_h over 0 <= arg eps_h < pi, which
    puts gamma_h in the first quadrant: real > 1 for real beta_h < 1 and
    positive imaginary for real beta_h > 1.  Written as i / sqrt(beta_h^2 - 1)
    with the principal root, whose argument beta_h^2 - 1 lies in the closed
    upper half plane; a signed zero in its imaginary part is forced to +0 so
    that the real beta_h < 1 case lands on +i sqrt(1 - beta_h^2).
    """
    bh = beta_h(beta, m_h)
    w = bh * bh - 1.0
    if abs(w) < 1e-12:
        raise ZeroDivisionError("beta_h = 1: the electron field is singular (eq. 24)")
    w = complex(w.real, abs(w.imag)) if w.imag == 0.0 else w
    if w.imag < 0:
        raise ValueError("passive host required: Im(beta_h^2) >= 0")
    return 1j / np.sqrt(w)


def k0_of(energy_eV: float) -> float:
    """Vacuum wavenumber k0 = omega/c in 1/nm for a loss energy in eV."""
    return energy_eV / HBAR_C_EV_NM


def transverse_wavenumber(energy_eV: float, beta: float, m_h: complex) -> complex:
    """k_t = omega / (gamma_h v) (eq. S9), the Bessel-argument scale of eq. (25)."""
    return k0_of(energy_eV) / (beta * gamma_h(beta, m_h))


def besselk01(z: np.ndarray):
    """K0(z), K1(z) for complex z with Re z >= 0 (scipy / AMOS)."""
    z = np.asarray(z, dtype=np.complex128)
    return special.kv(0, z), special.kv(1, z)


def _geometry(centres: np.ndarray, r0):
    c = np.asarray(centres, dtype=np.float64).reshape(-1, 3)
    x0, y0, z0 = (float(v) for v in np.asarray(r0, dtype=np.float64).reshape(3))
    dx = c[:, 0] - x0
    dy = c[:, 1] - y0
    dz = c[:, 2] - z0
    b = np.hypot(dx, dy)
    return dx, dy, dz, b


def incident_field(centres: np.ndarray, energy_eV: float, beta: float, m_h: complex,
                   r0) -> np.ndarray:
    """Shape e_hat of the electron's incident field at each dipole (eq. 25).

    e_hat = exp(i omega (z - z0)/v) * ( (x-x0)/b K1(k_t b),
                                        (y-y0)/b K1(k_t b),
                                        -(i/gamma_h) K0(k_t b) ),
    for an electron moving along +z through r0 (eqs. 20-21).
    Returns complex128 [n][3].
    """
    g = gamma_h(beta, m_h)
    k0 = k0_of(energy_eV)
    kt = k0 / (beta * g)
    dx, dy, dz, b = _geometry(centres, r0)
    if b.size and np.min(b) <= 0.0:
        raise ZeroDivisionError("trajectory passes through a dipole centre (b = 0)")
    K0, K1 = besselk01(kt * b)
    phase = np.exp(1j * k0 * dz / beta)
    e = np.empty((b.size, 3), dtype=np.complex128)
    e[:, 0] = phase * (dx / b) * K1
    e[:, 1] = phase * (dy / b) * K1
    e[:, 2] = phase * (-1j / g) * K0
    return e


def auxiliary_field(centres: np.ndarray, energy_eV: float, beta: float, m_h: complex,
                    r0) -> np.ndarray:
    """Shape g_hat of the auxiliary field of the conjugate source (eq. 34).

    g_hat = (-e_x, -e_y, +e_z) * exp(-2 i omega (z - z0)/v), in the same
    normalisation as `incident_field`.
    """
    e = incident_field(centres, energy_eV, beta, m_h, r0)
    dz = _geometry(centres, r0)[2]
    ph = np.exp(-2j * k0_of(energy_eV) * dz / beta)
    g = np.empty_like(e)
    g[:, 0] = -e[:, 0] * ph
    g[:, 1] = -e[:, 1] * ph
    g[:, 2] = e[:, 2] * ph
    return g
