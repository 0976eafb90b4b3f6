"""Synthetic particle permittivities.

The paper's optical data for silver and gold are not available, so the
workloads use a Drude model of the same plasmonic character (negative real
part with a small loss over the 1-4 eV range the paper's spectra cover).
"""

from __future__ import annotations

import numpy as np


def drude_eps(energy_eV, eps_inf: float = 9.5, omega_p_eV: float = 9.0,
              gamma_eV: float = 0.07) -> np.ndarray:
    """eps(E) = eps_inf - omega_p^2 / (E (E + i gamma)), E in eV (absolute)."""
    E = np.asarray(energy_eV, dtype=np.float64)
    return eps_inf - omega_p_eV ** 2 / (E * (E + 1j * gamma_eV))


def uniform_eps(n_occ: int, eps: complex) -> np.ndarray:
    """Same absolute permittivity at every occupied dipole."""
    return np.full(n_occ, complex(eps), dtype=np.complex128)
