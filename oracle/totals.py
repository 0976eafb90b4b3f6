"""Total-loss quantities around the particle-induced probabilities (test
infrastructure: only the tests, the smoke check and the benchmark's CPU leg
use this package).

* Free-space loss of the electron in a non-absorbing host (section 2.3).  Eq.
  (29) gives the power lost per unit path length, dW_0/dz = (mu0/8) q^2 omega
  (1 - c^2/(v^2 m_h^2)) for beta_h = beta m_h > 1 (zero below the Cherenkov
  threshold), and eq. (36) turns a power W into a probability per unit loss
  energy, Gamma = (2/pi) W / (hbar^2 omega).  Combined:
      d Gamma_0/dz = (2/pi) (mu0/8) q^2 (1 - 1/beta_h^2) / hbar^2
                   = alpha_fs (1 - 1/beta_h^2) / (hbar c)
  with mu0 q^2 c / (4 pi hbar) = alpha_fs.  Here it is evaluated in SI units
  straight from the first form, then converted to 1/(eV nm).
* P_CL^tot (eq. 41) = the common prefactor of eqs. (37), (42), (48) times
  C_enh - C_ext + C_sca, i.e. P_EELS - P_ext + P_CL.
* Gaussian broadening of a spectrum on a uniform energy grid, the spectrum
  taken as zero outside the grid: out_i = sum_j p_j g(E_i - E_j) dE, g of unit
  area and the given full width at half maximum.
"""

from __future__ import annotations

import numpy as np

# SI constants (CODATA 2018, exact where the SI fixes them)
MU0 = 1.25663706212e-6            # N A^-2
Q_E = 1.602176634e-19             # C
HBAR = 1.054571817e-34            # J s
EV = 1.602176634e-19              # J


def free_space_loss_per_nm(beta: float, m_h: complex) -> float:
    """d Gamma_0 / dz in 1/(eV nm); zero for beta_h <= 1.  Undefined (raises)
    in an absorbing host, where W_0 diverges (section 2.3)."""
    mh = complex(m_h)
    if mh.imag != 0.0:
        raise ValueError("W_0 is undefined in an absorbing host")
    bh = beta * mh.real
    if bh <= 1.0:
        return 0.0
    # eq. (29) per unit omega, then eq. (36): (2/pi) * (mu0/8) q^2 (1 - 1/bh^2) / hbar^2
    per_m_per_J = (2.0 / np.pi) * (MU0 / 8.0) * Q_E ** 2 * (1.0 - 1.0 / bh ** 2) / HBAR ** 2
    return per_m_per_J * EV * 1e-9   # 1/(J m) -> 1/(eV nm)


def cl_total(P_eels: float, P_ext: float, P_cl: float) -> float:
    """Eq. (41) from the probabilities of eqs. (37), (48), (42)."""
    return P_eels - P_ext + P_cl


def psf_gauss(energy_eV, p, fwhm_eV: float) -> np.ndarray:
    E = np.asarray(energy_eV, dtype=np.float64)
    v = np.asarray(p, dtype=np.float64)
    if E.size == 1:
        return v.copy()
    dE = (E[-1] - E[0]) / (E.size - 1)
    sigma = fwhm_eV / (2.0 * np.sqrt(2.0 * np.log(2.0)))
    out = np.empty_like(v)
    for i in range(E.size):
        acc = 0.0
        for j in range(E.size):
            u = (E[i] - E[j]) / sigma
            acc += v[j] * np.exp(-0.5 * u * u) / (sigma * np.sqrt(2.0 * np.pi)) * dE
        out[i] = acc
    return out
