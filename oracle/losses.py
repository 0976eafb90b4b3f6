"""Loss and emission probabilities from the DDA solution (sections 2.4-2.6).

With E_inc = C e_hat (eq. 25), the DDA unknowns p_hat solve A p_hat = e_hat
and the SI dipole moments are p = 4 pi eps0 m_h^2 C p_hat (eqs. 7-8 and the
normalisation in interaction.py).  Substituting into the powers and using
q^2/(4 pi eps0) = alpha_fs hbar c, omega = c k0, v = beta c, every probability
(per unit loss energy, in 1/eV) carries the common factor

    Pi = 4 alpha_fs k0^2 / (pi hbar c beta^4)        [1/(eV nm^3)]

and (the charge sign drops out, q^2):

* P_EELS (eqs. 32, 34, 37, 38), bilinear dot without conjugation:
      P_EELS = -Pi Im[ sum_i g_hat_i . p_hat_i / (m_h gamma_h)^2 ]
* P_ext (eqs. 17, 48):
      P_ext  =  Pi Im[ m_h^2 sum_i conj(e_hat_i) . p_hat_i ] / (|m_h|^4 |gamma_h|^2)
* P_abs (eq. 18), one formula for every host.  Eq. (18) integrates
  Im(eps) |E|^2 over the particle; with the DDA's cell relation
  P = (eps - eps_h) E (eq. 7), the field in cell i is
  E_i = 4 pi p_hat_i / ((m_i^2 - 1) d^3) in the normalisation above, which
  gives the weight  w18_i = 4 pi Im(m_h^2 m_i^2) / (|m_i^2 - 1|^2 d^3).
  The polarizability prescription changes the work the exciting field
  E_exc = p/alpha does on the dipole, Im(m_h^2 conj(1/alpha)) |p|^2, from its
  Clausius-Mossotti value, and part of that work is radiated (the self term
  of P_CL below).  Both corrections are added:
      w_i = w18_i + Im(m_h^2 conj(1/alpha_i - 1/alpha_CM,i))
                  - Re(m_h^2) (2/3) Re(k)^3
      P_abs = Pi/(|m_h|^4 |gamma_h|^2) sum_i w_i |p_hat_i|^2
  The weight is continuous in m_h (Im m_h -> 0+ gives the real-host value);
  the corrections vanish as d -> 0, so it tends to eq. (18) on any host; in a
  real host it is the DDA's discrete absorption sum_i [-Im(1/alpha_i)
  - (2/3) k^3] |p_hat_i|^2 m_h^2 (Draine's form), which with P_CL below makes
  P_ext = P_abs + P_CL an identity of the discrete system.  In an absorbing
  host that budget is off by
      Pi/(|m_h|^4 |gamma_h|^2) Im(m_h^2) [ (4 pi/d^3) sum_i (1/3 - 1/|m_i^2-1|^2) |p_hat_i|^2
                                          - Re(p_hat^H G_off p_hat) ],
  the host's own absorption that eqs. (16)-(18) leave ambiguous (section 2.2).
* P_CL (eq. 42), the power radiated by the dipoles, real host:
      P_CL   =  Pi/(m_h^2 |gamma_h|^2) [ Im(p_hat^H G_off p_hat) + (2/3) k^3 ||p_hat||^2 ]
  absorbing host: the same expression with m_h^2 -> Re(m_h^2) and k -> Re(k)
  in the self term, a nominal value (the paper calls CL in an absorbing host
  qualitative, section 2.6).
"""

from __future__ import annotations

import numpy as np

from .constants import ALPHA_FS, HBAR_C_EV_NM
from .electron import gamma_h, k0_of
from .polarizability import alpha_cm


def prefactor(energy_eV: float, beta: float) -> float:
    k0 = k0_of(energy_eV)
    return 4.0 * ALPHA_FS * k0 * k0 / (np.pi * HBAR_C_EV_NM * beta ** 4)


def p_eels(g_hat, p_hat, energy_eV, beta, m_h) -> float:
    g = gamma_h(beta, m_h)
    s = np.sum(np.asarray(g_hat) * np.asarray(p_hat))
    return float(-prefactor(energy_eV, beta) * np.imag(s / (complex(m_h) * g) ** 2))


def p_ext(e_hat, p_hat, energy_eV, beta, m_h) -> float:
    g = gamma_h(beta, m_h)
    mh = complex(m_h)
    s = np.sum(np.conj(np.asarray(e_hat)) * np.asarray(p_hat))
    return float(prefactor(energy_eV, beta) * np.imag(mh * mh * s) / (abs(mh) ** 4 * abs(g) ** 2))


def absorption_weight(alpha, m2, d, energy_eV, m_h) -> np.ndarray:
    """w_i of P_abs = Pi/(|m_h|^4 |gamma_h|^2) sum_i w_i |p_hat_i|^2 (eq. 18 with
    the cell relation of eq. 7, plus the polarizability's corrections)."""
    mh2 = complex(m_h) ** 2
    m2 = np.asarray(m2, dtype=np.complex128)
    kr = (complex(m_h) * k0_of(energy_eV)).real
    w18 = 4.0 * np.pi * np.imag(mh2 * m2) / (np.abs(m2 - 1.0) ** 2 * d ** 3)
    corr = np.conj(1.0 / np.asarray(alpha, dtype=np.complex128) - 1.0 / alpha_cm(m2, d))
    return w18 + np.imag(mh2 * corr) - mh2.real * (2.0 / 3.0) * kr ** 3


def p_abs(p_hat, alpha, m2, d, energy_eV, beta, m_h) -> float:
    g = gamma_h(beta, m_h)
    mh = complex(m_h)
    Pi = prefactor(energy_eV, beta)
    p2 = np.sum(np.abs(np.asarray(p_hat)) ** 2, axis=-1)  # |p_i|^2 per dipole
    w = absorption_weight(alpha, m2, d, energy_eV, m_h)
    return float(Pi / (abs(mh) ** 4 * abs(g) ** 2) * np.sum(w * p2))


def p_cl(p_hat, Gp_hat, energy_eV, beta, m_h) -> float:
    """Gp_hat = G_off p_hat (interaction part of A applied to p_hat)."""
    g = gamma_h(beta, m_h)
    mh = complex(m_h)
    Pi = prefactor(energy_eV, beta)
    p = np.asarray(p_hat)
    k = (mh * k0_of(energy_eV)).real
    quad = np.imag(np.vdot(p, np.asarray(Gp_hat))) + (2.0 / 3.0) * k ** 3 * np.vdot(p, p).real
    return float(Pi * (mh * mh).real / (abs(mh) ** 4 * abs(g) ** 2) * quad)
