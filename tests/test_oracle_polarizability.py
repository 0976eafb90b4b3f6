"""Pins for the dipole polarizabilities (limits and the optical theorem)."""

import numpy as np
import pytest

from oracle import polarizability as P


def test_dilute_limit_follows_eq7():
    """For m -> 1 the cell's dipole is its polarisation density times its
    volume, P = (eps - eps_h) E (eq. 7); in the normalisation
    p_tilde = p/(4 pi eps0 m_h^2) that is alpha -> d^3 (m^2 - 1)/(4 pi)."""
    d = 2.0
    for dm in [1e-6 + 0j, 1e-6j, -1e-6 + 1e-6j]:
        m2 = np.array([1.0 + dm])
        a = P.alpha_cm(m2, d)[0]
        ref = d ** 3 * dm / (4 * np.pi)
        assert abs(a - ref) <= 1e-5 * abs(ref)


@pytest.mark.parametrize("kind", ["rr", "ldr"])
def test_optical_theorem_for_lossless_dipole(kind):
    """A non-absorbing dipole in a lossless host must radiate exactly what it
    extinguishes: Im(1/alpha) = -(2/3) k^3 (radiative reaction)."""
    d = 1.3
    for m2 in [2.25, 4.0, -5.0, 0.5]:
        for k in [0.01, 0.1, 0.4]:
            a = P.polarizability(kind, np.array([m2 * 1.45 ** 2]), 1.45, d, k)[0]
            assert np.imag(1.0 / a) == pytest.approx(-(2.0 / 3.0) * k ** 3, rel=1e-12, abs=1e-18)


def test_ldr_and_rr_reduce_to_cm_for_small_kd():
    d = 1.0
    m2 = np.array([-10.0 + 1.0j, 2.5 + 0.1j])
    cm = P.alpha_cm(m2, d)
    for kind in ["rr", "ldr"]:
        prev = None
        for k in [1e-2, 1e-3, 1e-4]:
            rel = np.max(np.abs(P.polarizability(kind, m2 * 4.0, 2.0, d, k) - cm) / np.abs(cm))
            if prev is not None:
                assert rel < prev / 50  # at least second order in kd
            prev = rel
        assert prev < 1e-6


def test_relative_index_uses_host():
    """eq. (2): m = m_p / m_h."""
    m2 = P.relative_m2(np.array([4.0 + 0.4j]), 1.6 + 0.1j)
    assert m2[0] == pytest.approx((4.0 + 0.4j) / (1.6 + 0.1j) ** 2)
