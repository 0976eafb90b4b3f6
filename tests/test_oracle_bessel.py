"""Pins for the oracle's K0/K1 at complex arguments (eq. 25 needs them for
arg z in [-pi/2, 0]: absorbing, non-absorbing and Cherenkov hosts)."""

import mpmath as mp
import numpy as np
import pytest

from oracle import electron as el


def _grid():
    for r in np.geomspace(1e-4, 50.0, 23):
        for th in np.linspace(-np.pi / 2, 0.0, 9):
            yield r * np.exp(1j * th)


def test_scipy_k01_against_mpmath():
    mp.mp.dps = 30
    zs = np.array(list(_grid()))
    K0, K1 = el.besselk01(zs)
    for z, a0, a1 in zip(zs, K0, K1):
        r0 = complex(mp.besselk(0, z))
        r1 = complex(mp.besselk(1, z))
        assert abs(a0 - r0) <= 1e-13 * abs(r0)
        assert abs(a1 - r1) <= 1e-13 * abs(r1)


@pytest.mark.parametrize("m_h,beta,b", [(1.5 + 0.3j, 0.55, 4.0), (2.0 + 0.2j, 0.7, 3.0),
                                        (1.2 + 0.05j, 0.5, 10.0)])
def test_integral_representation_s8(m_h, beta, b):
    """Eq. (S8)-(S9): for Im beta_h > 0 the line integral
    I_S(b) = int du exp[i (omega b / v)(beta_h cosh u - sinh u)] equals
    2 K0(k_t b), k_t = omega/(gamma_h v).  The integrand decays doubly
    exponentially, so plain quadrature of it pins both K0 and the branch of
    gamma_h chosen in eq. (24)."""
    mp.mp.dps = 30
    energy = 2.0
    k0 = energy / 197.3269804
    wb = mp.mpf(k0 / beta * b)  # omega b / v
    bh = mp.mpc(beta * m_h)

    def f(u):
        return mp.exp(1j * wb * (bh * mp.cosh(u) - mp.sinh(u)))

    val = mp.quad(f, mp.linspace(-12, 12, 49))
    kt = el.transverse_wavenumber(energy, beta, m_h)
    K0, _ = el.besselk01(np.array([kt * b]))
    assert abs(complex(val) - 2 * K0[0]) <= 1e-11 * abs(2 * K0[0])


def test_imaginary_axis_hankel_relation():
    """Eqs. (S9)/(S13): for a non-absorbing Cherenkov host the argument is
    -i x (x > 0) and K0(-i x) = (pi i / 2) H0^(1)(x)."""
    mp.mp.dps = 30
    for x in [0.01, 0.3, 1.0, 2.5, 7.0, 20.0]:
        K0, K1 = el.besselk01(np.array([-1j * x]))
        h0 = complex(mp.hankel1(0, x))
        assert abs(K0[0] - 0.5j * np.pi * h0) <= 1e-13 * abs(h0)
