"""Pins for the electron kinematics and fields (section 2.2, eqs. 22-25;
section 2.4, eq. 34; section 2.7, eq. 47; section S4, eq. S15)."""

import json
import os

import mpmath as mp
import numpy as np
import pytest

from oracle import electron as el

HERE = os.path.dirname(os.path.abspath(__file__))
HBARC = 197.3269804


def _printed():
    with open(os.path.join(HERE, "golden", "paper_printed_values.json")) as f:
        return json.load(f)


def test_printed_beta_values():
    g = _printed()
    b = el.beta_from_kev(g["beta_100keV"]["kinetic_keV"])
    assert round(b, g["beta_100keV"]["decimals"]) == g["beta_100keV"]["value"]
    e = g["beta_h_100keV_mh2"]
    assert round(b * e["m_h"], e["decimals"]) == pytest.approx(e["value"])
    e = g["beta_h_100keV_mh1p45"]
    assert round(b * e["m_h"], e["decimals"]) == pytest.approx(e["value"])
    e = g["light_speed_mh2"]
    assert round(1.0 / e["m_h"], e["decimals"]) == e["value"]


@pytest.mark.parametrize("E", [30.0, 100.0, 200.0])
@pytest.mark.parametrize("m_h", [1.2, 1.45])
def test_eq47_kinetic_energy_rescaling(E, m_h):
    """Eq. (47) maps the kinetic energy to the one whose speed is m_h v."""
    b = el.beta_from_kev(E)
    if m_h * b >= 1:
        pytest.skip("no vacuum equivalent")
    E2 = el.kev_for_host_scaling(E, m_h * m_h)
    assert el.beta_from_kev(E2) == pytest.approx(m_h * b, rel=1e-12)


def test_gamma_h_branch():
    """Eq. (24): gamma_h in the first quadrant, real > 1 for beta_h < 1,
    positive imaginary for beta_h > 1, continuous as Im m_h -> 0+."""
    for beta in [0.3, 0.55, 0.7, 0.9]:
        for mre in np.linspace(1.0, 2.5, 16):
            for mim in [0.0, 1e-9, 1e-3, 0.1, 0.5]:
                mh = mre + 1j * mim
                if abs((beta * mh) ** 2 - 1) < 1e-6:
                    continue
                g = el.gamma_h(beta, mh)
                assert g.real >= 0 and g.imag >= 0
                if mim == 0.0:
                    if beta * mre < 1:
                        assert g.imag == 0 and g.real > 1
                    else:
                        assert g.real == 0 and g.imag > 0
                    g2 = el.gamma_h(beta, mre + 1e-12j)
                    assert abs(g2 - g) <= 1e-6 * abs(g)
    with pytest.raises(ZeroDivisionError):
        el.gamma_h(0.5, 2.0)


def test_gamma_h_signed_zero():
    """A -0 imaginary part must not flip real gamma_h to negative."""
    mh = complex(1.45, -0.0)
    g = el.gamma_h(0.55, mh)
    assert g.real > 1 and g.imag == 0


@pytest.mark.parametrize("m_h,beta", [(1.0, 0.55), (1.45, 0.55), (2.0, 0.55),
                                      (1.5 + 0.2j, 0.6), (2.0 + 0.01j, 0.7)])
def test_incident_field_from_potential_derivatives(m_h, beta):
    """Eq. (25) against eqs. (22)-(23) differentiated numerically.

    With J = exp(i omega (z - z0)/v) K0(k_t b) (eq. 23 up to q/2pi), eq. (22)
    gives E = i omega mu0 (q/2pi) (e_z J + grad(d_z J)/k^2); divided by the
    normalisation C of eq. (25) this is
    e_hat = i beta_h^2 gamma_h (e_z J + grad(d_z J)/k^2).
    """
    mp.mp.dps = 40
    E = 2.3
    k0 = E / HBARC
    g = el.gamma_h(beta, m_h)
    bh = beta * m_h
    kt = mp.mpc(el.transverse_wavenumber(E, beta, m_h))
    k = mp.mpc(m_h * k0)
    r0 = (1.3, -0.7, 2.1)

    def J(x, y, z):
        b = mp.sqrt((x - r0[0]) ** 2 + (y - r0[1]) ** 2)
        return mp.exp(1j * k0 / beta * (z - r0[2])) * mp.besselk(0, kt * b)

    pts = np.array([[6.0, 2.0, -3.0], [-4.5, 7.5, 4.0], [1.3 + 9.0, -0.7, 10.0]])
    e_or = el.incident_field(pts, E, beta, m_h, r0)
    for p, eo in zip(pts, e_or):
        x, y, z = (mp.mpf(v) for v in p)
        Jv = J(x, y, z)
        dxz = mp.diff(J, (x, y, z), (1, 0, 1))
        dyz = mp.diff(J, (x, y, z), (0, 1, 1))
        dzz = mp.diff(J, (x, y, z), (0, 0, 2))
        pre = 1j * mp.mpc(bh) ** 2 * mp.mpc(g)
        num = [pre * dxz / k ** 2, pre * dyz / k ** 2, pre * (Jv + dzz / k ** 2)]
        for a in range(3):
            assert abs(complex(num[a]) - eo[a]) <= 1e-10 * max(abs(eo[a]), 1e-300)


def test_aux_field_is_minus_conjugate_iff_gamma_real():
    """Section 2.4: E_a = -E_inc^* exactly when gamma_h is real (beta_h < 1)."""
    rng = np.random.default_rng(3)
    pts = rng.uniform(-10, 10, size=(40, 3))
    r0 = (14.0, 0.5, -2.0)
    e = el.incident_field(pts, 2.0, 0.55, 1.45, r0)
    a = el.auxiliary_field(pts, 2.0, 0.55, 1.45, r0)
    assert np.max(np.abs(a + np.conj(e))) <= 1e-14 * np.max(np.abs(e))
    # Cherenkov (gamma_h imaginary) and absorbing hosts: not equal
    for mh in [2.0, 1.45 + 0.1j]:
        e = el.incident_field(pts, 2.0, 0.55, mh, r0)
        a = el.auxiliary_field(pts, 2.0, 0.55, mh, r0)
        assert np.max(np.abs(a + np.conj(e))) > 1e-3 * np.max(np.abs(e))


def test_quasistatic_limit_s15():
    """Eq. (S15): for omega b << |gamma_h| v the field tends to that of a
    static line current, which in the normalisation of eq. (25) reads
    e_hat -> exp(i phi) (beta gamma_h / k0) (x - x0, y - y0, 0) / b^2."""
    E = 1e-4
    k0 = E / HBARC
    for mh, beta in [(1.0, 0.55), (1.45, 0.55), (2.0, 0.55)]:
        g = el.gamma_h(beta, mh)
        pts = np.array([[3.0, 1.0, 0.5], [-2.0, 4.0, -1.0]])
        e = el.incident_field(pts, E, beta, mh, (0.0, 0.0, 0.0))
        b2 = pts[:, 0] ** 2 + pts[:, 1] ** 2
        ph = np.exp(1j * k0 * pts[:, 2] / beta)
        ref_x = ph * beta * g / k0 * pts[:, 0] / b2
        ref_y = ph * beta * g / k0 * pts[:, 1] / b2
        assert np.allclose(e[:, 0], ref_x, rtol=1e-6)
        assert np.allclose(e[:, 1], ref_y, rtol=1e-6)
        assert np.all(np.abs(e[:, 2]) < 1e-3 * np.abs(e[:, 0]).max())


def test_trajectory_through_dipole_is_singular():
    with pytest.raises(ZeroDivisionError):
        el.incident_field(np.array([[1.0, 2.0, 3.0]]), 2.0, 0.55, 1.45, (1.0, 2.0, -5.0))
