"""Pins of the far-field CL oracle: a single dipole radiates (8 pi/3)|p|^2 over
the sphere (exact for a rule of degree >= 2), and for a small particle the
angular integral equals the matvec form of P_CL, whose quadratic form is
pinned in test_oracle_losses (the Green's tensor identity behind it is
independent of the far-field code)."""

import os
import sys

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(HERE))

from oracle import farfield as F  # noqa: E402
from oracle.dda import system  # noqa: E402
from oracle import cdense, losses  # noqa: E402
import workloads as W  # noqa: E402


def test_sphere_rule_weights_and_low_moments():
    d, w = F.sphere_rule(4, 8)
    assert np.sum(w) == pytest.approx(4 * np.pi, rel=1e-14)
    # integral of n n^T = (4 pi / 3) I
    M = np.einsum("q,qi,qj->ij", w, d, d)
    assert np.allclose(M, (4 * np.pi / 3) * np.eye(3), atol=1e-13)
    assert np.allclose(np.linalg.norm(d, axis=1), 1.0, atol=1e-15)


def test_single_dipole_radiates_eight_pi_thirds():
    rng = np.random.default_rng(1)
    p = rng.standard_normal((1, 3)) + 1j * rng.standard_normal((1, 3))
    c = np.array([[0.3, -0.2, 0.7]])
    d, w = F.sphere_rule(3, 5)
    A = F.amplitudes(c, p, 0.37, d)
    total = np.sum(w * F.transverse_intensity(A, d))
    assert total == pytest.approx(8 * np.pi / 3 * np.sum(np.abs(p) ** 2), rel=1e-13)


def test_transverse_part_drops_the_longitudinal_component():
    A = np.array([[1.0 + 2j, 0.0, 0.0]])
    n = np.array([[1.0, 0.0, 0.0]])
    assert F.transverse_intensity(A, n)[0] == pytest.approx(0.0, abs=1e-15)
    n = np.array([[0.0, 0.0, 1.0]])
    assert F.transverse_intensity(A, n)[0] == pytest.approx(5.0, rel=1e-15)


@pytest.mark.parametrize("m_h", [1.0, 1.45, 2.0])
def test_angular_integral_equals_matvec_form(m_h):
    """Random dipoles on a small lattice: (k^3/4pi) integral |A_perp|^2 =
    Im(p^H G_off p) + (2/3) k^3 |p|^2 to quadrature accuracy."""
    mask = W.random_mask(5, 4, 3, 0.7, seed=2)
    n = int(mask.sum())
    d = 3.0
    E, beta = 2.4, 0.55
    eps = np.full(n, -5.0 + 0.8j)
    c, alpha, k, _ = system(mask, d, eps, m_h, E)
    rng = np.random.default_rng(5)
    p = rng.standard_normal((n, 3)) + 1j * rng.standard_normal((n, 3))
    Gp = cdense.matvec(c, alpha, k, p, interaction_only=True)
    want = losses.p_cl(p, Gp, E, beta, m_h)
    dirs, w = F.sphere_rule(24, 48)
    got = np.sum(w * F.dp_domega(c, p, dirs, E, beta, m_h))
    assert got == pytest.approx(want, rel=1e-10)
