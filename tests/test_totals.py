"""Total-loss helpers (free-space loss, P_CL^tot, Gaussian broadening): the
oracle against what the paper and the mathematics fix, and the C-ABI host
functions against the oracle.  Host only: no GPU."""

import os
import sys

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(HERE))

from oracle import totals as T  # noqa: E402
from oracle.constants import ALPHA_FS, HBAR_C_EV_NM  # noqa: E402

LIB = os.path.join(os.path.dirname(HERE), "paper_2208_01348_amd", "libdda.so")


# ---------------------------------------------------------------- oracle pins
def test_frank_tamm_matches_the_fine_structure_form():
    """Eq. (29) in SI units equals alpha_fs (1 - 1/beta_h^2)/(hbar c): the two
    share no constant (mu0, q, hbar against alpha_fs, hbar c), so a dropped
    factor 2/pi, 1/8 or a unit slip fails."""
    for beta, mh in [(0.55, 2.0), (0.7, 1.6), (0.9, 1.2), (0.548, 1.05 / 0.548)]:
        bh = beta * mh
        want = ALPHA_FS * (1.0 - 1.0 / bh ** 2) / HBAR_C_EV_NM
        got = T.free_space_loss_per_nm(beta, mh)
        assert abs(got - want) <= 2e-9 * want, (beta, mh, got, want)


def test_frank_tamm_threshold_and_absorbing_host():
    assert T.free_space_loss_per_nm(0.55, 1.45) == 0.0      # beta_h = 0.80 < 1
    assert T.free_space_loss_per_nm(0.5, 2.0) == 0.0        # beta_h = 1 exactly
    assert T.free_space_loss_per_nm(0.55, 2.0) > 0.0        # the paper's Cherenkov case
    with pytest.raises(ValueError):
        T.free_space_loss_per_nm(0.7, 2.0 + 0.01j)


def test_frank_tamm_value_for_the_cherenkov_case():
    """100 keV electron (beta = 0.548) in m_h = 2: beta_h = 1.096, so about
    alpha_fs * 0.168 / 197.3 = 6.2e-6 per eV per nm."""
    v = T.free_space_loss_per_nm(0.5482, 2.0)
    assert 6.0e-6 < v < 6.4e-6


def test_cl_total_reduces_to_cl_below_threshold():
    """P_EELS = P_ext when beta_h < 1 (section 2.5), hence P_CL^tot = P_CL."""
    assert T.cl_total(0.37, 0.37, 0.11) == 0.11
    assert T.cl_total(0.50, 0.40, 0.10) == pytest.approx(0.20)


def test_psf_of_a_delta_is_the_gaussian():
    E = np.linspace(1.0, 3.0, 401)           # dE = 5 meV
    p = np.zeros_like(E)
    p[200] = 1.0 / (E[1] - E[0])             # unit area at 2 eV
    out = T.psf_gauss(E, p, 0.15)
    sigma = 0.15 / (2.0 * np.sqrt(2.0 * np.log(2.0)))
    assert out[200] == pytest.approx(1.0 / (sigma * np.sqrt(2 * np.pi)), rel=1e-12)
    # half maximum at +-FWHM/2 (15 grid steps)
    assert out[215] / out[200] == pytest.approx(0.5, rel=1e-12)
    assert out[185] / out[200] == pytest.approx(0.5, rel=1e-12)
    assert np.sum(out) * (E[1] - E[0]) == pytest.approx(1.0, rel=1e-9)


def test_psf_keeps_a_constant_away_from_the_ends():
    E = np.linspace(0.0, 4.0, 801)
    out = T.psf_gauss(E, np.full_like(E, 2.5), 0.2)
    assert out[400] == pytest.approx(2.5, rel=1e-10)
    # at the first point half the kernel falls off the grid; the sampled half
    # keeps its centre sample in full: 1/2 + g(0) dE / 2 of the area
    dE = E[1] - E[0]
    sigma = 0.2 / (2.0 * np.sqrt(2.0 * np.log(2.0)))
    assert out[0] == pytest.approx(2.5 * (0.5 + 0.5 * dE / (sigma * np.sqrt(2 * np.pi))),
                                   rel=1e-9)


# ------------------------------------------------- C-ABI host functions = oracle
@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        pytest.skip("libdda.so is not built")
    from paper_2208_01348_amd import _lib as L
    return L


def test_lib_free_space_loss_matches_oracle(lib):
    for beta, mh in [(0.55, 2.0), (0.7, 1.6), (0.55, 1.45), (0.9, 1.2)]:
        got = lib.dda_free_space_loss(beta, complex(mh))
        want = T.free_space_loss_per_nm(beta, mh)
        # the library uses alpha_fs and hbar c, the oracle SI constants
        assert abs(got - want) <= 2e-9 * want, (beta, mh, got, want)
    with pytest.raises(lib.DDAError):
        lib.dda_free_space_loss(0.7, 2.0 + 0.01j)


def test_lib_cl_total_matches_oracle(lib):
    rng = np.random.default_rng(3)
    P = rng.standard_normal((7, 4))
    got = lib.dda_cl_total(P, 2.0)
    want = [T.cl_total(r[0], r[1], r[3]) for r in P]
    assert np.array_equal(got, np.array(want))
    with pytest.raises(lib.DDAError):
        lib.dda_cl_total(P, 2.0 + 0.01j)


def test_lib_psf_matches_oracle(lib):
    rng = np.random.default_rng(4)
    E = np.linspace(1.0, 3.0, 129)
    p = rng.random(129)
    got = lib.dda_psf_gauss(E, p, 0.15)
    want = T.psf_gauss(E, p, 0.15)
    assert np.max(np.abs(got - want)) <= 1e-13 * np.max(np.abs(want))
    with pytest.raises(lib.DDAError):
        lib.dda_psf_gauss(np.array([1.0, 1.1, 1.3]), np.ones(3), 0.1)   # not uniform
