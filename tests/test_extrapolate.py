"""Richardson extrapolation (section 3.2): the oracle against what the
mathematics fixes, and the C-ABI host function against the oracle.  Host only."""

import os
import sys

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(HERE))

from oracle import extrapolate as X  # noqa: E402

LIB = os.path.join(os.path.dirname(HERE), "paper_2208_01348_amd", "libdda.so")
# the paper's series n_x = 128 ... 32 for one particle size
N_PAPER = [128, 108, 91, 76, 64, 54, 45, 38, 32]


def test_exact_quadratic_is_recovered_with_zero_interval():
    d = 150.0 / np.array(N_PAPER)
    y = 2.5 - 0.7 * d + 0.3 * d * d
    a, ci = X.richardson(d, y)
    assert a == pytest.approx(2.5, rel=1e-13)
    assert ci < 1e-12


def test_three_points_interpolate_and_give_no_interval():
    d = np.array([1.0, 0.8, 0.5])
    y = np.array([3.0, 2.0, 1.5])
    a, ci = X.richardson(d, y)
    # the quadratic through three points, evaluated at 0 by Lagrange's formula
    L0 = sum(y[i] * np.prod([(0 - d[j]) / (d[i] - d[j]) for j in range(3) if j != i])
             for i in range(3))
    assert a == pytest.approx(L0, rel=1e-12)
    assert np.isnan(ci)


def test_linear_in_the_data_and_invariant_to_the_length_unit():
    rng = np.random.default_rng(1)
    d = 100.0 / np.array(N_PAPER)
    y1, y2 = rng.standard_normal(9), rng.standard_normal(9)
    a1, _ = X.richardson(d, y1)
    a2, _ = X.richardson(d, y2)
    a12, _ = X.richardson(d, y1 + 3.0 * y2)
    assert a12 == pytest.approx(a1 + 3.0 * a2, rel=1e-10, abs=1e-12)
    a_nm, ci_nm = X.richardson(d, y1)
    a_um, ci_um = X.richardson(d * 1e-3, y1)
    assert a_um == pytest.approx(a_nm, rel=1e-9)
    assert ci_um == pytest.approx(ci_nm, rel=1e-9)


def test_weights_follow_d_cubed_errors():
    """A perturbation at the coarsest lattice moves the result far less than
    the same perturbation at the finest (weights d^-6)."""
    d = 150.0 / np.array(N_PAPER)
    base = 1.0 + 0.2 * d
    a0, _ = X.richardson(d, base)
    y = base.copy(); y[-1] += 1e-3            # coarsest
    a_coarse, _ = X.richardson(d, y)
    y = base.copy(); y[0] += 1e-3             # finest
    a_fine, _ = X.richardson(d, y)
    assert abs(a_coarse - a0) < 0.1 * abs(a_fine - a0)


def test_interval_is_twice_the_standard_error():
    """The half-width equals 2 sqrt(s^2 [(X^T W X)^-1]_00), computed here by a
    separate route (pseudo-inverse of the weighted design)."""
    rng = np.random.default_rng(2)
    d = 150.0 / np.array(N_PAPER)
    y = 1.0 + 0.1 * d + 0.05 * d * d + 1e-3 * d ** 3 * rng.standard_normal(9)
    a, ci = X.richardson(d, y)
    W = np.diag(d ** -6.0)
    Xd = np.stack([np.ones(9), d, d * d], axis=1)
    cov = np.linalg.pinv(Xd.T @ W @ Xd)
    coef = cov @ Xd.T @ W @ y
    r = y - Xd @ coef
    s2 = (r @ W @ r) / 6.0
    assert a == pytest.approx(coef[0], rel=1e-9)
    assert ci == pytest.approx(2.0 * np.sqrt(s2 * cov[0, 0]), rel=1e-7)


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        pytest.skip("libdda.so is not built")
    from paper_2208_01348_amd import _lib as L
    return L


def test_lib_matches_oracle(lib):
    rng = np.random.default_rng(3)
    for n in (3, 5, 9):
        d = 150.0 / np.array(N_PAPER[:n])
        y = 1.0 + 0.3 * d - 0.02 * d * d + 1e-3 * d ** 3 * rng.standard_normal(n)
        a_l, ci_l = lib.dda_richardson(d, y)
        a_o, ci_o = X.richardson(d, y)
        assert a_l == pytest.approx(a_o, rel=1e-10)
        if n == 3:
            assert np.isnan(ci_l) and np.isnan(ci_o)
        else:
            assert ci_l == pytest.approx(ci_o, rel=1e-8)
    with pytest.raises(lib.DDAError):
        lib.dda_richardson([1.0, 1.0, 1.0], [1.0, 2.0, 3.0])   # one size only
    with pytest.raises(lib.DDAError):
        lib.dda_richardson([1.0, 0.5], [1.0, 2.0])
