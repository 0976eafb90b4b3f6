"""Pins for the dipole interaction (eq. 5) and the dense system matrix."""

import mpmath as mp
import numpy as np
import pytest

from oracle import cdense
from oracle.interaction import dense_matrix, green_tensor, interaction_matrix


@pytest.mark.parametrize("k", [0.05, 0.02 + 0.004j, 0.3 + 0.05j])
def test_green_tensor_is_hessian_of_scalar_green_function(k):
    """G_tilde = (k^2 I + grad grad) exp(ikR)/R, i.e. 4 pi k^2 times the
    Green's tensor of eq. (5); checked with numerical derivatives."""
    mp.mp.dps = 40
    kk = mp.mpc(k)

    def phi(x, y, z):
        r = mp.sqrt(x * x + y * y + z * z)
        return mp.exp(1j * kk * r) / r

    for R in [(1.0, 0.0, 0.0), (2.0, -1.5, 0.5), (-3.0, 4.0, 12.0)]:
        G = green_tensor(np.array([R]), k)[0]
        X = tuple(mp.mpf(v) for v in R)
        for a in range(3):
            for b in range(3):
                order = [0, 0, 0]
                order[a] += 1
                order[b] += 1
                h = mp.diff(phi, X, tuple(order))
                ref = h + (kk * kk * phi(*X) if a == b else 0)
                assert abs(complex(ref) - G[a, b]) <= 1e-12 * max(abs(complex(ref)), 1e-30) + 1e-15


def test_imaginary_part_at_coincidence_eq15():
    """Eq. (15): Im G(r, r') -> k I/(6 pi) as r -> r' in a lossless host,
    i.e. Im G_tilde -> (2/3) k^3 I."""
    k = 0.07
    for R in [(0.1, 0, 0), (0.03, 0.02, -0.01)]:  # k R ~ 1e-3..1e-2
        G = green_tensor(np.array([R]), k)[0]
        assert np.allclose(np.imag(G), (2.0 / 3.0) * k ** 3 * np.eye(3), rtol=0, atol=1e-4 * k ** 3)


def test_reciprocity_matrix_symmetric():
    """Section 2.4: G(r, r') = G(r', r)^T, so the DDA matrix is complex symmetric."""
    rng = np.random.default_rng(0)
    c = rng.uniform(-5, 5, size=(30, 3))
    alpha = rng.uniform(0.1, 1, 30) + 1j * rng.uniform(0, 1, 30)
    A = dense_matrix(c, alpha, 0.03 + 0.002j)
    assert np.max(np.abs(A - A.T)) <= 1e-15 * np.max(np.abs(A))
    G = green_tensor(c[:5, None, :] - c[None, 5:10, :], 0.05)
    Gm = green_tensor(c[None, 5:10, :] - c[:5, None, :], 0.05)
    assert np.array_equal(G, Gm)  # even in R


def test_c_matvec_matches_dense_matrix():
    """The on-the-fly C product equals the explicit matrix product."""
    rng = np.random.default_rng(1)
    n = 64
    c = rng.uniform(-6, 6, size=(n, 3))
    alpha = rng.uniform(0.1, 1, n) + 1j * rng.uniform(0, 1, n)
    k = 0.04 + 0.001j
    x = rng.standard_normal((n, 3)) + 1j * rng.standard_normal((n, 3))
    A = dense_matrix(c, alpha, k)
    y = cdense.matvec(c, alpha, k, x)
    ref = (A @ x.ravel()).reshape(n, 3)
    assert np.max(np.abs(y - ref)) <= 1e-13 * np.max(np.abs(ref))
    G = interaction_matrix(c, k)
    g = cdense.matvec(c, alpha, k, x, interaction_only=True)
    ref = (G @ x.ravel()).reshape(n, 3)
    assert np.max(np.abs(g - ref)) <= 1e-13 * np.max(np.abs(ref))
