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


# ------------------------------------------- integrated interaction (igt) ----
from oracle.interaction import integrated_green_tensor, near_offsets  # noqa: E402


def _static_cube_integral_by_faces(R, d, n=40):
    """Divergence theorem for the static tensor grad grad (1/r): the volume
    integral over the cube equals the sum over its faces of grad_j(1/r) n_i,
    with grad(1/r) = -r/|r|^3; here by 2D Gauss-Legendre on each face (a
    route independent of the volume rule)."""
    u, w = np.polynomial.legendre.leggauss(n)
    s = 0.5 * d * u
    A, B = np.meshgrid(s, s, indexing="ij")
    W = np.outer(w, w) * (0.5 * d) ** 2
    out = np.zeros((3, 3))
    for ax in range(3):
        for sign in (-1.0, 1.0):
            P = np.zeros(A.shape + (3,))
            o = [i for i in range(3) if i != ax]
            P[..., ax] = sign * 0.5 * d
            P[..., o[0]] = A
            P[..., o[1]] = B
            r = np.asarray(R)[None, None, :] + P
            rn = np.linalg.norm(r, axis=-1)
            g = -r / rn[..., None] ** 3          # grad(1/r) at the face points
            for j in range(3):
                out[ax, j] += sign * np.sum(W * g[..., j])
    return out / d ** 3


@pytest.mark.parametrize("o", [(1, 0, 0), (1, 1, 0), (1, 1, 1), (2, 1, 0), (0, 0, 3)])
def test_igt_static_limit_equals_face_integrals(o):
    """k -> 0: G_tilde -> grad grad (1/R); its cube average equals the face
    integrals of the divergence theorem, to the precision of the rules."""
    d = 1.3
    R = d * np.array(o, dtype=float)
    vol = integrated_green_tensor(R, 1e-7, d).real
    faces = _static_cube_integral_by_faces(R, d)
    assert np.max(np.abs(vol - faces)) <= 1e-11 * np.max(np.abs(faces))
    # the static tensor is traceless (1/r is harmonic away from the origin)
    assert abs(np.trace(vol)) <= 1e-12 * np.max(np.abs(vol))


@pytest.mark.parametrize("k", [0.05, 0.02 + 0.002j])
def test_igt_far_offsets_follow_the_second_order_cube_average(k):
    """For a smooth integrand the cube average is f(R) + (d^2/24) lap f(R) +
    O(d^4); lap G_tilde = -k^2 G_tilde away from the origin, so the average is
    G_tilde (1 - (kd)^2/24) up to a fourth-order remainder, which for small kd
    shrinks as (d/R)^4 (and the near rule must resolve it: n = 24 vs 32
    agree)."""
    d = 1.0
    errs = []
    for r in (6.0, 12.0):
        R = np.array([r, 0.4 * r, -0.3 * r])
        avg = integrated_green_tensor(R, k, d)
        pt = green_tensor(R[None, :], k)[0] * (1.0 - (k * d) ** 2 / 24.0)
        errs.append(np.max(np.abs(avg - pt)) / np.max(np.abs(pt)))
    assert errs[1] < errs[0] / 10.0  # ~ (d/R)^4: 16x for R doubled
    assert errs[0] < 1e-3
    R = np.array([1.0, 1.0, 0.0]) * d
    a24 = integrated_green_tensor(R, k, d, n=24)
    a32 = integrated_green_tensor(R, k, d, n=32)
    assert np.max(np.abs(a24 - a32)) <= 1e-13 * np.max(np.abs(a32))


def test_igt_trace_is_the_scalar_average():
    """tr G_tilde = (3k^2 + lap) e^{ikr}/r = 2k^2 e^{ikr}/r away from the
    origin, so the trace of the cell average is 2k^2 times the cell average of
    the scalar Green's function."""
    k, d = 0.4 + 0.03j, 1.0
    R = np.array([1.0, 0.0, 1.0])
    u, w = np.polynomial.legendre.leggauss(24)
    s = 0.5 * d * u
    S = np.stack(np.meshgrid(s, s, s, indexing="ij"), axis=-1).reshape(-1, 3)
    W = (np.einsum("i,j,k->ijk", w, w, w) / 8.0).reshape(-1)
    rr = np.linalg.norm(R[None, :] + S, axis=-1)
    scal = np.sum(W * np.exp(1j * k * rr) / rr)
    assert np.trace(integrated_green_tensor(R, k, d)) == pytest.approx(2 * k * k * scal, rel=1e-12)


def test_igt_symmetry_and_offsets():
    """The cell average is symmetric and even in R (reciprocity survives), and
    the near offsets are the 122 lattice vectors within 3 cells."""
    k, d = 0.2 + 0.01j, 0.9
    for o in [(1, 2, 0), (2, -1, 2)]:
        R = d * np.array(o, float)
        a = integrated_green_tensor(R, k, d)
        b = integrated_green_tensor(-R, k, d)
        assert np.max(np.abs(a - a.T)) <= 1e-15 * np.max(np.abs(a))
        assert np.max(np.abs(a - b)) <= 1e-13 * np.max(np.abs(a))
    offs = near_offsets()
    assert len(offs) == 122 and (0, 0, 0) not in offs
