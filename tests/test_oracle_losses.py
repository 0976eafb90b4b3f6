"""Pins for the solve and the loss/emission reductions (sections 2.4-2.7)."""

import numpy as np
import pytest

from oracle import electron as el
from oracle.dda import solve_point, system
from oracle.interaction import dense_matrix
from oracle.solve import bicgstab, lu_solve
from workloads import sphere_mask, capped_rod_mask, random_mask

HBARC = 197.3269804
ALPHA = 7.2973525693e-3


def _one_dipole():
    return np.ones((1, 1, 1), dtype=np.uint8)


@pytest.mark.parametrize("pol", ["ldr", "rr", "cm"])
def test_single_dipole_vacuum_matches_textbook_small_particle_formula(pol):
    """One dipole in vacuum: the classic small-particle loss probability
    (e.g. Garcia de Abajo, Rev. Mod. Phys. 82, 209 (2010)), per unit loss
    energy, written in its own notation:
      Gamma = 4 alpha_fs E^2 / (pi (hbar c)^3 beta^4 gamma^2)
              [K1(omega b/v gamma)^2 + K0(omega b/v gamma)^2 / gamma^2] Im(alpha)."""
    d, E, beta, b = 2.0, 3.0, 0.55, 5.0
    eps = -8.0 + 0.8j
    res = solve_point(_one_dipole(), d, [eps], 1.0, beta, (b, 0.0, 0.0), E, pol=pol)
    _, alpha, _, _ = system(_one_dipole(), d, [eps], 1.0, E, pol)
    gam = 1.0 / np.sqrt(1 - beta * beta)
    x = (E / HBARC) * b / (beta * gam)
    K0, K1 = el.besselk01(np.array([x]))
    ref = 4 * ALPHA * E ** 2 / (np.pi * HBARC ** 3 * beta ** 4 * gam ** 2) * \
        (K1[0] ** 2 + K0[0] ** 2 / gam ** 2).real * np.imag(alpha[0])
    assert res.p_eels == pytest.approx(ref, rel=1e-12)
    assert res.p_ext == pytest.approx(ref, rel=1e-12)


@pytest.mark.parametrize("m_h,beta", [(1.45, 0.55), (2.0, 0.55), (1.5 + 0.05j, 0.6),
                                      (2.0 + 0.01j, 0.7)])
def test_single_dipole_closed_form_any_host(m_h, beta):
    """One dipole, p = alpha e_hat.  From eqs. (25), (34), (37):
    P_EELS = Pi Im[alpha (K1^2 + K0^2/gamma_h^2) / (m_h^2 gamma_h^2)],
    Pi = 4 alpha_fs k0^2/(pi hbar c beta^4), K at k_t b (hand derivation; the
    (x-x0)^2 + (y-y0)^2 = b^2 collapse of the transverse part is what it tests)."""
    d, E = 1.5, 2.2
    eps = -6.0 + 0.5j
    r0 = (3.0, 4.0, -7.0)
    res = solve_point(_one_dipole(), d, [eps], m_h, beta, r0, E, pol="ldr")
    _, alpha, _, _ = system(_one_dipole(), d, [eps], m_h, E, "ldr")
    g = el.gamma_h(beta, m_h)
    kt = el.transverse_wavenumber(E, beta, m_h)
    K0, K1 = el.besselk01(np.array([kt * 5.0]))
    Pi = 4 * ALPHA * (E / HBARC) ** 2 / (np.pi * HBARC * beta ** 4)
    ref = Pi * np.imag(alpha[0] * (K1[0] ** 2 + K0[0] ** 2 / g ** 2) / (m_h * g) ** 2)
    assert res.p_eels == pytest.approx(ref, rel=1e-12)


def _small_case(m_h=1.45, beta=0.55, eps=-10.0 + 1.0j, n=6, d=2.0, E=2.5, pol="ldr"):
    mask = sphere_mask(n, d, n * d / 2)
    r0 = (n * d / 2 + 2.0, 0.3, 0.0)
    return mask, d, eps, m_h, beta, r0, E, pol


def test_energy_budget_discrete_identity():
    """Real host, beta_h < 1: P_EELS = P_ext (section 2.4) and
    P_ext = P_abs + P_CL (the budget of Fig. 1 / eq. 41 with W_0 = 0)."""
    mask, d, eps, m_h, beta, r0, E, pol = _small_case()
    r = solve_point(mask, d, [eps] * int(mask.sum()), m_h, beta, r0, E, pol=pol)
    assert r.p_eels == pytest.approx(r.p_ext, rel=1e-11)
    assert r.p_abs + r.p_cl == pytest.approx(r.p_ext, rel=1e-11)
    assert r.p_eels > 0 and r.p_cl > 0 and r.p_abs > 0


def test_lossless_particle_and_host():
    """Non-absorbing particle and host, beta_h < 1: nothing is absorbed and
    every lost quantum is emitted, P_abs = 0 and P_EELS = P_CL (section S6)."""
    mask, d, eps, m_h, beta, r0, E, pol = _small_case(eps=3.0 + 0j)
    r = solve_point(mask, d, [eps] * int(mask.sum()), m_h, beta, r0, E, pol=pol)
    assert abs(r.p_abs) <= 1e-10 * r.p_cl
    assert r.p_eels == pytest.approx(r.p_cl, rel=1e-10)


def test_cherenkov_eels_differs_from_extinction():
    """beta_h > 1: W_enh != W_ext (section 2.4, Fig. 8), so P_EELS != P_ext,
    while P_CL stays positive (section 2.6)."""
    mask, d, eps, m_h, beta, r0, E, pol = _small_case(m_h=2.0, beta=0.7, d=5.0, E=3.0)
    r = solve_point(mask, d, [eps] * int(mask.sum()), m_h, beta, r0, E, pol=pol)
    assert abs(r.p_eels - r.p_ext) > 1e-3 * abs(r.p_ext)
    assert r.p_cl > 0
    # the discrete budget still closes for the extinction form
    assert r.p_abs + r.p_cl == pytest.approx(r.p_ext, rel=1e-10)


def test_scale_invariance_host_to_vacuum_eq45():
    """Eq. (45): host m_h at hbar omega equals vacuum with v -> m_h v,
    m_p -> m_p/m_h and hbar omega -> m_h hbar omega, same geometry."""
    mask, d, eps, m_h, beta, r0, E, pol = _small_case()
    n = int(mask.sum())
    host = solve_point(mask, d, [eps] * n, m_h, beta, r0, E, pol=pol)
    vac = solve_point(mask, d, [eps / m_h ** 2] * n, 1.0, beta * m_h, r0, E * m_h, pol=pol)
    for f in ["p_eels", "p_ext", "p_abs", "p_cl"]:
        assert getattr(vac, f) == pytest.approx(getattr(host, f), rel=1e-11)


def test_scale_invariance_geometric_eq46():
    """Eq. (46): keep omega, scale v -> m_h v, m_p -> m_p/m_h and every length
    by m_h; the vacuum probabilities are m_h times the host ones."""
    mask, d, eps, m_h, beta, r0, E, pol = _small_case()
    n = int(mask.sum())
    host = solve_point(mask, d, [eps] * n, m_h, beta, r0, E, pol=pol)
    vac = solve_point(mask, d * m_h, [eps / m_h ** 2] * n, 1.0, beta * m_h,
                      tuple(m_h * v for v in r0), E, pol=pol)
    assert vac.p_eels == pytest.approx(m_h * host.p_eels, rel=1e-11)
    assert vac.p_cl == pytest.approx(m_h * host.p_cl, rel=1e-11)


@pytest.mark.parametrize("xi,eta,m_h,beta", [(2.0, 1.0, 1.45, 0.55), (0.5, 1.25, 2.0, 0.6),
                                             (1.5, 1.1, 1.8 + 0.05j, 0.7)])
def test_general_scale_invariance_eq43_44(xi, eta, m_h, beta):
    """Eqs. (43)-(44): m_h -> m_h/eta, m_p -> m_p/eta, v -> eta v, lengths
    -> lengths/xi, omega -> xi eta omega give P -> P/xi; the Cherenkov and
    absorbing cases included (only P_EELS and P_ext are defined there)."""
    mask, d, eps, _, _, r0, E, pol = _small_case(m_h=m_h, beta=beta, d=3.0)
    n = int(mask.sum())
    a = solve_point(mask, d, [eps] * n, m_h, beta, r0, E, pol=pol)
    b = solve_point(mask, d / xi, [eps / eta ** 2] * n, m_h / eta, beta * eta,
                    tuple(v / xi for v in r0), E * xi * eta, pol=pol)
    assert b.p_eels == pytest.approx(a.p_eels / xi, rel=1e-10)
    assert b.p_ext == pytest.approx(a.p_ext / xi, rel=1e-10)


def test_z0_shift_changes_nothing():
    """Section S5: moving the beam centre along the trajectory only changes a
    constant phase of the fields; every probability is unchanged."""
    mask, d, eps, m_h, beta, r0, E, pol = _small_case(m_h=2.0 + 0.01j, beta=0.7)
    n = int(mask.sum())
    a = solve_point(mask, d, [eps] * n, m_h, beta, r0, E, pol=pol)
    b = solve_point(mask, d, [eps] * n, m_h, beta, (r0[0], r0[1], r0[2] + 37.3), E, pol=pol)
    for f in ["p_eels", "p_ext", "p_abs", "p_cl"]:
        assert getattr(b, f) == pytest.approx(getattr(a, f), rel=1e-11)


def test_bicgstab_matches_lu():
    mask = capped_rod_mask(12, 4, 4, 1.0, radius=2.0, length=12.0)
    d, E, m_h, beta = 1.0, 2.0, 1.45, 0.55
    n = int(mask.sum())
    centres, alpha, k, _ = system(mask, d, [-6.0 + 0.6j] * n, m_h, E)
    e = el.incident_field(centres, E, beta, m_h, (8.0, 0.0, 0.0))
    p_lu = lu_solve(centres, alpha, k, e)
    p_it, it, res = bicgstab(centres, alpha, k, e, tol=1e-13)
    assert res <= 1e-13
    assert np.max(np.abs(p_it - p_lu)) <= 1e-10 * np.max(np.abs(p_lu))


def test_reciprocity_of_solutions():
    """A = A^T implies e1 . A^-1 e2 = e2 . A^-1 e1 (bilinear)."""
    mask = random_mask(5, 4, 3, 0.7, seed=11)
    centres, alpha, k, _ = system(mask, 1.7, [2.0 + 0.3j] * int(mask.sum()), 1.3 + 0.02j, 2.7)
    rng = np.random.default_rng(4)
    e1 = rng.standard_normal((len(alpha), 3)) + 1j * rng.standard_normal((len(alpha), 3))
    e2 = rng.standard_normal((len(alpha), 3)) + 1j * rng.standard_normal((len(alpha), 3))
    A = dense_matrix(centres, alpha, k)
    x1 = np.linalg.solve(A, e1.ravel())
    x2 = np.linalg.solve(A, e2.ravel())
    assert np.sum(e2.ravel() * x1) == pytest.approx(np.sum(e1.ravel() * x2), rel=1e-12)


# ---------------------------------------------------------------- P_abs ----
# P_abs is one formula for every host (eq. 18 with the cell relation of
# eq. 7, plus the polarizability's corrections).  These pins fix it from
# outside the formula: continuity across the real axis of m_h, the
# coincidences with eq. (18) written out from the cell field, and the
# closed-form budget defect in an absorbing host.

def _lu_point(pol, m_h, eps=-10.0 + 1.0j, beta=0.55, E=2.5, n=6, d=2.0):
    mask = sphere_mask(n, d, n * d / 2)
    r0 = (n * d / 2 + 2.0, 0.3, 0.0)
    nn = int(mask.sum())
    return solve_point(mask, d, [eps] * nn, m_h, beta, r0, E, pol=pol, method="lu"), mask, d


@pytest.mark.parametrize("pol", ["ldr", "cm", "rr"])
def test_p_abs_and_p_cl_continuous_across_the_real_axis(pol):
    """Im m_h -> 0+ changes every probability by O(Im m_h): the absorbing-host
    branch of P_abs and of the nominal P_CL joins the real-host one (the
    earlier split jumped by 6e-4 relative with LDR)."""
    a, _, _ = _lu_point(pol, 1.45)
    b, _, _ = _lu_point(pol, 1.45 + 1e-10j)
    for f in ["p_eels", "p_ext", "p_abs", "p_cl"]:
        assert getattr(b, f) == pytest.approx(getattr(a, f), rel=1e-8), f
    # and the discrete budget holds in that limit
    assert b.p_abs + b.p_cl == pytest.approx(b.p_ext, rel=1e-8)


def _eq18_cell_form(res, mask, d, eps, m_h, beta, E):
    """Eq. (18) written out: W_abs ~ sum over cells of Im(eps_p) |E_i|^2 d^3 with
    E_i from P = (eps_p - eps_h) E (eq. 7), in the units of P_* (1/eV)."""
    mh = complex(m_h)
    m2 = eps / mh ** 2
    p = res.p_hat
    E_cell = 4.0 * np.pi * p / ((m2 - 1.0) * d ** 3)           # field per cell
    s = np.sum(np.imag(eps) * np.sum(np.abs(E_cell) ** 2, axis=1)) * d ** 3 / (4.0 * np.pi)
    g = el.gamma_h(beta, m_h)
    Pi = 4 * ALPHA * (E / HBARC) ** 2 / (np.pi * HBARC * beta ** 4)
    return Pi * s / (abs(mh) ** 4 * abs(g) ** 2)


def test_p_abs_rr_real_host_is_eq18():
    """With the radiative-reaction polarizability in a real host the dipole's
    work less its radiation is exactly the cell form of eq. (18)."""
    eps, m_h, beta, E = -10.0 + 1.0j, 1.45, 0.55, 2.5
    res, mask, d = _lu_point("rr", m_h, eps=eps, beta=beta, E=E)
    ref = _eq18_cell_form(res, mask, d, eps, m_h, beta, E)
    assert res.p_abs == pytest.approx(ref, rel=1e-11)


@pytest.mark.parametrize("m_h", [1.45, 2.0 + 0.01j, 1.3 + 0.2j])
def test_p_abs_cm_is_eq18_less_self_radiation(m_h):
    """Clausius-Mossotti has no radiative correction: P_abs is eq. (18)'s cell
    form less the nominal self-radiated power (2/3) Re(k)^3 ||p||^2 weighted
    by Re(m_h^2), on real and absorbing hosts."""
    eps, beta, E = -10.0 + 1.0j, 0.55, 2.5
    res, mask, d = _lu_point("cm", m_h, eps=eps, beta=beta, E=E)
    ref = _eq18_cell_form(res, mask, d, eps, m_h, beta, E)
    mh = complex(m_h)
    kr = (mh * E / HBARC).real
    g = el.gamma_h(beta, m_h)
    Pi = 4 * ALPHA * (E / HBARC) ** 2 / (np.pi * HBARC * beta ** 4)
    rad = Pi * (mh * mh).real / (abs(mh) ** 4 * abs(g) ** 2) * (2.0 / 3.0) * kr ** 3 * \
        np.sum(np.abs(res.p_hat) ** 2)
    assert res.p_abs == pytest.approx(ref - rad, rel=1e-11)


@pytest.mark.parametrize("m_h", [1.45, 2.0 + 0.01j])
def test_p_abs_ldr_tends_to_eq18_as_d_shrinks(m_h):
    """The LDR corrections to the weight are O((kd)^2): halving d at fixed k
    divides their share of the eq. (18) weight by about four."""
    from oracle.losses import absorption_weight
    from oracle.polarizability import alpha_ldr
    eps, E = np.array([-10.0 + 1.0j, 3.0 + 0.5j]), 2.5
    mh = complex(m_h)
    m2 = eps / mh ** 2
    k = mh * E / HBARC
    shares = []
    for d in [2.0, 1.0, 0.5, 0.25]:
        w = absorption_weight(alpha_ldr(m2, d, k), m2, d, E, m_h)
        w18 = 4.0 * np.pi * np.imag(mh * mh * m2) / (np.abs(m2 - 1.0) ** 2 * d ** 3)
        shares.append(np.abs(w / w18 - 1.0))
    for a, b in zip(shares, shares[1:]):
        assert np.all(b < a / 3.5) and np.all(b > a / 4.5)


@pytest.mark.parametrize("pol,m_h", [("ldr", 2.0 + 0.01j), ("cm", 1.3 + 0.2j), ("rr", 1.5 + 0.05j)])
def test_absorbing_host_budget_defect_closed_form(pol, m_h):
    """In an absorbing host P_ext - P_abs - P_CL is not zero; from A p = e it
    equals Pi Im(m_h^2)/(|m_h|^4 |gamma_h|^2) [(4 pi/d^3) sum_i (1/3 -
    1/|m_i^2-1|^2) |p_i|^2 - Re(p^H G_off p)], with G_off from the explicit
    interaction matrix here."""
    from oracle.interaction import interaction_matrix
    eps, beta, E = -10.0 + 1.0j, 0.6, 2.5
    res, mask, d = _lu_point(pol, m_h, eps=eps, beta=beta, E=E)
    mh = complex(m_h)
    centres, _, k, m2 = system(mask, d, [eps] * int(mask.sum()), m_h, E, pol)
    G = interaction_matrix(centres, k)
    p = res.p_hat.ravel()
    X = np.vdot(p, G @ p)
    p2 = np.sum(np.abs(res.p_hat) ** 2, axis=1)
    g = el.gamma_h(beta, m_h)
    Pi = 4 * ALPHA * (E / HBARC) ** 2 / (np.pi * HBARC * beta ** 4)
    defect = Pi * (mh * mh).imag / (abs(mh) ** 4 * abs(g) ** 2) * (
        4.0 * np.pi / d ** 3 * np.sum((1.0 / 3.0 - 1.0 / np.abs(m2 - 1.0) ** 2) * p2) - X.real)
    assert res.p_ext - res.p_abs - res.p_cl == pytest.approx(defect, rel=1e-9, abs=1e-12 * abs(res.p_ext))
    assert abs(defect) > 1e-6 * abs(res.p_ext)  # the case does test something


def test_dense_rows_equal_rows_of_the_full_product():
    """oracle_dense_matvec_rows (the reference of the sampled full-size GPU
    checks) returns exactly the chosen rows of the full C product, for both
    modes and an absorbing host."""
    from oracle import cdense
    rng = np.random.default_rng(7)
    for n, k in [(50, 0.05), (173, 0.04 + 0.003j)]:
        c = rng.uniform(-6, 6, size=(n, 3))
        alpha = rng.uniform(0.1, 1, n) + 1j * rng.uniform(0, 1, n)
        x = rng.standard_normal((n, 3)) + 1j * rng.standard_normal((n, 3))
        rows = np.sort(rng.choice(n, size=min(n, 37), replace=False))
        rows = np.concatenate([rows, [0, n - 1]])
        for io in (False, True):
            full = cdense.matvec(c, alpha, k, x, interaction_only=io)
            part = cdense.matvec_rows(c, alpha, k, x, rows, interaction_only=io)
            assert np.array_equal(part, full[rows])


# ------------------------------------------------------------------ QMR ----
@pytest.mark.parametrize("m_h", [1.45, 2.0 + 0.01j])
def test_qmr_cs_matches_lu(m_h):
    """QMR for the complex-symmetric DDA system (section S5) reaches the dense
    LU solution."""
    from oracle.solve import qmr_cs
    mask = capped_rod_mask(12, 4, 4, 1.0, radius=2.0, length=12.0)
    d, E, beta = 1.0, 2.0, 0.6
    n = int(mask.sum())
    centres, alpha, k, _ = system(mask, d, [-6.0 + 0.6j] * n, m_h, E)
    e = el.incident_field(centres, E, beta, m_h, (8.0, 0.0, 0.0))
    p_lu = lu_solve(centres, alpha, k, e)
    p_q, it, res = qmr_cs(centres, alpha, k, e, tol=1e-13)
    assert res <= 1e-13 and it > 10
    assert np.max(np.abs(p_q - p_lu)) <= 1e-10 * np.max(np.abs(p_lu))


def test_qmr_cs_is_minres_for_a_real_symmetric_matrix():
    """For a real symmetric matrix the bilinear form is the inner product, the
    Lanczos vectors are orthonormal and the quasi-minimal residual is the
    minimal one: QMR-CS's iterates are MINRES's (scipy, Paige-Saunders),
    iteration by iteration; an indefinite matrix makes it non-trivial."""
    from scipy.sparse.linalg import minres
    from oracle.solve import qmr_cs
    rng = np.random.default_rng(3)
    n = 40
    Q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    lam = np.concatenate([rng.uniform(1.0, 5.0, 30), rng.uniform(-3.0, -0.5, 10)])
    A = (Q * lam) @ Q.T
    A = 0.5 * (A + A.T)
    b = rng.standard_normal(n)
    ours = {}

    def cb(it, x, tau):
        ours[it] = np.real(x).copy()

    qmr_cs(None, None, None, b.astype(np.complex128), tol=1e-300, maxit=25,
           matvec=lambda v: A @ v, callback=cb)
    theirs = []
    minres(A, b, rtol=1e-300, maxiter=25, callback=lambda xk: theirs.append(xk.copy()))
    for i in range(1, 21):
        assert np.linalg.norm(ours[i] - theirs[i - 1]) <= 1e-9 * np.linalg.norm(theirs[i - 1]), i


def test_qmr_cs_quasi_residual_bounds_the_residual_and_decreases():
    """|tau| never increases within a cycle, and with unit-norm Lanczos
    vectors the true residual never exceeds sqrt(n + 1) |tau_{n+1}| (up to
    the rounding floor of the residual, ~1e-15 ||b||, below which the
    recursion's quasi-residual keeps falling while the true one cannot)."""
    from oracle.interaction import dense_matrix
    from oracle.solve import qmr_cs
    mask = random_mask(5, 4, 3, 0.7, seed=11)
    centres, alpha, k, _ = system(mask, 1.7, [2.0 + 0.3j] * int(mask.sum()), 1.3 + 0.02j, 2.7)
    A = dense_matrix(centres, alpha, k)
    rng = np.random.default_rng(5)
    b = rng.standard_normal((len(alpha), 3)) + 1j * rng.standard_normal((len(alpha), 3))
    taus, ok = [], []

    def cb(it, x, tau):
        r = np.linalg.norm(b.ravel() - A @ x.ravel())
        ok.append(r <= np.sqrt(it + 1) * abs(tau) * (1 + 1e-9) + 1e-13 * np.linalg.norm(b))
        taus.append(abs(tau))

    qmr_cs(centres, alpha, k, b, tol=1e-300, maxit=40, callback=cb)
    assert all(ok)
    assert all(t1 <= t0 * (1 + 1e-12) for t0, t1 in zip(taus, taus[1:]))


def test_igt_interaction_keeps_the_budget_and_changes_the_result():
    """With the cell-averaged near interaction the matrix is still complex
    symmetric, so the discrete budget P_ext = P_abs + P_CL (real host) still
    holds; the near-field change moves the result by far more than rounding."""
    mask, d, eps, m_h, beta, r0, E, pol = _small_case()
    n = int(mask.sum())
    a = solve_point(mask, d, [eps] * n, m_h, beta, r0, E, pol=pol, interaction="igt")
    b = solve_point(mask, d, [eps] * n, m_h, beta, r0, E, pol=pol, method="lu")
    assert a.p_eels == pytest.approx(a.p_ext, rel=1e-11)
    assert a.p_abs + a.p_cl == pytest.approx(a.p_ext, rel=1e-11)
    assert abs(a.p_eels - b.p_eels) > 1e-3 * abs(b.p_eels)
