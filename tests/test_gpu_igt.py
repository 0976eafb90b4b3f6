"""GPU parity of the integrated interaction (DDA_INT_IGT: the Green's tensor
averaged over the source cell for near offsets, point values beyond) against
the oracle's dense matrix built with its own cubature (numpy Gauss-Legendre,
32 nodes per axis; the library's rule has 24): FFT matvec at 1e-12 (FP64) and 1e-5 (FP32), losses
against dense LU at 1e-9 (FP64) and 1e-5 (mixed)."""

import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

import workloads as W  # noqa: E402
from oracle.dda import solve_point, system  # noqa: E402
from oracle.interaction import dense_matrix_igt  # noqa: E402
from paper_2208_01348_amd.solver import DDASolver  # noqa: E402


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def to_dev(f, dtype=torch.complex128):
    return torch.from_numpy(np.ascontiguousarray(np.transpose(f, (0, 2, 1)))).to(dtype).cuda()


def from_dev(t):
    return np.transpose(t.to(torch.complex128).cpu().numpy(), (0, 2, 1))


LATTICES = [
    ("single_dipole", np.ones((1, 1, 1), np.uint8), 1.0),
    ("ragged_5x7x3", W.random_mask(5, 7, 3, 0.7, seed=1), 1.7),
    ("rod_24x6x6", W.capped_rod_mask(24, 6, 6, 1.0, 3.0, 24.0), 1.0),
    ("sphere_12", W.sphere_mask(12, 1.0, 6.0), 1.0),
    ("box_8x8x20", W.box_mask(8, 8, 20), 0.8),        # five-pass chain (my != mz)
    ("random_3x30x30", W.random_mask(3, 30, 30, 0.25, seed=2), 1.1),  # five-pass, y/z grid 64
]


@pytest.mark.parametrize("name,mask,d", LATTICES)
@pytest.mark.parametrize("m_h", [1.45 + 0j, 2.0 + 0.01j])
def test_igt_matvec_parity(name, mask, d, m_h):
    E = 2.4
    n = int(mask.sum())
    rng = np.random.default_rng(3)
    eps = (-7.0 + 0.8j) + 0.2 * rng.standard_normal(n)
    x = rng.standard_normal((2, n, 3)) + 1j * rng.standard_normal((2, n, 3))
    say("igt matvec", name, m_h, "n_occ", n)
    s = DDASolver(mask, d, m_h, interaction="igt")
    y = from_dev(s.matvec(E, eps, to_dev(x)))
    y32 = from_dev(s.matvec(E, eps, to_dev(x, torch.complex64), precision="mixed"))
    c, alpha, k, _ = system(mask, d, eps, m_h, E)
    A = dense_matrix_igt(c, alpha, k, d)
    for r in range(2):
        ref = (A @ x[r].reshape(-1)).reshape(n, 3)
        e64 = np.linalg.norm(y[r] - ref) / np.linalg.norm(ref)
        e32 = np.linalg.norm(y32[r] - ref) / np.linalg.norm(ref)
        say(f"  rhs {r}: fp64 {e64:.2e} fp32 {e32:.2e}")
        assert e64 <= 1e-12 and e32 <= 1e-5
    s.close()


@pytest.mark.parametrize("solver,precision,bar", [("cocg", "fp64", 1e-9), ("bicgstab", "fp64", 1e-9),
                                                  ("cocg", "mixed", 1e-5), ("qmr", "fp64", 1e-9)])
@pytest.mark.parametrize("m_h,beta", [(1.45 + 0j, 0.55), (2.0 + 0.01j, 0.7)])
def test_igt_losses_match_oracle(solver, precision, bar, m_h, beta):
    mask = W.capped_rod_mask(12, 6, 6, 2.0, 6.0, 24.0)
    d = 2.0
    n = int(mask.sum())
    energies = np.array([1.9, 2.7])
    r0 = np.array([[16.0, 1.0, 0.0]])
    eps = np.repeat(W.drude_eps(energies)[:, None], n, axis=1)
    say("igt losses", solver, precision, m_h)
    s = DDASolver(mask, d, m_h, precision=precision, solver=solver, interaction="igt",
                  tol=1e-12 if precision == "fp64" else 1e-10, maxit=20000)
    P, info = s.spectrum(energies, beta, eps, r0)
    assert all(i.status == 0 for i in info), info
    point = DDASolver(mask, d, m_h, precision="fp64", solver="cocg", tol=1e-12, maxit=20000)
    Pp, _ = point.spectrum(energies, beta, eps, r0)
    point.close()
    for i, E in enumerate(energies):
        ref = solve_point(mask, d, eps[i], m_h, beta, r0[0], float(E), interaction="igt")
        vals = [ref.p_eels, ref.p_ext, ref.p_abs, ref.p_cl]
        scale = max(abs(v) for v in vals)
        for g, v, nm in zip(P[i], vals, ["eels", "ext", "abs", "cl"]):
            err = abs(g - v) / max(abs(v), 1e-3 * scale)
            say(f"  E={E} {nm}: gpu={g:.15e} oracle={v:.15e} rel={err:.2e}")
            assert err <= bar, (nm, err)
        # the integrated interaction does change the answer
        assert abs(P[i][0] - Pp[i][0]) > 1e-4 * abs(Pp[i][0])
    s.close()
