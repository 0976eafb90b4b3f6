"""GPU parity of CL resolved over directions (dda_cl_directions, FP64 matrix
cores) against the FP64 oracle (oracle/farfield.py), and its angular integral
against P_CL of dda_eels_cl for a converged solution."""

import os
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

import workloads as W  # noqa: E402
from oracle import farfield as F  # noqa: E402
from oracle.lattice import dipole_centres  # noqa: E402
from paper_2208_01348_amd import _lib as L  # noqa: E402
from paper_2208_01348_amd.solver import DDASolver  # noqa: E402


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def to_dev(f: np.ndarray) -> torch.Tensor:
    """[nrhs][n][3] (oracle layout) -> device [nrhs][3][n] complex128."""
    a = np.ascontiguousarray(np.transpose(np.asarray(f), (0, 2, 1)))
    return torch.from_numpy(a).to(torch.complex128).cuda()


@pytest.mark.parametrize("n_traj,rule", [(1, (6, 10)), (3, (12, 25)), (30, (5, 7))])
def test_directions_match_oracle(n_traj, rule):
    """Random dipole moments, several energies and trajectories: 3 n_traj
    columns of 3, 9 and 90 (one, one and two column tiles of 64), and 60, 300
    and 35 directions (ragged tiles of 16)."""
    mask = W.random_mask(9, 6, 5, 0.6, seed=7)
    d, m_h, beta = 2.0, 1.45, 0.55
    n = int(mask.sum())
    energies = np.array([1.7, 2.9])
    rng = np.random.default_rng(n_traj)
    nrhs = energies.size * n_traj
    p = rng.standard_normal((nrhs, n, 3)) + 1j * rng.standard_normal((nrhs, n, 3))
    dirs, w = F.sphere_rule(*rule)
    say("far field", n_traj, dirs.shape[0], "n_occ", n)
    s = DDASolver(mask, d, m_h)
    dp, pcl = s.cl_directions(energies, beta, n_traj, to_dev(p), dirs, w)
    c = dipole_centres(mask, d)
    worst = 0.0
    for r in range(nrhs):
        E = energies[r // n_traj]
        ref = F.dp_domega(c, p[r], dirs, E, beta, m_h)
        err = np.max(np.abs(dp[r] - ref)) / np.max(np.abs(ref))
        worst = max(worst, err)
        assert abs(pcl[r] - np.sum(w * ref)) <= 1e-12 * abs(np.sum(w * ref))
    say("  worst relative error per direction", worst)
    assert worst <= 1e-12
    s.close()


@pytest.mark.parametrize("m_h,beta", [(1.0, 0.55), (1.45, 0.55), (2.0, 0.70)])
def test_angular_integral_equals_p_cl(m_h, beta):
    """For a converged FP64 solution the integral over the sphere equals P_CL
    of dda_eels_cl (the quadratic form of Im G), Cherenkov host included."""
    mask = W.capped_rod_mask(12, 6, 6, 2.0, 6.0, 24.0)
    n = int(mask.sum())
    energies = np.array([1.8, 2.6])
    eps = np.repeat(W.drude_eps(energies)[:, None], n, axis=1)
    r0 = np.array([[16.0, 1.0, 0.0], [0.0, 7.0, 3.0]])
    s = DDASolver(mask, 2.0, m_h, tol=1e-12, maxit=20000, solver="cocg")
    e = s.einc(energies, beta, r0)
    p, info, st = s.solve(energies, eps, e, r0.shape[0])
    assert st == L.DDA_OK
    P = s.losses(energies, beta, eps, r0, e, p)
    dirs, w = F.sphere_rule(24, 48)
    _, pcl = s.cl_directions(energies, beta, r0.shape[0], p, dirs, w, want_dp=False)
    for i in range(P.shape[0]):
        say(f"  rhs {i}: P_CL {P[i][3]:.15e} far field {pcl[i]:.15e}")
        assert abs(pcl[i] - P[i][3]) <= 1e-9 * abs(P[i][3])
    s.close()


def test_full_size_sampled_directions():
    """Nanorod lattice (39,464 dipoles), a handful of directions per energy."""
    w = W.c2_nanorod_spectrum()
    n = int(w.mask.sum())
    energies = np.array([w.energies[10], w.energies[90]])
    rng = np.random.default_rng(9)
    p = rng.standard_normal((2, n, 3)) + 1j * rng.standard_normal((2, n, 3))
    dirs, _ = F.sphere_rule(3, 6)
    s = DDASolver(w.mask, w.d, w.m_h)
    dp, _ = s.cl_directions(energies, w.beta, 1, to_dev(p), dirs)
    c = dipole_centres(w.mask, w.d)
    for r in range(2):
        ref = F.dp_domega(c, p[r], dirs, energies[r], w.beta, w.m_h)
        err = np.max(np.abs(dp[r] - ref)) / np.max(np.abs(ref))
        say(f"  energy {energies[r]:.3f}: max relative error {err:.2e}")
        assert err <= 1e-11
    s.close()


def test_rejections():
    mask = W.random_mask(4, 4, 4, 0.6, seed=1)
    n = int(mask.sum())
    p = torch.zeros((1, 3, n), dtype=torch.complex128, device="cuda")
    s = DDASolver(mask, 1.0, 2.0 + 0.01j)
    with pytest.raises(L.DDAError):
        s.cl_directions([2.0], 0.7, 1, p, np.array([[0.0, 0.0, 1.0]]))
    s.close()
    s = DDASolver(mask, 1.0, 1.45)
    with pytest.raises(L.DDAError):
        s.cl_directions([2.0], 0.55, 1, p, np.array([[0.0, 0.0, 2.0]]))
    s.close()
