"""GPU parity: the HIP path (through the C ABI) against the FP64 CPU oracle.

Tolerances: FP64 path 1e-9 relative on loss probabilities (the stated bar),
kernels tighter (their arithmetic is FP64 throughout: the electron field and
the FFT matvec agree with the oracle to ~1e-13); mixed precision 1e-5.
"""

import json
import os
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

import workloads as W  # noqa: E402
from oracle import cdense  # noqa: E402
from oracle import electron as el  # noqa: E402
from oracle.dda import solve_point, system  # noqa: E402
from oracle.lattice import dipole_centres  # noqa: E402
from paper_2208_01348_amd import _lib as L  # noqa: E402
from paper_2208_01348_amd.solver import DDASolver  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def to_dev(f: np.ndarray, dtype=torch.complex128) -> torch.Tensor:
    """[nrhs][n][3] (oracle layout) -> device [nrhs][3][n]."""
    a = np.ascontiguousarray(np.transpose(np.asarray(f), (0, 2, 1)))
    return torch.from_numpy(a).to(dtype).cuda()


def from_dev(t: torch.Tensor) -> np.ndarray:
    """device [nrhs][3][n] -> [nrhs][n][3] complex128."""
    return np.transpose(t.to(torch.complex128).cpu().numpy(), (0, 2, 1))


def rel(a, b):
    return float(np.linalg.norm(np.ravel(a - b)) / max(np.linalg.norm(np.ravel(b)), 1e-300))


# ------------------------------------------------------------------ Bessel
def test_device_besselk01_against_mpmath():
    import mpmath as mp
    mp.mp.dps = 30
    zs = []
    for r in np.geomspace(1e-4, 60.0, 41):
        for th in np.linspace(-np.pi / 2, 0.0, 11):
            zs.append(r * np.exp(1j * th))
    zs = np.array(zs)
    say("besselk01 on", zs.size, "points")
    K0, K1 = L.dda_debug_besselk01(zs)
    worst = 0.0
    for z, a0, a1 in zip(zs, K0, K1):
        r0 = complex(mp.besselk(0, z))
        r1 = complex(mp.besselk(1, z))
        worst = max(worst, abs(a0 - r0) / abs(r0), abs(a1 - r1) / abs(r1))
    say("worst relative error", worst)
    assert worst <= 5e-15


# ------------------------------------------------------------ electron field
FIELD_CASES = [
    ("vacuum", 1.0 + 0j, 0.55),
    ("glass", 1.45 + 0j, 0.55),
    ("cherenkov", 2.0 + 0j, 0.55),
    ("absorbing_cherenkov", 2.0 + 0.01j, 0.70),
    ("lossy", 1.5 + 0.3j, 0.6),
]


@pytest.mark.parametrize("name,m_h,beta", FIELD_CASES)
def test_einc_parity(name, m_h, beta):
    mask = W.random_mask(11, 9, 7, 0.6, seed=5)
    d = 2.5
    energies = np.array([1.0, 2.2, 3.9])
    # the 11 x 9 lattice has a dipole column at (0, 0): keep trajectories off it
    r0 = np.array([[16.0, 1.25, -3.0], [0.3, -0.2, 0.0], [-20.0, 14.0, 50.0]])
    say("einc", name)
    s = DDASolver(mask, d, m_h)
    e = s.einc(energies, beta, r0)
    torch.cuda.synchronize()
    got = from_dev(e)
    c = dipole_centres(mask, d)
    k = 0
    for E in energies:
        for t in range(r0.shape[0]):
            ref = el.incident_field(c, E, beta, m_h, r0[t])
            err = np.max(np.abs(got[k] - ref)) / np.max(np.abs(ref))
            assert err <= 1e-13, (name, E, t, err)
            k += 1
    s.close()


# ------------------------------------------------------------------ matvec
MATVEC_LATTICES = [
    ("single_dipole", np.ones((1, 1, 1), np.uint8), 1.0),
    ("ragged_5x7x3", W.random_mask(5, 7, 3, 0.7, seed=1), 1.7),
    ("box_12x6x24", W.box_mask(12, 6, 24), 1.0),
    ("rod_24x6x6", W.capped_rod_mask(24, 6, 6, 1.0, 3.0, 24.0), 1.0),
    ("sphere_16", W.sphere_mask(16, 1.0, 8.0), 1.0),
    ("random_9x4x13", W.random_mask(9, 4, 13, 0.5, seed=3), 2.0),
    # five-pass chain (y grid 16, z grid 24) with an x grid of 32: the z-conv
    # blocks take their XCD-grouped order, with whole runs and a ragged tail
    ("random_16x8x12", W.random_mask(16, 8, 12, 0.7, seed=5), 1.1),
    # y, z grids of 48: both precisions take the three-pass (yz plane in LDS)
    # chain
    ("random_5x17x17", W.random_mask(5, 17, 17, 0.6, seed=9), 1.3),
    ("sphere_32", W.sphere_mask(32, 1.0, 16.0), 1.0),
    # the x kernels split a plane's rows into uneven groups: 19 rows over two
    # blocks in FP64 (x grid 128), 25 rows over two in FP32 (x grid 192)
    ("random_64x19x19", W.random_mask(64, 19, 19, 0.25, seed=4), 1.0),
    ("random_96x25x25", W.random_mask(96, 25, 25, 0.08, seed=6), 1.0),
    # y, z grids of 16 and 24: the register yz kernel at its smallest lengths
    # (at 24 its blocks have threads beyond the (component, ky) quads, which
    # take part in the D loads and product only)
    ("random_6x8x7", W.random_mask(6, 8, 7, 0.6, seed=12), 1.2),
    ("random_10x11x9", W.random_mask(10, 11, 9, 0.6, seed=13), 0.9),
]


@pytest.mark.parametrize("name,mask,d", MATVEC_LATTICES)
@pytest.mark.parametrize("m_h", [1.45 + 0j, 2.0 + 0.01j])
def test_matvec_fp64_parity(name, mask, d, m_h):
    E = 2.7
    n = int(mask.sum())
    rng = np.random.default_rng(7)
    eps = (-8.0 + 0.9j) + 0.3 * rng.standard_normal(n)  # varies per dipole
    x = rng.standard_normal((3, n, 3)) + 1j * rng.standard_normal((3, n, 3))
    say("matvec fp64", name, m_h, "n_occ", n)
    s = DDASolver(mask, d, m_h)
    xd = to_dev(x)
    y = from_dev(s.matvec(E, eps, xd))
    yi = from_dev(s.matvec(E, None, xd, interaction_only=True))
    c, alpha, k, _ = system(mask, d, eps, m_h, E)
    for r in range(3):
        ref = cdense.matvec(c, alpha, k, x[r])
        assert rel(y[r], ref) <= 1e-12, (name, r, rel(y[r], ref))
        refi = cdense.matvec(c, alpha, k, x[r], interaction_only=True)
        if n > 1:
            assert rel(yi[r], refi) <= 1e-12
    s.close()


@pytest.mark.parametrize("name,mask,d", MATVEC_LATTICES[1:])
def test_matvec_fp32_parity(name, mask, d):
    E, m_h = 2.2, 1.45 + 0j
    n = int(mask.sum())
    rng = np.random.default_rng(8)
    eps = np.full(n, -6.0 + 0.5j)
    x = rng.standard_normal((2, n, 3)) + 1j * rng.standard_normal((2, n, 3))
    say("matvec fp32", name)
    s = DDASolver(mask, d, m_h)
    y = from_dev(s.matvec(E, eps, to_dev(x, torch.complex64), precision="mixed"))
    c, alpha, k, _ = system(mask, d, eps, m_h, E)
    for r in range(2):
        ref = cdense.matvec(c, alpha, k, x[r])
        assert rel(y[r], ref) <= 1e-5, (name, rel(y[r], ref))
    s.close()


# ------------------------------------------------------- solve + reductions
SOLVE_CASES = [
    ("glass", 1.45 + 0j, 0.55),
    ("vacuum", 1.0 + 0j, 0.55),
    ("cherenkov", 2.0 + 0j, 0.70),
    ("absorbing_cherenkov", 2.0 + 0.01j, 0.70),
]


def _small_particle():
    mask = W.capped_rod_mask(12, 6, 6, 2.0, 6.0, 24.0)
    return mask, 2.0, np.array([[16.0, 1.0, 0.0], [0.0, 7.0, 3.0]])


@pytest.mark.parametrize("name,m_h,beta", SOLVE_CASES)
@pytest.mark.parametrize("precision,bar", [("fp64", 1e-9), ("mixed", 1e-5)])
@pytest.mark.parametrize("solver", ["bicgstab", "cocg"])
def test_losses_match_oracle(name, m_h, beta, precision, bar, solver):
    mask, d, r0 = _small_particle()
    n = int(mask.sum())
    energies = np.array([1.8, 2.6])
    eps_tab = W.drude_eps(energies)
    eps = np.repeat(eps_tab[:, None], n, axis=1)
    say("losses", name, precision, solver, "n_occ", n)
    s = DDASolver(mask, d, m_h, precision=precision, tol=1e-12 if precision == "fp64" else 1e-10,
                  maxit=20000, solver=solver)
    P, info = s.spectrum(energies, beta, eps, r0)
    say("  iterations", [i.iters for i in info], "matvecs", [i.matvecs for i in info])
    for i, inf in enumerate(info):
        assert inf.status == 0 and inf.rel_residual <= (1e-12 if precision == "fp64" else 1e-10)
    k = 0
    for ie, E in enumerate(energies):
        for t in range(r0.shape[0]):
            ref = solve_point(mask, d, eps[ie], m_h, beta, r0[t], E, method="lu")
            got = P[k]
            vals = [ref.p_eels, ref.p_ext, ref.p_abs, ref.p_cl]
            scale = max(abs(v) for v in vals)
            for g, v, nm in zip(got, vals, ["eels", "ext", "abs", "cl"]):
                err = abs(g - v) / max(abs(v), 1e-3 * scale)
                say(f"  E={E} t={t} {nm}: gpu={g:.15e} oracle={v:.15e} rel={err:.2e}")
                assert err <= bar, (name, precision, E, t, nm, err)
            k += 1
    s.close()


@pytest.mark.parametrize("solver,precision,bar", [("cocg", "mixed", 1e-5), ("cocg", "fp64", 1e-9),
                                                  ("bicgstab", "mixed", 1e-5),
                                                  ("bicgstab", "fp64", 1e-9)])
def test_losses_when_precisions_use_different_chains(solver, precision, bar):
    """A 5 x 25 x 25 lattice (FFT grid 12 x 64 x 64): the FP32 matvecs of the
    mixed path run the three-pass chain (its 64 x 64 plane fits in LDS in
    FP32), its FP64 reliable updates and the FP64 path the five-pass one; both
    D layouts come from one build."""
    mask = W.random_mask(5, 25, 25, 0.6, seed=9)
    d = 1.3
    n = int(mask.sum())
    energies = np.array([2.1])
    eps = np.repeat(W.drude_eps(energies)[:, None], n, axis=1)
    r0 = np.array([[9.0, 0.65, 0.0]])
    say("mixed chains", precision, "n_occ", n)
    s = DDASolver(mask, d, 1.45, precision=precision, solver=solver,
                  tol=1e-12 if precision == "fp64" else 1e-10, maxit=20000)
    assert tuple(s.grid) == (12, 64, 64)
    s.set_timing(True)
    P, info = s.spectrum(energies, 0.55, eps, r0)
    assert info[0].status == 0
    # the FP64 matvecs (every one on the FP64 path, the checks of the mixed
    # one) take the five-pass chain; the FP32 ones take the fused yz kernel
    assert s.kernel_time("zconv")[1] > 0
    assert (s.kernel_time("yzconv")[1] > 0) == (precision == "mixed")
    s.set_timing(False)
    ref = solve_point(mask, d, eps[0], 1.45, 0.55, r0[0], energies[0], method="lu")
    vals = [ref.p_eels, ref.p_ext, ref.p_abs, ref.p_cl]
    for g, v in zip(P[0], vals):
        assert abs(g - v) <= bar * abs(v), (g, v)
    s.close()


@pytest.mark.parametrize("solver,precision,bar", [("bicgstab", "mixed", 1e-5),
                                                  ("bicgstab", "fp64", 1e-9),
                                                  ("cocg", "mixed", 1e-5)])
def test_losses_when_every_precision_uses_the_five_pass_chain(solver, precision, bar):
    """A sparse 3 x 33 x 33 lattice: its yz grid is longer than 64, so the
    FP32 matvecs run the five-pass chain too, with the fused partial rows of
    the pack kernel (COCG x^T y, BiCGStab <rhat, v> and <t, s>, ||t||^2) in
    both precisions; against dense LU."""
    mask = W.random_mask(3, 33, 33, 0.3, seed=11)
    d = 1.2
    n = int(mask.sum())
    energies = np.array([2.2])
    eps = np.repeat(W.drude_eps(energies)[:, None], n, axis=1)
    r0 = np.array([[6.0, 0.6, 0.0]])
    say("five-pass chains", solver, precision, "n_occ", n)
    s = DDASolver(mask, d, 1.45, precision=precision, solver=solver,
                  tol=1e-12 if precision == "fp64" else 1e-10, maxit=20000)
    assert s.grid[1] > 64 and s.grid[2] > 64, s.grid
    P, info = s.spectrum(energies, 0.55, eps, r0)
    assert info[0].status == 0, info[0]
    ref = solve_point(mask, d, eps[0], 1.45, 0.55, r0[0], energies[0], method="lu")
    vals = [ref.p_eels, ref.p_ext, ref.p_abs, ref.p_cl]
    scale = max(abs(v) for v in vals)
    for g, v, nm in zip(P[0], vals, ["eels", "ext", "abs", "cl"]):
        err = abs(g - v) / max(abs(v), 1e-3 * scale)
        say(f"  {nm}: gpu={g:.15e} oracle={v:.15e} rel={err:.2e}")
        assert err <= bar, (nm, err)
    s.close()


def _xy_grid(n):
    """FFT length the library picks for n cells (the smallest supported length
    of at least 2 n - 1)."""
    return next(s for s in (96, 128) if s >= 2 * n - 1)


@pytest.mark.parametrize("nx,ny,nz,frac", [(48, 48, 3, 0.025), (64, 64, 2, 0.02),
                                           (44, 37, 3, 0.03)])
@pytest.mark.parametrize("solver", ["cocg", "bicgstab", "qmr"])
@pytest.mark.parametrize("n_energy", [2, 20])
def test_losses_on_the_fused_xy_chain(nx, ny, nz, frac, solver, n_energy):
    """Sparse nx x ny x nz lattices (FFT grids 96 x 96 and 128 x 128 in x
    and y; the last with nx != ny and ny below half the grid, so the rows past
    ny and the columns past nx are padding): the FP32 matvecs of the mixed path
    run the fused xy chain (xyfft, zconv, ixyfft_pack) with the Krylov updates
    in its first kernel (folded with the end of the previous iteration for
    batches of at most eight, as for 2 energies and the last of the 20) and the
    fused partial rows of its pack; against dense LU at every energy."""
    mask = W.random_mask(nx, ny, nz, frac, seed=nx + ny + nz)
    d = 1.1
    n = int(mask.sum())
    energies = np.linspace(1.7, 2.9, n_energy)
    eps = np.repeat(W.drude_eps(energies)[:, None], n, axis=1)
    r0 = np.array([[nx * d / 2 + 0.55, ny * d + 2.0, 0.0]])
    say("fused xy chain", nx, ny, nz, solver, n_energy, "n_occ", n)
    s = DDASolver(mask, d, 1.45, precision="mixed", solver=solver, tol=1e-10, maxit=20000)
    assert s.grid[0] == _xy_grid(nx) and s.grid[1] == _xy_grid(ny) == s.grid[0], s.grid
    s.set_timing(True)
    s.matvec(2.0, eps[0], torch.zeros((3, 3, n), dtype=torch.complex64, device="cuda"),
             precision="mixed")
    torch.cuda.synchronize()
    assert [s.kernel_time(k)[1] for k in ("xyfft", "zconv", "ixyfft_pack")] == [1, 1, 1]
    assert [s.kernel_time(k)[1] for k in ("unpack_xfft", "yfft", "iyfft", "ixfft_pack")] == [0] * 4
    s.set_timing(False)
    P, info = s.spectrum(energies, 0.55, eps, r0)
    say("  iterations", [i.iters for i in info])
    assert all(i.status == 0 for i in info), info
    for ie, E in enumerate(energies):
        ref = solve_point(mask, d, eps[ie], 1.45, 0.55, r0[0], E, method="lu")
        vals = [ref.p_eels, ref.p_ext, ref.p_abs, ref.p_cl]
        scale = max(abs(v) for v in vals)
        for g, v, nm in zip(P[ie], vals, ["eels", "ext", "abs", "cl"]):
            err = abs(g - v) / max(abs(v), 1e-3 * scale)
            assert err <= 1e-5, (nx, ny, solver, E, nm, err)
    s.close()


@pytest.mark.parametrize("nx,ny", [(48, 48), (64, 64), (40, 44), (47, 34), (50, 60)])
def test_fused_xy_chain_matvec_matches_dense(nx, ny):
    """The FP32 products y = A x and G_off x of the fused xy chain on a fully
    occupied nx x ny x 3 lattice (FFT grids 96 x 96 or 128 x 128 in x and y:
    exactly twice the box, or with padding rows and columns past ny and nx,
    nx above or below ny) against the oracle's dense rows, for 16 right-hand
    sides at once."""
    mask = np.ones((3, ny, nx), np.uint8)
    n = int(mask.sum())
    E = 2.2
    eps = np.full(n, -6.0 + 0.9j)
    rng = np.random.default_rng(nx * 1000 + ny)
    x = rng.standard_normal((16, n, 3)) + 1j * rng.standard_normal((16, n, 3))
    s = DDASolver(mask, 1.0, 1.45)
    assert s.grid[0] == _xy_grid(nx) and s.grid[1] == _xy_grid(ny) == s.grid[0], s.grid
    s.set_timing(True)
    s.matvec(E, eps, torch.zeros((16, n, 3), dtype=torch.complex64, device="cuda"),
             precision="mixed")
    torch.cuda.synchronize()
    assert [s.kernel_time(k)[1] for k in ("xyfft", "ixyfft_pack")] == [1, 1]
    s.set_timing(False)
    xd = to_dev(x, torch.complex64)
    y = from_dev(s.matvec(E, eps, xd, precision="mixed"))
    yi = from_dev(s.matvec(E, None, xd, precision="mixed", interaction_only=True))
    c, alpha, k, _ = system(mask, 1.0, eps, 1.45, E)
    rows = np.unique(np.concatenate([[0, n - 1, n // 2], rng.integers(0, n, 125)]))
    for r in range(x.shape[0]):
        for got, io in ((y[r], False), (yi[r], True)):
            ref = cdense.matvec_rows(c, alpha, k, x[r], rows, interaction_only=io)
            err = np.max(np.abs(got[rows] - ref)) / np.max(np.abs(ref))
            say("  xy chain", nx, ny, "rhs", r, "G only" if io else "A", "err", err)
            assert err <= 1e-5, (r, io, err)
    s.close()


@pytest.mark.parametrize("nx", [32, 33, 64])
@pytest.mark.parametrize("solver,precision,bar", [("cocg", "mixed", 1e-5), ("bicgstab", "mixed", 1e-5),
                                                  ("cocg", "fp64", 1e-9)])
def test_losses_on_long_x_grids(nx, solver, precision, bar):
    """Rods with x grids of 64, 96 and 128 on a 12 x 12 yz grid (three-pass
    chain with the LDS-tiled yz kernel; the fused direction update and the
    x^T y rows of COCG included) against dense LU."""
    mask = W.capped_rod_mask(nx, 6, 6, 1.0, 3.0, float(nx))
    n = int(mask.sum())
    energies = np.array([2.3])
    eps = np.repeat(W.drude_eps(energies)[:, None], n, axis=1)
    r0 = np.array([[nx / 2 + 2.0, 0.5, 0.0]])
    say("register x passes", nx, solver, precision, "n_occ", n)
    s = DDASolver(mask, 1.0, 1.45, precision=precision, solver=solver,
                  tol=1e-12 if precision == "fp64" else 1e-10, maxit=20000)
    P, info = s.spectrum(energies, 0.55, eps, r0)
    assert info[0].status == 0, info[0]
    ref = solve_point(mask, 1.0, eps[0], 1.45, 0.55, r0[0], energies[0], method="lu")
    vals = [ref.p_eels, ref.p_ext, ref.p_abs, ref.p_cl]
    scale = max(abs(v) for v in vals)
    for g, v, nm in zip(P[0], vals, ["eels", "ext", "abs", "cl"]):
        err = abs(g - v) / max(abs(v), 1e-3 * scale)
        say(f"  {nm}: gpu={g:.15e} oracle={v:.15e} rel={err:.2e}")
        assert err <= bar, (nx, nm, err)
    s.close()


@pytest.mark.parametrize("solver,precision", [("bicgstab", "fp64"), ("cocg", "fp64"),
                                              ("cocg", "mixed")])
def test_c1_full_size_matches_oracle_golden(solver, precision):
    with open(os.path.join(HERE, "golden", "oracle_c1.json")) as f:
        gold = json.load(f)
    w = W.c1_single_solve()
    say("c1 full size", w.n_occ, solver, precision)
    s = DDASolver(w.mask, w.d, w.m_h, tol=1e-12 if precision == "fp64" else 1e-10, maxit=50000,
                  solver=solver, precision=precision)
    P, info = s.spectrum(w.energies, w.beta, w.eps_dipoles(0)[None, :], w.r0)
    say("iters", info[0].iters, "residual", info[0].rel_residual)
    for j, nm in enumerate(["p_eels", "p_ext", "p_abs", "p_cl"]):
        err = abs(P[0][j] - gold[nm]) / abs(gold[nm])
        say(f"  {nm}: gpu={P[0][j]:.15e} oracle={gold[nm]:.15e} rel={err:.2e}")
        assert err <= (1e-9 if precision == "fp64" else 1e-5)
    s.close()


@pytest.mark.parametrize("solver,precision", [("bicgstab", "fp64"), ("cocg", "fp64"),
                                              ("cocg", "mixed")])
def test_batch_equals_single(solver, precision):
    """Energies x trajectories as one batch give the same result as one solve
    per right-hand side (each right-hand side runs the same arithmetic in the
    same order whatever else shares the launch).  Twelve right-hand sides: the
    COCG batch starts above the slot count up to which the finalizer is folded
    into the direction update and ends below it, while each single solve
    folds throughout."""
    mask, d, r0 = _small_particle()
    n = int(mask.sum())
    energies = np.array([1.5, 1.8, 2.0, 2.2, 2.5, 2.8])
    eps = np.repeat(W.drude_eps(energies)[:, None], n, axis=1)
    s = DDASolver(mask, d, 1.45, tol=1e-11, maxit=20000, solver=solver, precision=precision)
    Pb, _ = s.spectrum(energies, 0.55, eps, r0)
    k = 0
    for ie, E in enumerate(energies):
        for t in range(r0.shape[0]):
            P1, _ = s.spectrum([E], 0.55, eps[ie:ie + 1], r0[t:t + 1])
            assert np.allclose(Pb[k], P1[0], rtol=1e-13, atol=0), (ie, t)
            k += 1
    s.close()


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("timing", [False, True])
def test_cocg_graph_replay_equals_direct_launches(precision, timing):
    """COCG intervals sent as captured, replayed and updated HIP graphs give
    bit-identical iterates, residuals and counts to the same kernels launched
    one by one (and with kernel timing on, which launches one by one).
    Energies converge at different iterations, so the active list shrinks and
    the graph is updated many times; torch work and synchronisations run
    between the solves."""
    mask, d, r0 = _small_particle()
    n = int(mask.sum())
    energies = np.linspace(1.2, 3.0, 7)
    eps = np.repeat(W.drude_eps(energies)[:, None], n, axis=1)
    out = []
    for graphs in (False, True, True):
        s = DDASolver(mask, d, 1.45, tol=1e-11, maxit=20000, solver="cocg", precision=precision,
                      check_every=4, use_graphs=graphs)
        if timing:
            s.set_timing(True, kernels=["yzconv", "zconv", "ixfft_pack"])
        e = s.einc(energies, 0.55, r0)
        p, info, st = s.solve(energies, eps, e, r0.shape[0])
        assert st == L.DDA_OK
        _ = (torch.ones(1000, device="cuda") * 2).sum().item()  # unrelated torch work
        torch.cuda.synchronize()
        out.append((from_dev(p), [(i.iters, i.matvecs, i.rel_residual, i.status) for i in info]))
        if timing:
            assert sum(s.kernel_time(k)[1] for k in ("yzconv", "zconv")) > 0
        s.close()
    iters = [i[0] for i in out[0][1]]
    assert len(set(iters)) > 1, iters  # the active list did shrink
    for pk, ik in out[1:]:
        assert ik == out[0][1]
        assert np.array_equal(pk, out[0][0])


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_bicgstab_same_iterates_for_any_interval_and_graphs(precision):
    """BiCGStab closes an iteration either in the next iteration's direction
    update or, at the end of an interval, in a finalize kernel.  Both forms run
    the same arithmetic in the same order, so the solution, the iteration count
    and the residual are bit-identical for check intervals of 1 (every
    iteration closed by the finalize kernel), 5 and 16, with captured graphs
    and without.  Energies converge at different iterations, so slots go
    quiet inside intervals."""
    mask, d, r0 = _small_particle()
    n = int(mask.sum())
    energies = np.linspace(1.2, 3.0, 5)
    eps = np.repeat(W.drude_eps(energies)[:, None], n, axis=1)
    out = []
    for check, graphs in ((1, False), (5, True), (16, True), (16, False)):
        s = DDASolver(mask, d, 1.45, tol=1e-11, maxit=20000, solver="bicgstab",
                      precision=precision, check_every=check, use_graphs=graphs)
        e = s.einc(energies, 0.55, r0)
        p, info, st = s.solve(energies, eps, e, r0.shape[0])
        assert st == L.DDA_OK
        torch.cuda.synchronize()
        out.append((from_dev(p), [(i.iters, i.rel_residual, i.status) for i in info]))
        s.close()
    iters = [i[0] for i in out[0][1]]
    assert len(set(iters)) > 1, iters
    for pk, ik in out[1:]:
        assert ik == out[0][1]
        assert np.array_equal(pk, out[0][0])


ZC2_CODES = [tx | ((nt // 64) << 6) | (alt << 12) for tx in (2, 4, 8, 16) for nt in (256, 512)
             for alt in (0, 1)]


@pytest.mark.parametrize("shape", [(12, 12, 12), (12, 12, 16), (16, 8, 12), (16, 12, 24),
                                   (8, 20, 40), (6, 20, 64), (48, 48, 24)])
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_every_autotuner_candidate_gives_identical_matvecs(shape, precision):
    """The autotuner's tile candidates only regroup lines into blocks: every
    candidate of the five-pass z and y passes (my != mz) gives the same matvec
    to the last bit (the fused yz kernel of a cubic grid has a single shape
    per length; on the 48 x 48 x 24 lattice the FP32 matvecs take the fused
    xy chain, whose z pass has the same candidates).  z grids of 48 and 96 take the two-stage z pass, whose codes
    are TX | (threads / 64) << 6 | plan << 12; the two radix plans of a length
    (first radix 16 or 8) round differently, so results are bit-identical
    within a plan and agree to rounding across plans."""
    nx, ny, nz = shape
    mask = np.ones((nz, ny, nx), np.uint8)
    s = DDASolver(mask, 1.0, 1.45)
    n = s.n_occ
    eps = np.full(n, -8 + 0.7j)
    dt = torch.complex128 if precision == "fp64" else torch.complex64
    prec = L.DDA_PREC_FP64 if precision == "fp64" else L.DDA_PREC_MIXED
    x = torch.randn((5, 3, n), dtype=dt, device="cuda")
    mx, my, mz = s.grid
    yzc = [0, 256, 512, 1024] if my == mz else [0]
    zc = [0] if my == mz else [0, 1, 2, 4, 8] + ZC2_CODES
    mc = [0] if my == mz else [0, 4, 8, 16, 32]
    ref = {}
    tried = 0
    for yt in yzc:
        for zt in zc:
            for mt in mc:
                try:
                    L.dda_set_tuning(s.ctx, prec, zt, mt, yt)
                except L.DDAError:
                    continue  # not a candidate for this grid and precision
                y = s.matvec(2.2, eps, x, precision=precision).cpu().numpy()
                tried += 1
                plan = (zt >> 12) & 1
                if plan not in ref:
                    ref[plan] = y
                else:
                    assert np.array_equal(y, ref[plan]), (yt, zt, mt)
    assert tried >= (1 if my == mz else 3)
    if len(ref) == 2:
        bar = 1e-13 if precision == "fp64" else 1e-6
        assert np.linalg.norm(ref[0] - ref[1]) <= bar * np.linalg.norm(ref[0])
    s.close()


def test_device_resident_permittivities_equal_host_ones():
    """Permittivities passed in device memory are read in place and give the
    same solution and probabilities as the same values passed from the host."""
    mask, d, r0 = _small_particle()
    n = int(mask.sum())
    E = np.array([1.6, 2.4])
    eps = np.repeat(W.drude_eps(E)[:, None], n, axis=1)
    eps[:, ::7] *= 1.3  # not homogeneous
    s = DDASolver(mask, d, 1.45, tol=1e-10, solver="cocg", precision="mixed")
    P_h, info_h = s.spectrum(E, 0.55, eps, r0)
    P_d, info_d = s.spectrum(E, 0.55, torch.from_numpy(eps).cuda(), r0)
    assert [i.iters for i in info_h] == [i.iters for i in info_d]
    assert np.array_equal(P_h, P_d)
    s.close()


# ------------------------------------------------------------ edge cases
def test_errors_and_degenerate_inputs():
    mask = W.sphere_mask(6, 1.0, 3.0)
    s = DDASolver(mask, 1.0, 1.45)
    n = s.n_occ
    # trajectory through a dipole centre: b = 0 in eq. (25)
    with pytest.raises(L.DDAError) as ei:
        s.einc([2.0], 0.55, np.array([[0.5, 0.5, 0.0]]))
    assert ei.value.status == L.DDA_ESINGULAR
    # beta_h = 1
    with pytest.raises(L.DDAError) as ei:
        s.einc([2.0], 1.0 / 1.45, np.array([[5.0, 0.0, 0.0]]))
    assert ei.value.status == L.DDA_ESINGULAR
    e = s.einc([2.0], 0.55, np.array([[5.0, 0.0, 0.0]]))
    with pytest.raises(L.DDAError) as ei:
        s.solve([2.0], np.full((1, n), np.nan + 0j), e, 1)
    assert ei.value.status == L.DDA_EINVAL
    # iteration limit: best iterate kept, status reported
    s2 = DDASolver(mask, 1.0, 1.45, tol=1e-12, maxit=1, check_every=1)
    e2 = s2.einc([2.0], 0.55, np.array([[5.0, 0.0, 0.0]]))
    p, info, st = s2.solve([2.0], np.full((1, n), -10 + 1j), e2, 1, raise_on_error=False)
    assert st == L.DDA_ENOCONV and info[0].status == L.DDA_ENOCONV and info[0].iters >= 1
    s.close()
    s2.close()
    # non-passive host
    with pytest.raises(L.DDAError):
        DDASolver(mask, 1.0, 1.45 - 0.1j)
    # empty lattice: every call is a no-op
    s3 = DDASolver(np.zeros((4, 4, 4), np.uint8), 1.0, 1.45)
    assert s3.n_occ == 0
    s3.close()


# --------------------------------------------- full sizes, sampled outputs
@pytest.mark.parametrize("wname", ["c2", "c3"])
def test_full_size_matvec_sampled(wname):
    w = W.c2_nanorod_spectrum() if wname == "c2" else W.c3_cherenkov()
    mask, d, m_h = w.mask, w.d, w.m_h
    n = int(mask.sum())
    E = float(w.energies[len(w.energies) // 2])
    eps = np.full(n, w.eps_table()[len(w.energies) // 2])
    rng = np.random.default_rng(11)
    x = rng.standard_normal((1, n, 3)) + 1j * rng.standard_normal((1, n, 3))
    say("full-size matvec", wname, "n_occ", n)
    s = DDASolver(mask, d, m_h)
    y = from_dev(s.matvec(E, eps, to_dev(x)))[0]
    y32 = from_dev(s.matvec(E, eps, to_dev(x, torch.complex64), precision="mixed"))[0]
    c, alpha, k, _ = system(mask, d, eps, m_h, E)
    rows = np.unique(np.concatenate([[0, n - 1], rng.integers(0, n, 62)]))
    ref = cdense.matvec_rows(c, alpha, k, x[0], rows)
    scale = np.max(np.abs(ref))
    err = np.max(np.abs(y[rows] - ref)) / scale
    err32 = np.max(np.abs(y32[rows] - ref)) / scale
    say("  fp64 sampled max err", err, " fp32", err32)
    assert err <= 1e-12
    assert err32 <= 1e-5
    # the electron field at full size (all dipoles, FP64)
    e = from_dev(s.einc([E], w.beta, w.r0))
    for t in range(w.r0.shape[0]):
        ref_e = el.incident_field(c, E, w.beta, m_h, w.r0[t])
        assert np.max(np.abs(e[t] - ref_e)) <= 1e-13 * np.max(np.abs(ref_e))
    s.close()
