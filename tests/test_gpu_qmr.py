"""GPU parity of the QMR solver for complex-symmetric systems (section S5's
solver family) against the FP64 CPU oracle's dense LU, on the three-pass and
five-pass chains, in FP64 (1e-9) and mixed precision (1e-5); and its
determinism: batch = single solve and captured graphs = direct launches, bit
for bit."""

import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

import workloads as W  # noqa: E402
from oracle.dda import solve_point  # noqa: E402
from paper_2208_01348_amd import _lib as L  # noqa: E402
from paper_2208_01348_amd.solver import DDASolver  # noqa: E402


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def check(P, refs, bar, label):
    for got, ref in zip(P, refs):
        vals = [ref.p_eels, ref.p_ext, ref.p_abs, ref.p_cl]
        scale = max(abs(v) for v in vals)
        for g, v, nm in zip(got, vals, ["eels", "ext", "abs", "cl"]):
            err = abs(g - v) / max(abs(v), 1e-3 * scale)
            say(f"  {label} {nm}: gpu={g:.15e} oracle={v:.15e} rel={err:.2e}")
            assert err <= bar, (label, nm, err)


CASES = [("glass", 1.45 + 0j, 0.55), ("cherenkov", 2.0 + 0j, 0.70),
         ("absorbing_cherenkov", 2.0 + 0.01j, 0.70)]
LATTICES = {
    # three-pass chain (yz plane in LDS) in both precisions
    "rod_12x6x6": (lambda: W.capped_rod_mask(12, 6, 6, 2.0, 6.0, 24.0), 2.0, (16.0, 1.0, 0.0)),
    # five-pass chain in both precisions (yz grid longer than 64)
    "sparse_3x33x33": (lambda: W.random_mask(3, 33, 33, 0.3, seed=11), 1.2, (6.0, 0.6, 0.0)),
}


@pytest.mark.parametrize("lattice", list(LATTICES))
@pytest.mark.parametrize("name,m_h,beta", CASES)
@pytest.mark.parametrize("precision,bar", [("fp64", 1e-9), ("mixed", 1e-5)])
def test_qmr_losses_match_oracle(lattice, name, m_h, beta, precision, bar):
    mk, d, r0 = LATTICES[lattice]
    mask = mk()
    n = int(mask.sum())
    energies = np.array([1.8, 2.6])
    eps = np.repeat(W.drude_eps(energies)[:, None], n, axis=1)
    say("qmr", lattice, name, precision, "n_occ", n)
    s = DDASolver(mask, d, m_h, precision=precision, solver="qmr",
                  tol=1e-12 if precision == "fp64" else 1e-10, maxit=20000, check_every=8)
    P, info = s.spectrum(energies, beta, eps, np.array([r0]))
    say("  iterations", [i.iters for i in info], "matvecs", [i.matvecs for i in info],
        "residuals", [i.rel_residual for i in info])
    assert all(i.status == 0 for i in info), info
    refs = [solve_point(mask, d, eps[i], m_h, beta, r0, float(energies[i]), method="lu")
            for i in range(energies.size)]
    check(P, refs, bar, f"qmr/{precision}")
    s.close()


def test_qmr_on_the_nanorod_chain():
    """The sparse 96 x 24 x 24 lattice (x grid 192, 48 x 48 yz plane): QMR in
    both precisions against dense LU."""
    mask = W.random_mask(96, 24, 24, 0.012, seed=21)
    n = int(mask.sum())
    d = 20.0 / 24.0
    energies = np.array([2.45])
    eps = np.repeat(W.drude_eps(energies)[:, None], n, axis=1)
    r0 = np.array([[45.0, 0.0, 0.0]])
    ref = solve_point(mask, d, eps[0], 1.45, 0.55, r0[0], float(energies[0]), method="lu")
    for precision, bar in [("fp64", 1e-9), ("mixed", 1e-5)]:
        s = DDASolver(mask, d, 1.45, precision=precision, solver="qmr",
                      tol=1e-12 if precision == "fp64" else 1e-10, maxit=20000)
        P, info = s.spectrum(energies, 0.55, eps, r0)
        assert info[0].status == 0, info
        check(P, [ref], bar, f"nanorod qmr/{precision}")
        s.close()


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_qmr_batch_equals_single_and_graphs_equal_direct(precision):
    mask = W.capped_rod_mask(12, 6, 6, 2.0, 6.0, 24.0)
    n = int(mask.sum())
    energies = np.linspace(1.3, 2.9, 5)
    eps = np.repeat(W.drude_eps(energies)[:, None], n, axis=1)
    r0 = np.array([[16.0, 1.0, 0.0]])
    outs = []
    for graphs in (True, False):
        s = DDASolver(mask, 2.0, 1.45, precision=precision, solver="qmr", tol=1e-11,
                      maxit=20000, check_every=6, use_graphs=graphs)
        e = s.einc(energies, 0.55, r0)
        p, info, st = s.solve(energies, eps, e, 1)
        assert st == L.DDA_OK
        torch.cuda.synchronize()
        outs.append((p.cpu().numpy(), [(i.iters, i.matvecs, i.rel_residual) for i in info]))
        if graphs:
            for i in (0, 2, 4):
                p1, info1, st1 = s.solve(energies[i:i + 1], eps[i:i + 1], e[i:i + 1], 1)
                assert st1 == L.DDA_OK
                assert (info1[0].iters, info1[0].matvecs, info1[0].rel_residual) == outs[0][1][i]
                assert np.array_equal(p1.cpu().numpy()[0], outs[0][0][i])
        s.close()
    assert len(set(i[0] for i in outs[0][1])) > 1  # slots left the active list at different times
    assert outs[0][1] == outs[1][1]
    assert np.array_equal(outs[0][0], outs[1][0])
