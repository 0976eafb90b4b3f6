"""The allocation-free electron-field entry point (dda_einc_electron_noalloc)
against dda_einc_electron through the C ABI: identical fields, bit for bit,
on two calls in a row (the second smaller, so stale staging contents would
show), and the size limits rejected with DDA_EINVAL."""

import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

import workloads as W  # noqa: E402
from oracle import electron as el  # noqa: E402
from oracle.lattice import dipole_centres  # noqa: E402
from paper_2208_01348_amd import _lib as L  # noqa: E402
from paper_2208_01348_amd.solver import DDASolver  # noqa: E402


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _field(s, n_rhs):
    return torch.full((n_rhs, 3, s.n_occ), complex(np.nan, np.nan), dtype=torch.complex128,
                      device="cuda")


@pytest.mark.parametrize("m_h,beta", [(1.45 + 0j, 0.55), (2.0 + 0.01j, 0.7)])
def test_noalloc_einc_equals_the_allocating_call(m_h, beta):
    mask = W.capped_rod_mask(24, 8, 8, 1.0, 4.0, 24.0)
    s = DDASolver(mask, 1.0, m_h)
    c = dipole_centres(mask, 1.0)
    calls = [
        (np.linspace(1.0, 3.9, 9), np.array([[14.0, 0.5, 0.0], [0.0, 6.0, 3.0], [-15.0, -1.0, 9.0],
                                              [2.0, -5.5, -4.0]])),
        (np.array([2.7, 1.3]), np.array([[13.0, 2.0, 1.0]])),  # smaller: stale rows would show
    ]
    for E, r0 in calls:
        say("noalloc einc", m_h, E.size, "energies", r0.shape[0], "trajectories")
        n_rhs = E.size * r0.shape[0]
        ref = _field(s, n_rhs)
        got = _field(s, n_rhs)
        with s._ordered():
            L.dda_einc_electron(s.ctx, E, beta, r0, ref.data_ptr())
            L.dda_einc_electron_noalloc(s.ctx, E, beta, r0, got.data_ptr())
        torch.cuda.synchronize()
        a, b = ref.cpu().numpy(), got.cpu().numpy()
        assert np.all(np.isfinite(b))
        assert np.array_equal(a, b)
        # and the oracle's eq. (25) at the stated tolerance of the FP64 field
        k = 0
        for e in E:
            for t in range(r0.shape[0]):
                want = el.incident_field(c, e, beta, m_h, r0[t]).T
                assert np.max(np.abs(b[k] - want)) <= 1e-13 * np.max(np.abs(want))
                k += 1
    s.close()


def test_noalloc_einc_rejects_sizes_beyond_its_limit():
    mask = W.sphere_mask(6, 1.0, 3.0)
    s = DDASolver(mask, 1.0, 1.45)
    E = np.linspace(1.0, 3.0, L.DDA_EINC_NOALLOC_MAX_ENERGIES + 1)
    r0 = np.array([[5.0, 0.0, 0.0]])
    out = torch.empty((E.size, 3, s.n_occ), dtype=torch.complex128, device="cuda")
    with pytest.raises(L.DDAError) as ei:
        L.dda_einc_electron_noalloc(s.ctx, E, 0.55, r0, out.data_ptr())
    assert ei.value.status == L.DDA_EINVAL
    r0m = np.tile(r0 + [[0.0, 0.0, 1.0]], (L.DDA_EINC_NOALLOC_MAX_TRAJ + 1, 1))
    with pytest.raises(L.DDAError) as ei:
        L.dda_einc_electron_noalloc(s.ctx, E[:1], 0.55, r0m, out.data_ptr())
    assert ei.value.status == L.DDA_EINVAL
    # the largest allowed batch of energies works and equals the allocating call
    E = E[:L.DDA_EINC_NOALLOC_MAX_ENERGIES]
    a = torch.empty((E.size, 3, s.n_occ), dtype=torch.complex128, device="cuda")
    b = torch.empty_like(a)
    with s._ordered():
        L.dda_einc_electron(s.ctx, E, 0.55, r0, a.data_ptr())
        L.dda_einc_electron_noalloc(s.ctx, E, 0.55, r0, b.data_ptr())
    torch.cuda.synchronize()
    assert torch.equal(a, b)
    s.close()
