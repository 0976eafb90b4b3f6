"""Named synthetic workloads.

They stand in for the paper's experiments, whose optical data and measured
spectra are not available: silver/gold spheres and rods probed by ~100 keV
electrons (beta ~ 0.55) in vacuum, in glass-like hosts (m_h = 1.45) and in
dense Cherenkov hosts (m_h = 2), on lattices of 16-128 dipoles per side
(sections 3.2-3.4).  Every random draw is seeded.
"""

from __future__ import annotations

from dataclasses import dataclass, field
from typing import Callable, List, Optional, Tuple

import numpy as np

from .materials import drude_eps
from .shapes import capped_rod_mask, ellipsoid_mask, sphere_mask


@dataclass
class Workload:
    name: str
    nx: int
    ny: int
    nz: int
    d: float                       # dipole size, nm
    mask_fn: Callable[[int, int, int, float], np.ndarray]  # (nx, ny, nz, d) -> mask
    m_h: complex                   # host refractive index
    beta: float                    # electron speed / c
    r0: np.ndarray                 # [n_traj][3] trajectory points, nm
    energies: np.ndarray           # [n_energy] loss energies, eV
    eps_fn: Callable[[np.ndarray], np.ndarray]  # energies -> absolute eps [n_energy]
    polarizability: str = "ldr"
    tol: float = 1e-10
    precision: str = "fp64"
    notes: str = ""
    _mask: Optional[np.ndarray] = field(default=None, repr=False)

    @property
    def mask(self) -> np.ndarray:
        if self._mask is None:
            self._mask = self.mask_fn(self.nx, self.ny, self.nz, self.d)
        return self._mask

    @property
    def n_occ(self) -> int:
        return int(self.mask.sum())

    @property
    def n_traj(self) -> int:
        return int(np.asarray(self.r0).reshape(-1, 3).shape[0])

    def eps_table(self) -> np.ndarray:
        """Absolute permittivity per energy, complex128 [n_energy]."""
        return np.asarray(self.eps_fn(np.asarray(self.energies)), dtype=np.complex128)

    def eps_dipoles(self, e_index: int) -> np.ndarray:
        """Per-dipole absolute permittivity at one energy (homogeneous particle)."""
        return np.full(self.n_occ, self.eps_table()[e_index], dtype=np.complex128)


def c1_single_solve() -> Workload:
    """16^3 sphere (R = 8 nm, d = 1 nm), eps = -10+1i, host 1.45, beta 0.55,
    electron 2 nm outside the surface, one energy 2.5 eV, LDR, BiCGStab."""
    n, d, R = 16, 1.0, 8.0
    return Workload(
        name="c1_sphere16_single", nx=n, ny=n, nz=n, d=d,
        mask_fn=lambda nx, ny, nz, dd: sphere_mask(nx, dd, R),
        m_h=1.45 + 0j, beta=0.55, r0=np.array([[R + 2.0, 0.0, 0.0]]),
        energies=np.array([2.5]),
        eps_fn=lambda E: np.full(np.shape(E), -10.0 + 1.0j),
        tol=1e-10,
    )


def c2_nanorod_spectrum(n_energy: int = 128) -> Workload:
    """Capped rod 20 x 20 x 80 nm lying along x on 96 x 24 x 24 cells
    (d = 20/24 nm); electron along +z, 5 nm beyond the tip apex (x0 = 45 nm);
    Drude eps 9.5 - 9.0^2/(E(E + 0.07i)); 128 energies over [1, 3] eV."""
    nx, ny, nz = 96, 24, 24
    d = 20.0 / 24.0
    return Workload(
        name="c2_rod96x24x24_spectrum", nx=nx, ny=ny, nz=nz, d=d,
        mask_fn=lambda nx, ny, nz, dd: capped_rod_mask(nx, ny, nz, dd, radius=10.0, length=80.0,
                                                       axis="x"),
        m_h=1.45 + 0j, beta=0.55, r0=np.array([[45.0, 0.0, 0.0]]),
        energies=np.linspace(1.0, 3.0, n_energy),
        eps_fn=lambda E: drude_eps(E, 9.5, 9.0, 0.07),
        tol=1e-10,
    )


def c3_cherenkov(n_energy: int = 64) -> Workload:
    """64^3 sphere (R = 32 nm, d = 1 nm) in an absorbing dense host
    m_h = 2.0 + 0.01i, beta = 0.70 (beta_h = 1.4 + 0.007i); trajectories
    2 nm outside the surface and through the centre (a cell corner)."""
    n, d, R = 64, 1.0, 32.0
    return Workload(
        name="c3_sphere64_cherenkov", nx=n, ny=n, nz=n, d=d,
        mask_fn=lambda nx, ny, nz, dd: sphere_mask(nx, dd, R),
        m_h=2.0 + 0.01j, beta=0.70,
        r0=np.array([[R + 2.0, 0.0, 0.0], [0.0, 0.0, 0.0]]),
        energies=np.linspace(1.5, 4.0, n_energy),
        eps_fn=lambda E: drude_eps(E, 9.5, 9.0, 0.02),
        tol=1e-10, precision="mixed",
    )


def c4_impact_map(n_energy: int = 32, n_side: int = 16, seed: int = 2208_01348) -> Workload:
    """Random ellipsoid (semi-axes ~ U[15, 40] nm, seeded) on 48^3 cells with
    d = 2 max(a, b, c)/48; a 16 x 16 impact grid on cell boundaries x 32
    energies over [1, 4] eV; host 1.45, beta 0.55, Drude as the rod."""
    rng = np.random.default_rng(seed)
    a, b, c = rng.uniform(15.0, 40.0, size=3)
    n = 48
    d = 2.0 * max(a, b, c) / n
    j = np.arange(n_side)
    xs = -24.0 * d + (3 * j + 2) * d
    X0, Y0 = np.meshgrid(xs, xs, indexing="ij")
    r0 = np.stack([X0.ravel(), Y0.ravel(), np.zeros(X0.size)], axis=1)
    return Workload(
        name="c4_ellipsoid48_impact_map", nx=n, ny=n, nz=n, d=d,
        mask_fn=lambda nx, ny, nz, dd: ellipsoid_mask(nx, ny, nz, dd, a, b, c),
        m_h=1.45 + 0j, beta=0.55, r0=r0,
        energies=np.linspace(1.0, 4.0, n_energy),
        eps_fn=lambda E: drude_eps(E, 9.5, 9.0, 0.07),
        tol=1e-8, precision="mixed",
        notes=f"semi-axes a={a:.4f} b={b:.4f} c={c:.4f} nm",
    )


def c5_request_stream(n_requests: int = 2000, rate_per_s: float = 200.0, seed: int = 5,
                      sides=(24, 32, 48, 64, 96)) -> List[Tuple[float, Workload]]:
    """Poisson stream of spectrum requests: (arrival time s, workload)."""
    rng = np.random.default_rng(seed)
    t = np.cumsum(rng.exponential(1.0 / rate_per_s, size=n_requests))
    out = []
    for i in range(n_requests):
        shape = int(rng.integers(3))
        n = int(rng.choice(np.asarray(sides)))
        while True:
            m_h = float(rng.uniform(1.0, 2.0))
            beta = float(rng.uniform(0.4, 0.8))
            if abs(m_h * beta - 1.0) >= 1e-3:
                break
        n_e = int(rng.integers(8, 65))
        d = 1.0
        half = n * d / 2.0
        if shape == 0:
            mask_fn = (lambda nx, ny, nz, dd, half=half: sphere_mask(nx, dd, half))
            extent = half
        elif shape == 1:
            mask_fn = (lambda nx, ny, nz, dd, half=half: capped_rod_mask(
                nx, ny, nz, dd, radius=half / 4.0, length=2.0 * half, axis="x"))
            extent = half
        else:
            a, b, c = rng.uniform(0.3, 1.0, size=3) * half
            mask_fn = (lambda nx, ny, nz, dd, a=a, b=b, c=c: ellipsoid_mask(nx, ny, nz, dd, a, b, c))
            extent = a
        w = Workload(
            name=f"req{i}", nx=n, ny=n, nz=n, d=d, mask_fn=mask_fn,
            m_h=m_h + 0j, beta=beta, r0=np.array([[extent + 2.0, 0.0, 0.0]]),
            energies=np.linspace(1.0, 4.0, n_e),
            eps_fn=lambda E: drude_eps(E, 9.5, 9.0, 0.07),
            tol=1e-8, precision="mixed",
        )
        out.append((float(t[i]), w))
    return out


def scaled_down(w: Workload, factor: int, n_energy: Optional[int] = None) -> Workload:
    """Same physical shape on a lattice `factor` times coarser (d * factor)."""
    nx, ny, nz = w.nx // factor, w.ny // factor, w.nz // factor
    d = w.d * factor
    energies = w.energies if n_energy is None else np.linspace(
        float(w.energies[0]), float(w.energies[-1]), n_energy)
    return Workload(
        name=f"{w.name}_coarse{factor}", nx=nx, ny=ny, nz=nz, d=d, mask_fn=w.mask_fn,
        m_h=w.m_h, beta=w.beta, r0=np.array(w.r0, dtype=np.float64),
        energies=energies, eps_fn=w.eps_fn, polarizability=w.polarizability,
        tol=w.tol, precision=w.precision, notes=w.notes,
    )
