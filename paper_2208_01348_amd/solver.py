"""Torch-facing convenience wrapper over the C ABI.

Torch provides device memory and the stream; every step of the path (the
electron field, the FFT matvecs, the Krylov iterations and the loss sums)
runs in libdda's HIP kernels.  This module only allocates tensors and passes
their pointers.

By default a solver runs on a non-blocking stream of its own (default
priority, created by the library), so that the library can capture its
iteration intervals as HIP graphs while other threads keep using the legacy
default stream; every call is ordered after the work already queued on
torch's current stream, and the current stream waits for the call's work
before torch touches the outputs.
"""

from __future__ import annotations

import contextlib
from dataclasses import dataclass
from typing import List, Optional, Sequence

import numpy as np
import torch

from . import _lib as L

_POL = {"ldr": L.DDA_POL_LDR, "cm": L.DDA_POL_CM, "rr": L.DDA_POL_RR}
_PREC = {"fp64": L.DDA_PREC_FP64, "mixed": L.DDA_PREC_MIXED}
_SOLVER = {"bicgstab": L.DDA_SOLVER_BICGSTAB, "cocg": L.DDA_SOLVER_COCG, "qmr": L.DDA_SOLVER_QMR}


@dataclass
class SolveInfo:
    iters: int
    matvecs: int
    rel_residual: float
    status: int


class DDASolver:
    """One lattice and host medium on one GPU (the current torch device)."""

    def __init__(self, mask: np.ndarray, d_nm: float, m_h: complex, polarizability: str = "ldr",
                 precision: str = "fp64", tol: float = 1e-10, maxit: int = 100000,
                 solver: str = "bicgstab",
                 check_every: int = 16, stream: Optional[torch.cuda.Stream] = None,
                 use_graphs: bool = True, interaction: str = "point"):
        m = np.ascontiguousarray(np.asarray(mask, dtype=np.uint8))
        if m.ndim != 3:
            raise ValueError("mask must be [nz][ny][nx]")
        self.nz, self.ny, self.nx = m.shape
        self.d = float(d_nm)
        self.m_h = complex(m_h)
        self.device = torch.device("cuda", torch.cuda.current_device())
        self._own_stream = None
        if stream is None:
            self._own_stream = L.dda_stream_create()
            stream = torch.cuda.ExternalStream(self._own_stream, device=self.device)
        self.stream = stream
        opt = L.dda_default_options()
        opt.polarizability = _POL[polarizability]
        opt.precision = _PREC[precision]
        opt.solver = _SOLVER[solver]
        opt.tol = float(tol)
        opt.maxit = int(maxit)
        opt.check_every = int(check_every)
        opt.use_graphs = 1 if use_graphs else 0
        opt.interaction = {"point": L.DDA_INT_POINT, "igt": L.DDA_INT_IGT}[interaction]
        self.ctx = L.dda_setup(m, self.nx, self.ny, self.nz, self.d, self.m_h.real,
                               self.m_h.imag, opt, self.stream.cuda_stream)
        self.n_occ = L.dda_n_occ(self.ctx)
        self.grid = L.dda_grid_dims(self.ctx)

    def close(self) -> None:
        if self.ctx is not None:
            L.dda_destroy(self.ctx)
            self.ctx = None
        if self._own_stream is not None:
            L.dda_stream_destroy(self._own_stream)
            self._own_stream = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @contextlib.contextmanager
    def _ordered(self):
        cur = torch.cuda.current_stream(self.device)
        if cur.cuda_stream != self.stream.cuda_stream:
            self.stream.wait_stream(cur)
        try:
            yield
        finally:
            if cur.cuda_stream != self.stream.cuda_stream:
                cur.wait_stream(self.stream)

    def _eps(self, eps, n_energy: int):
        if isinstance(eps, torch.Tensor) and eps.is_cuda:
            if eps.numel() != n_energy * self.n_occ:
                raise ValueError("eps must hold n_energy x n_occ values")
            return eps.contiguous()
        return np.asarray(eps, dtype=np.complex128).reshape(n_energy, self.n_occ)

    def _field(self, nrhs: int, dtype=torch.complex128) -> torch.Tensor:
        return torch.empty((nrhs, 3, self.n_occ), dtype=dtype, device=self.device)

    def einc(self, energies: Sequence[float], beta: float, r0: np.ndarray,
             out: Optional[torch.Tensor] = None) -> torch.Tensor:
        E = np.atleast_1d(np.asarray(energies, dtype=np.float64))
        R = np.asarray(r0, dtype=np.float64).reshape(-1, 3)
        e = out if out is not None else self._field(E.size * R.shape[0])
        with self._ordered():
            L.dda_einc_electron(self.ctx, E, beta, R, e.data_ptr())
        return e

    def solve(self, energies: Sequence[float], eps: np.ndarray, einc: torch.Tensor,
              n_traj: int, out: Optional[torch.Tensor] = None, raise_on_error: bool = True):
        """eps: complex [n_energy][n_occ] (absolute permittivity per dipole), a
        host array or a contiguous complex128 tensor on the device."""
        E = np.atleast_1d(np.asarray(energies, dtype=np.float64))
        p = out if out is not None else self._field(E.size * n_traj)
        eps = self._eps(eps, E.size)
        with self._ordered():
            st, info = L.dda_solve(self.ctx, E, eps, einc.data_ptr(), n_traj, p.data_ptr(),
                                   raise_on_error=raise_on_error)
        return p, [SolveInfo(*i) for i in info], st

    def losses(self, energies: Sequence[float], beta: float, eps: np.ndarray, r0: np.ndarray,
               einc: torch.Tensor, p: torch.Tensor) -> np.ndarray:
        E = np.atleast_1d(np.asarray(energies, dtype=np.float64))
        eps = self._eps(eps, E.size)
        with self._ordered():
            return L.dda_eels_cl(self.ctx, E, beta, eps, r0, einc.data_ptr(), p.data_ptr())

    def cl_directions(self, energies: Sequence[float], beta: float, n_traj: int,
                      p: torch.Tensor, dirs: np.ndarray, weights: Optional[np.ndarray] = None,
                      want_dp: bool = True):
        """CL per unit solid angle [rhs][n_dir] in 1/(eV sr) for the solution p
        (as solve() returns it), and its weighted sum over the directions."""
        E = np.atleast_1d(np.asarray(energies, dtype=np.float64))
        if p.dtype != torch.complex128 or not p.is_contiguous():
            raise ValueError("p must be a contiguous complex128 tensor")
        with self._ordered():
            return L.dda_cl_directions(self.ctx, E, beta, n_traj, p.data_ptr(), dirs, weights,
                                       want_dp)

    def matvec(self, energy: float, eps: Optional[np.ndarray], x: torch.Tensor,
               precision: str = "fp64", interaction_only: bool = False,
               out: Optional[torch.Tensor] = None) -> torch.Tensor:
        y = out if out is not None else torch.empty_like(x)
        with self._ordered():
            L.dda_matvec(self.ctx, energy, eps, _PREC[precision], interaction_only,
                         x.data_ptr(), y.data_ptr(), x.shape[0])
        return y

    def spectrum(self, energies: Sequence[float], beta: float, eps: np.ndarray, r0: np.ndarray):
        """Electron field -> solve -> losses for every (energy, trajectory).
        Returns (probabilities [n_energy * n_traj][4], solve infos)."""
        R = np.asarray(r0, dtype=np.float64).reshape(-1, 3)
        e = self.einc(energies, beta, R)
        p, info, _ = self.solve(energies, eps, e, R.shape[0])
        return self.losses(energies, beta, eps, R, e, p), info

    def set_timing(self, enabled: bool, kernels=None) -> None:
        L.dda_set_timing(self.ctx, enabled, kernels)

    def kernel_time(self, name: str):
        """(average ms per launch, launches, average right-hand sides per launch)."""
        return L.dda_kernel_time(self.ctx, name)

    def drop_cache(self) -> None:
        L.dda_drop_cache(self.ctx)
