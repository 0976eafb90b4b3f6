"""ctypes binding of libdda (include/dda.h): same names, argument marshalling
only.  Every computation runs in the library's HIP kernels; there is no CPU
fallback, and loading fails loudly when the library has not been built."""

from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libdda.so")

DDA_OK, DDA_EINVAL, DDA_ENOMEM, DDA_EDEVICE, DDA_ENOCONV, DDA_EBREAKDOWN, DDA_ESINGULAR = \
    0, -1, -2, -3, -4, -5, -6
STATUS_NAMES = {0: "DDA_OK", -1: "DDA_EINVAL", -2: "DDA_ENOMEM", -3: "DDA_EDEVICE",
                -4: "DDA_ENOCONV", -5: "DDA_EBREAKDOWN", -6: "DDA_ESINGULAR"}
DDA_POL_LDR, DDA_POL_CM, DDA_POL_RR = 0, 1, 2
DDA_SOLVER_BICGSTAB, DDA_SOLVER_COCG, DDA_SOLVER_QMR = 0, 1, 2
DDA_INT_POINT, DDA_INT_IGT = 0, 1
DDA_PREC_FP64, DDA_PREC_MIXED = 0, 1

# every symbol include/dda.h declares
EXPORTED = ["dda_default_options", "dda_beta_from_keV", "dda_setup", "dda_n_occ",
            "dda_grid_dims", "dda_einc_electron", "dda_einc_electron_noalloc", "dda_solve", "dda_eels_cl", "dda_matvec",
            "dda_set_timing", "dda_kernel_time", "dda_drop_cache", "dda_destroy",
            "dda_last_error", "dda_debug_besselk01", "dda_workspace_bytes", "dda_engine_open",
            "dda_engine_submit", "dda_engine_submit_lattice", "dda_engine_poll", "dda_engine_status", "dda_engine_close",
            "dda_set_host", "dda_stream_create", "dda_stream_destroy", "dda_tuning",
            "dda_set_tuning", "dda_free_space_loss", "dda_cl_total", "dda_psf_gauss",
            "dda_cl_directions", "dda_richardson"]


class DDAError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


class Options(ctypes.Structure):
    _fields_ = [("polarizability", ctypes.c_int), ("solver", ctypes.c_int),
                ("precision", ctypes.c_int), ("tol", ctypes.c_double),
                ("maxit", ctypes.c_int), ("check_every", ctypes.c_int),
                ("use_graphs", ctypes.c_int), ("interaction", ctypes.c_int)]


class SolveInfo(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int), ("matvecs", ctypes.c_int),
                ("rel_residual", ctypes.c_double), ("status", ctypes.c_int)]


class Result(ctypes.Structure):
    _fields_ = [("p_eels", ctypes.c_double), ("p_ext", ctypes.c_double),
                ("p_abs", ctypes.c_double), ("p_cl", ctypes.c_double)]


_lib = None
_vp = ctypes.c_void_p
_i = ctypes.c_int
_d = ctypes.c_double
_i64 = ctypes.c_int64


def load() -> ctypes.CDLL:
    """Loads libdda.so; raises RuntimeError when it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                           "(hipcc for gfx950); there is no fallback path")
    lib = ctypes.CDLL(LIB_PATH)
    sig = {
        "dda_default_options": (None, [_vp]),
        "dda_beta_from_keV": (_d, [_d]),
        "dda_setup": (_i, [_vp, _i, _i, _i, _d, _d, _d, _vp, _vp, _vp]),
        "dda_n_occ": (_i, [_vp, _vp]),
        "dda_grid_dims": (_i, [_vp, _vp, _vp, _vp]),
        "dda_einc_electron": (_i, [_vp, _i, _vp, _d, _vp, _i, _vp]),
        "dda_einc_electron_noalloc": (_i, [_vp, _i, _vp, _d, _vp, _i, _vp]),
        "dda_solve": (_i, [_vp, _i, _vp, _vp, _vp, _i, _vp, _vp]),
        "dda_eels_cl": (_i, [_vp, _i, _vp, _d, _vp, _vp, _i, _vp, _vp, _vp]),
        "dda_matvec": (_i, [_vp, _d, _vp, _i, _i, _vp, _vp, _i]),
        "dda_set_timing": (_i, [_vp, _i]),
        "dda_kernel_time": (_i, [_vp, ctypes.c_char_p, _vp, _vp, _vp]),
        "dda_drop_cache": (_i, [_vp]),
        "dda_destroy": (_i, [_vp]),
        "dda_last_error": (ctypes.c_char_p, []),
        "dda_debug_besselk01": (_i, [_vp, _i64, _vp]),
        "dda_workspace_bytes": (_i, [_vp, _i, _vp]),
        "dda_engine_open": (_i, [_vp, _i]),
        "dda_engine_submit": (_i, [_vp, _i64, _d, _vp, _vp, _vp]),
        "dda_engine_submit_lattice": (_i, [_vp, _vp, _i64, _d, _vp, _vp, _vp]),
        "dda_engine_poll": (_i, [_vp, _i, _vp, _vp, _i, _vp]),
        "dda_engine_status": (_i, [_vp, _vp, _vp, _vp]),
        "dda_engine_close": (_i, [_vp]),
        "dda_set_host": (_i, [_vp, _d, _d]),
        "dda_stream_create": (_i, [_vp]),
        "dda_stream_destroy": (_i, [_vp]),
        "dda_tuning": (_i, [_vp, _i, _vp, _vp, _vp, _vp, _vp]),
        "dda_set_tuning": (_i, [_vp, _i, _i, _i, _i]),
        "dda_free_space_loss": (_i, [_d, _d, _d, _vp]),
        "dda_cl_total": (_i, [_vp, _i, _d, _vp]),
        "dda_psf_gauss": (_i, [_vp, _vp, _i, _d, _vp]),
        "dda_cl_directions": (_i, [_vp, _i, _vp, _d, _i, _vp, _i, _vp, _vp, _vp, _vp]),
        "dda_richardson": (_i, [_vp, _vp, _i, _vp, _vp]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


def _check(st: int) -> int:
    if st != DDA_OK:
        raise DDAError(st, load().dda_last_error().decode())
    return st


def _ptr(a: np.ndarray) -> int:
    return a.ctypes.data


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


def _eps_pairs(eps) -> np.ndarray:
    e = np.ascontiguousarray(np.asarray(eps, dtype=np.complex128))
    return e.view(np.float64)


def _eps_ptr(eps):
    """(pointer, keep-alive) for a permittivity array: a contiguous complex128
    device tensor is passed in place; anything else becomes a host array."""
    if getattr(eps, "is_cuda", False):
        if str(eps.dtype) != "torch.complex128" or not eps.is_contiguous():
            raise ValueError("device permittivities must be contiguous complex128")
        return eps.data_ptr(), eps
    e = _eps_pairs(eps)
    return _ptr(e), e


def dda_default_options() -> Options:
    o = Options()
    load().dda_default_options(ctypes.byref(o))
    return o


def dda_beta_from_keV(kinetic_keV: float) -> float:
    return float(load().dda_beta_from_keV(float(kinetic_keV)))


def dda_free_space_loss(beta: float, m_h: complex) -> float:
    """d Gamma_0 / dz in eV^-1 nm^-1 (host closed form)."""
    out = ctypes.c_double()
    _check(load().dda_free_space_loss(float(beta), float(m_h.real), float(m_h.imag),
                                      ctypes.byref(out)))
    return out.value


def dda_cl_total(P: np.ndarray, m_h: complex) -> np.ndarray:
    """P_CL^tot from rows (P_EELS, P_ext, P_abs, P_CL) (host closed form)."""
    rows = np.ascontiguousarray(np.asarray(P, dtype=np.float64).reshape(-1, 4))
    out = np.empty(rows.shape[0])
    _check(load().dda_cl_total(_ptr(rows), rows.shape[0], float(complex(m_h).imag), _ptr(out)))
    return out


def dda_psf_gauss(energy_eV, p, fwhm_eV: float) -> np.ndarray:
    """Spectrum convolved with a unit-area Gaussian of the given FWHM (host)."""
    E = _f64(energy_eV)
    v = _f64(p)
    if E.shape != v.shape or E.ndim != 1:
        raise ValueError("energies and spectrum must be 1-D of one length")
    out = np.empty_like(v)
    _check(load().dda_psf_gauss(_ptr(E), _ptr(v), E.size, float(fwhm_eV), _ptr(out)))
    return out


def dda_richardson(d_nm, values):
    """(extrapolated value at d = 0, 95 % half-width) of one quantity."""
    d = _f64(d_nm).reshape(-1)
    v = _f64(values).reshape(-1)
    if d.shape != v.shape:
        raise ValueError("one value per dipole size")
    a = ctypes.c_double()
    ci = ctypes.c_double()
    _check(load().dda_richardson(_ptr(d), _ptr(v), d.size, ctypes.byref(a), ctypes.byref(ci)))
    return a.value, ci.value


def dda_cl_directions(ctx, energies, beta: float, n_traj: int, p_ptr: int, dirs, weights=None,
                      want_dp: bool = True):
    """(dP/dOmega [rhs][n_dir] or None, P_CL over the weights [rhs] or None)."""
    E = _f64(energies).reshape(-1)
    D = _f64(dirs).reshape(-1, 3)
    nrhs = E.size * n_traj
    dp = np.empty((nrhs, D.shape[0])) if want_dp else None
    w = None if weights is None else _f64(weights).reshape(-1)
    pcl = np.empty(nrhs) if w is not None else None
    _check(load().dda_cl_directions(ctx, E.size, _ptr(E), float(beta), n_traj,
                                    ctypes.c_void_p(p_ptr), D.shape[0], _ptr(D),
                                    None if w is None else _ptr(w),
                                    None if dp is None else _ptr(dp),
                                    None if pcl is None else _ptr(pcl)))
    return dp, pcl


def dda_setup(mask: np.ndarray, nx: int, ny: int, nz: int, d_nm: float, mh_re: float,
              mh_im: float, opt: Options, hip_stream: int = 0) -> ctypes.c_void_p:
    m = np.ascontiguousarray(np.asarray(mask, dtype=np.uint8))
    if m.size != nx * ny * nz:
        raise ValueError("mask size does not match nx*ny*nz")
    ctx = ctypes.c_void_p()
    _check(load().dda_setup(_ptr(m), nx, ny, nz, float(d_nm), float(mh_re), float(mh_im),
                            ctypes.byref(opt), ctypes.c_void_p(hip_stream or None),
                            ctypes.byref(ctx)))
    return ctx


def dda_tuning(ctx, precision: int):
    """Autotuned tiles of one precision's matvec chain, or None before tuning:
    {zconv_tx, mid_tx, yz_threads, t_default_ms, t_best_ms}."""
    a, b, c = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
    t0, t1 = ctypes.c_double(), ctypes.c_double()
    st = load().dda_tuning(ctx, int(precision), ctypes.byref(a), ctypes.byref(b), ctypes.byref(c),
                           ctypes.byref(t0), ctypes.byref(t1))
    if st == 1:
        return None
    _check(st)
    return {"zconv_tx": a.value, "mid_tx": b.value, "yz_threads": c.value,
            "t_default_ms": round(t0.value, 5), "t_best_ms": round(t1.value, 5)}


def dda_set_tuning(ctx, precision: int, zconv_tx: int = 0, mid_tx: int = 0,
                   yz_threads: int = 0) -> None:
    _check(load().dda_set_tuning(ctx, int(precision), int(zconv_tx), int(mid_tx),
                                 int(yz_threads)))


def dda_stream_create() -> int:
    s = ctypes.c_void_p()
    _check(load().dda_stream_create(ctypes.byref(s)))
    return int(s.value)


def dda_stream_destroy(stream: int) -> None:
    _check(load().dda_stream_destroy(ctypes.c_void_p(stream)))


def dda_set_host(ctx, mh_re: float, mh_im: float) -> None:
    _check(load().dda_set_host(ctx, float(mh_re), float(mh_im)))


def dda_n_occ(ctx) -> int:
    n = ctypes.c_int64()
    _check(load().dda_n_occ(ctx, ctypes.byref(n)))
    return int(n.value)


def dda_grid_dims(ctx):
    a, b, c = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
    _check(load().dda_grid_dims(ctx, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c)))
    return a.value, b.value, c.value


def dda_einc_electron(ctx, energy_eV, beta: float, r0_nm, einc_dev: int) -> None:
    E = _f64(energy_eV).ravel()
    R = _f64(r0_nm).reshape(-1, 3)
    _check(load().dda_einc_electron(ctx, E.size, _ptr(E), float(beta), _ptr(R), R.shape[0],
                                    ctypes.c_void_p(einc_dev)))


DDA_EINC_NOALLOC_MAX_ENERGIES = 4096
DDA_EINC_NOALLOC_MAX_TRAJ = 4096


def dda_einc_electron_noalloc(ctx, energy_eV, beta: float, r0_nm, einc_dev: int) -> None:
    E = _f64(energy_eV).ravel()
    R = _f64(r0_nm).reshape(-1, 3)
    _check(load().dda_einc_electron_noalloc(ctx, E.size, _ptr(E), float(beta), _ptr(R),
                                            R.shape[0], ctypes.c_void_p(einc_dev)))


def dda_solve(ctx, energy_eV, eps_dipole, einc_dev: int, n_traj: int, p_dev: int,
              raise_on_error: bool = True):
    """eps_dipole: complex [n_energy][n_occ].  Returns (status, info array)."""
    E = _f64(energy_eV).ravel()
    eps, keep = _eps_ptr(eps_dipole)
    info = (SolveInfo * max(1, E.size * n_traj))()
    st = load().dda_solve(ctx, E.size, _ptr(E), ctypes.c_void_p(eps), ctypes.c_void_p(einc_dev),
                          n_traj, ctypes.c_void_p(p_dev), info)
    if raise_on_error and st not in (DDA_OK,):
        _check(st)
    return st, [(i.iters, i.matvecs, i.rel_residual, i.status) for i in info[:E.size * n_traj]]


def dda_eels_cl(ctx, energy_eV, beta: float, eps_dipole, r0_nm, einc_dev: int,
                p_dev: int) -> np.ndarray:
    """Returns float64 [n_energy * n_traj][4]: P_EELS, P_ext, P_abs, P_CL (1/eV)."""
    E = _f64(energy_eV).ravel()
    R = _f64(r0_nm).reshape(-1, 3)
    eps, keep = _eps_ptr(eps_dipole)
    out = np.zeros((E.size * R.shape[0], 4), dtype=np.float64)
    _check(load().dda_eels_cl(ctx, E.size, _ptr(E), float(beta), ctypes.c_void_p(eps), _ptr(R),
                              R.shape[0], ctypes.c_void_p(einc_dev), ctypes.c_void_p(p_dev),
                              _ptr(out)))
    return out


def dda_matvec(ctx, energy_eV: float, eps_dipole, precision: int, interaction_only: bool,
               x_dev: int, y_dev: int, nrhs: int) -> None:
    eps = _eps_pairs(eps_dipole) if eps_dipole is not None else None
    _check(load().dda_matvec(ctx, float(energy_eV), None if eps is None else _ptr(eps),
                             int(precision), int(bool(interaction_only)), ctypes.c_void_p(x_dev),
                             ctypes.c_void_p(y_dev), int(nrhs)))


KERNEL_NAMES = ["unpack_xfft", "yfft", "zconv", "iyfft", "ixfft_pack", "yzconv", "xyfft",
                "ixyfft_pack"]


def dda_set_timing(ctx, enabled, kernels=None) -> None:
    """enabled: False/True; kernels: optional list of names to time."""
    if not enabled:
        v = 0
    elif kernels is None:
        v = 1
    else:
        v = sum(1 << KERNEL_NAMES.index(k) for k in kernels)
        v = v if v != 1 else (1 << 5) | 1  # bit 0 alone must not read as "all"
    _check(load().dda_set_timing(ctx, int(v)))


def dda_kernel_time(ctx, name: str):
    """(average ms per launch, launches, average right-hand sides per launch)."""
    ms = ctypes.c_double()
    n = ctypes.c_int64()
    u = ctypes.c_double()
    _check(load().dda_kernel_time(ctx, name.encode(), ctypes.byref(ms), ctypes.byref(n),
                                  ctypes.byref(u)))
    return float(ms.value), int(n.value), float(u.value)


def dda_workspace_bytes(ctx, n_slots: int) -> int:
    b = ctypes.c_size_t()
    _check(load().dda_workspace_bytes(ctx, int(n_slots), ctypes.byref(b)))
    return int(b.value)


def dda_engine_open(ctx, max_slots: int) -> None:
    _check(load().dda_engine_open(ctx, int(max_slots)))


def dda_engine_submit(ctx, tag: int, energy_eV: float, eps_dipole, einc_dev: int,
                      p_dev: int) -> None:
    """eps_dipole: complex [n_occ] for this energy."""
    eps = _eps_pairs(eps_dipole)
    _check(load().dda_engine_submit(ctx, int(tag), float(energy_eV), _ptr(eps),
                                    ctypes.c_void_p(einc_dev), ctypes.c_void_p(p_dev)))


def dda_engine_submit_lattice(ctx, lat, tag: int, energy_eV: float, eps_dipole, einc_dev: int,
                              p_dev: int) -> None:
    """A system of lattice context `lat` (same box) in ctx's engine;
    eps_dipole: complex [n_occ(lat)]."""
    eps = _eps_pairs(eps_dipole)
    _check(load().dda_engine_submit_lattice(ctx, lat, int(tag), float(energy_eV), _ptr(eps),
                                            ctypes.c_void_p(einc_dev), ctypes.c_void_p(p_dev)))


def dda_engine_poll(ctx, max_intervals: int, capacity: int = 256):
    """Returns [(tag, (iters, matvecs, rel_residual, status)), ...] of finished systems."""
    tags = (ctypes.c_int64 * max(1, capacity))()
    info = (SolveInfo * max(1, capacity))()
    n = ctypes.c_int()
    _check(load().dda_engine_poll(ctx, int(max_intervals), tags, info, int(capacity),
                                  ctypes.byref(n)))
    return [(int(tags[k]), (info[k].iters, info[k].matvecs, info[k].rel_residual,
                            info[k].status)) for k in range(n.value)]


def dda_engine_status(ctx):
    """(queued, running, finished-not-returned)."""
    q, r, f = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
    _check(load().dda_engine_status(ctx, ctypes.byref(q), ctypes.byref(r), ctypes.byref(f)))
    return q.value, r.value, f.value


def dda_engine_close(ctx) -> None:
    _check(load().dda_engine_close(ctx))


def dda_drop_cache(ctx) -> None:
    _check(load().dda_drop_cache(ctx))


def dda_destroy(ctx) -> None:
    _check(load().dda_destroy(ctx))


def dda_last_error() -> str:
    return load().dda_last_error().decode()


def dda_debug_besselk01(z) -> np.ndarray:
    zz = np.ascontiguousarray(np.asarray(z, dtype=np.complex128).ravel())
    out = np.zeros((zz.size, 4), dtype=np.float64)
    _check(load().dda_debug_besselk01(_ptr(zz.view(np.float64)), zz.size, _ptr(out)))
    return out[:, 0] + 1j * out[:, 1], out[:, 2] + 1j * out[:, 3]
