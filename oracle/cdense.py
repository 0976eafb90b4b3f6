"""ctypes loader for the oracle's plain-C dense matvec (dense_matvec.c).

The shared object is built with gcc (-O2 -fopenmp) into this directory by
`build()`; `load()` builds it on first use when it is missing or older than
its source.
"""

from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "dense_matvec.c")
_LIB = os.path.join(_HERE, "liboracle_dense.so")
_lib = None


def build() -> str:
    """Compile dense_matvec.c with gcc; returns the path of the shared object."""
    tmp = _LIB + ".tmp"
    subprocess.run(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11", _SRC,
                    "-lm", "-o", tmp], check=True)
    os.replace(tmp, _LIB)
    return _LIB


def load():
    global _lib
    if _lib is not None:
        return _lib
    if (not os.path.exists(_LIB)) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        build()
    lib = ctypes.CDLL(_LIB)
    lib.oracle_dense_matvec.argtypes = [
        ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_double, ctypes.c_double,
        ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int]
    lib.oracle_dense_matvec.restype = None
    lib.oracle_num_threads.restype = ctypes.c_int
    lib.oracle_dense_matvec_rows.argtypes = [
        ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_double, ctypes.c_double,
        ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p, ctypes.c_int]
    lib.oracle_dense_matvec_rows.restype = None
    _lib = lib
    return lib


def num_threads() -> int:
    return int(load().oracle_num_threads())


def matvec(centres: np.ndarray, alpha: np.ndarray, k: complex, x: np.ndarray,
           interaction_only: bool = False) -> np.ndarray:
    """y = A x (or y = G_off x) for x of shape [n][3] complex128."""
    lib = load()
    c = np.ascontiguousarray(centres, dtype=np.float64)
    n = c.shape[0]
    xx = np.ascontiguousarray(x, dtype=np.complex128).reshape(n, 3)
    if interaction_only:
        ai = np.zeros(n, dtype=np.complex128)
    else:
        ai = np.ascontiguousarray(1.0 / np.asarray(alpha, dtype=np.complex128))
    y = np.empty((n, 3), dtype=np.complex128)
    lib.oracle_dense_matvec(n, c.ctypes.data, ai.ctypes.data, float(np.real(k)),
                            float(np.imag(k)), xx.ctypes.data, y.ctypes.data,
                            1 if interaction_only else 0)
    return y


def matvec_rows(centres: np.ndarray, alpha: np.ndarray, k: complex, x: np.ndarray,
                rows: np.ndarray, interaction_only: bool = False) -> np.ndarray:
    """Rows `rows` of A x (or of G_off x); returns [len(rows)][3] complex128."""
    lib = load()
    c = np.ascontiguousarray(centres, dtype=np.float64)
    n = c.shape[0]
    xx = np.ascontiguousarray(x, dtype=np.complex128).reshape(n, 3)
    rr = np.ascontiguousarray(rows, dtype=np.int64)
    if interaction_only:
        ai = np.zeros(n, dtype=np.complex128)
    else:
        ai = np.ascontiguousarray(1.0 / np.asarray(alpha, dtype=np.complex128))
    y = np.empty((rr.size, 3), dtype=np.complex128)
    lib.oracle_dense_matvec_rows(n, c.ctypes.data, ai.ctypes.data, float(np.real(k)),
                                 float(np.imag(k)), xx.ctypes.data, rr.ctypes.data, rr.size,
                                 y.ctypes.data, 1 if interaction_only else 0)
    return y
