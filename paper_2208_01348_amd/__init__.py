"""MI355X-native DDA solve for fast-electron EELS and cathodoluminescence
(Kichigin & Yurkin, arXiv 2208.01348): C-ABI library libdda (HIP, gfx950)
and its Python binding."""

from . import _lib as lib  # noqa: F401
from ._lib import DDAError, load  # noqa: F401

__all__ = ["lib", "load", "DDAError", "DDASolver"]


def __getattr__(name):
    if name == "DDASolver":  # imports torch lazily
        from .solver import DDASolver
        return DDASolver
    raise AttributeError(name)
