"""The C-ABI library loads and exports every symbol include/dda.h declares
(no compute calls: this runs without a GPU)."""

import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    with open(os.path.join(ROOT, "include", "dda.h")) as f:
        text = f.read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(dda_[A-Za-z0-9_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = _declared()
    for n in ["dda_setup", "dda_einc_electron", "dda_solve", "dda_eels_cl", "dda_destroy",
              "dda_last_error"]:
        assert n in names


def test_library_exports_every_declared_symbol():
    from paper_2208_01348_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        pytest.fail("libdda.so is not built (run __graft_entry__.build())")
    lib = ctypes.CDLL(_lib.LIB_PATH)
    for n in _declared():
        assert hasattr(lib, n), n
    assert sorted(_lib.EXPORTED) == _declared()


def test_binding_fails_loudly_without_library(monkeypatch, tmp_path):
    from paper_2208_01348_amd import _lib
    monkeypatch.setattr(_lib, "_lib", None)
    monkeypatch.setattr(_lib, "LIB_PATH", str(tmp_path / "missing.so"))
    with pytest.raises(RuntimeError):
        _lib.load()


def test_host_only_calls():
    """Calls that touch no device: options and the beta helper (eq. 47 side)."""
    from paper_2208_01348_amd import _lib
    o = _lib.dda_default_options()
    assert o.polarizability == _lib.DDA_POL_LDR and o.tol == 1e-10
    assert abs(_lib.dda_beta_from_keV(100.0) - 0.5482208619) < 1e-9
