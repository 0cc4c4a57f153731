"""The C-ABI library loads and exports every symbol the header declares
(no compute calls: this runs without a GPU)."""
import ctypes
import os

import pytest

from paper_2309_05331_amd import hode


def test_header_symbols_exported():
    if not os.path.exists(hode.LIBPATH):
        pytest.skip("libhode.so not built")
    L = ctypes.CDLL(hode.LIBPATH)
    names = hode.exported_symbols()
    assert "hode_integrate_adaptive" in names and len(names) >= 20
    missing = [n for n in names if not hasattr(L, n)]
    assert not missing, missing


def test_binding_signatures_cover_header():
    if not os.path.exists(hode.LIBPATH):
        pytest.skip("libhode.so not built")
    L = hode.lib()
    for n in hode.exported_symbols():
        assert getattr(L, n).argtypes is not None, n


def test_missing_library_fails_loudly(monkeypatch, tmp_path):
    monkeypatch.setattr(hode, "_lib", None)
    monkeypatch.setattr(hode, "LIBPATH", str(tmp_path / "absent.so"))
    with pytest.raises(RuntimeError, match="not built"):
        hode.lib()
