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


def _header_trace_width():
    import re
    hdr = os.path.join(os.path.dirname(hode.HERE), "include", "hode.h")
    m = re.search(r"#define\s+HODE_TRACE_W\s+(\d+)", open(hdr).read())
    assert m, "HODE_TRACE_W missing from the header"
    return int(m.group(1))


def test_trace_width_matches_header():
    # a C caller sizes trace buffers from the header's constant: the library
    # (and the binding, which asks the library) must agree with it
    if not os.path.exists(hode.LIBPATH):
        pytest.skip("libhode.so not built")
    w = _header_trace_width()
    assert w == 8 + 16
    assert hode.lib().hode_trace_width() == w
    assert hode.TRACE_W == w
