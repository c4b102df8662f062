"""CPU-side checks of the C ABI boundary (no GPU compute).

* libutri.so loads and exports every function include/utri.h declares;
* argument checks that return before any device work give their documented codes;
* the product path (package sources) never imports or links the oracle, and the
  binding fails loudly when the library is missing.
"""
import ctypes as C
import os
import re

import pytest

from paper_2602_14084_amd import utri

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "utri.h")
PKG = os.path.join(ROOT, "paper_2602_14084_amd")


@pytest.fixture(scope="module")
def L():
    if not os.path.exists(utri.LIB_PATH):
        from paper_2602_14084_amd import build
        build.build()
    return utri.lib()


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(utri_[a-z_0-9]+)\s*\(", text)))


def test_header_declares_the_abi():
    names = declared_functions()
    assert set(names) == set(utri.ABI_FUNCTIONS)


def test_library_exports_every_declared_symbol(L):
    for name in declared_functions():
        assert hasattr(L, name), name


def test_strerror(L):
    for code in [0, -1, -2, -3, -4, -5, -6, 17]:
        s = utri.utri_strerror(code)
        assert isinstance(s, str) and s


def test_host_side_argument_checks(L):
    vp = C.c_void_p
    out = vp()
    # NULL output handle, negative sizes, bad pointer kind, NULL inputs with m_in > 0
    assert L.utri_graph_load(None, None, None, 0, 10, 0, None, None) == utri.UTRI_E_INVALID
    assert L.utri_graph_load(None, None, None, -1, 10, 0, None, C.byref(out)) == utri.UTRI_E_INVALID
    assert L.utri_graph_load(None, None, None, 0, -1, 0, None, C.byref(out)) == utri.UTRI_E_INVALID
    assert L.utri_graph_load(None, None, None, 0, 10, 7, None, C.byref(out)) == utri.UTRI_E_INVALID
    assert L.utri_graph_load(None, None, None, 5, 10, 0, None, C.byref(out)) == utri.UTRI_E_INVALID
    assert L.utri_graph_load(None, None, None, 0, 1 << 31, 0, None, C.byref(out)) == utri.UTRI_E_RANGE
    # NULL handle everywhere
    res = (C.c_int64 * 2)()
    E = C.c_double()
    assert L.utri_count(None, 0.6, 1, 3, res, None) == utri.UTRI_E_INVALID
    assert L.utri_expected(None, C.byref(E), None) == utri.UTRI_E_INVALID
    assert L.utri_graph_info(None, None, None, None, None, None) == utri.UTRI_E_INVALID
    assert L.utri_graph_free(None) == utri.UTRI_OK


def test_product_path_never_touches_the_oracle():
    for dirpath, _, files in os.walk(PKG):
        for f in files:
            if f.endswith((".py", ".hip", ".h", ".cpp")):
                text = open(os.path.join(dirpath, f)).read()
                assert not re.search(r"^\s*(import|from)\s+oracle\b", text, re.M), f
                assert "liboracle" not in text, f
                assert "oracle.c" not in text, f


def test_binding_fails_loudly_without_library(monkeypatch, tmp_path):
    monkeypatch.setattr(utri, "_lib", None)
    monkeypatch.setattr(utri, "LIB_PATH", str(tmp_path / "missing.so"))
    with pytest.raises(RuntimeError):
        utri.lib()
