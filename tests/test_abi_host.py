"""Host-side checks of the C-ABI library: it loads, exports every function the
header declares, and rejects bad arguments before touching a device."""

import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mrhs.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(mrhs_[a-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    from paper_2211_13719_amd import _lib

    return _lib.lib


def test_header_declares_functions():
    names = declared_functions()
    assert "mrhs_dwc_apply" in names and "mrhs_create" in names


def test_every_declared_symbol_exported(lib):
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_covers_header():
    from paper_2211_13719_amd import _lib

    assert sorted(_lib.SIGNATURES) == declared_functions()


def test_create_rejects_bad_shapes(lib):
    h = C.c_void_p()
    dims = (C.c_int32 * 4)(8, 8, 1, 8)
    assert lib.mrhs_create(C.byref(h), dims, -1, 0, None) == 2  # SHAPE
    assert b"below 2" in lib.mrhs_last_error(None)
    dims = (C.c_int32 * 4)(8, 8, 8, 8)
    assert lib.mrhs_create(C.byref(h), dims, 0, 0, None) == 1  # INVALID_ARG: t_bc
    assert b"t_bc" in lib.mrhs_last_error(None)
    dims = (C.c_int32 * 4)(512, 512, 512, 512)
    assert lib.mrhs_create(C.byref(h), dims, -1, 0, None) == 2
    assert lib.mrhs_create(None, dims, -1, 0, None) == 1


def test_null_context_rejected(lib):
    assert lib.mrhs_dwc_apply(None, None, None, 1, 1) == 1
    assert lib.mrhs_set_gauge(None, None, 0, 0) == 1
    assert lib.mrhs_build_clover(None, 1.0, 0.1) == 1
    assert lib.mrhs_last_error(None) is not None
