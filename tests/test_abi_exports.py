"""The C-ABI library loads on the CPU host and exports every entry point that
include/msfv.h declares (no compute calls: those need a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "msfv.h")
LIB = os.path.join(ROOT, "paper_1707_07598_amd", "libmsfv.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(msfv_[a-z_]+)\s*\(", text)))


def test_header_declares_the_path():
    names = declared_functions()
    for required in ["msfv_create", "msfv_destroy", "msfv_set_sources", "msfv_set_receivers",
                     "msfv_forward", "msfv_jtv", "msfv_misfit_grad", "msfv_sync"]:
        assert required in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="libmsfv.so not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    for name in declared_functions():
        assert hasattr(lib, name), name


@pytest.mark.skipif(not os.path.exists(LIB), reason="libmsfv.so not built")
def test_binding_covers_every_declared_symbol():
    from paper_1707_07598_amd import _lib
    assert set(declared_functions()) == set(_lib.SIGNATURES)
    lib = _lib.load()
    assert lib.msfv_status_string(_lib.MSFV_ENOCONV) == b"iteration cap reached"


def test_missing_library_fails_loudly(tmp_path):
    from paper_1707_07598_amd import _lib
    saved = _lib._lib
    _lib._lib = None
    try:
        with pytest.raises(ImportError):
            _lib.load(str(tmp_path / "nope.so"))
    finally:
        _lib._lib = saved
