"""CPU-side checks of the C ABI: the library loads and exports every function
include/jet.h declares; the Python binding names the same set."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "jet.h")
LIB = os.path.join(ROOT, "paper_2304_13194_amd", "libjet.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"\b(jet_[a-z_]+)\s*\(", text)
    return sorted(set(names))


def test_header_declares_the_boundary():
    names = declared_functions()
    for must in ("jet_refine", "jet_coarsen", "jet_partition", "jet_context_create", "jet_strerror"):
        assert must in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="libjet.so not built")
def test_library_exports_every_declared_function():
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_lists_every_declared_function():
    from paper_2304_13194_amd import jet
    assert sorted(jet.EXPORTS) == declared_functions()


@pytest.mark.skipif(not os.path.exists(LIB), reason="libjet.so not built")
def test_strerror_without_gpu():
    lib = ctypes.CDLL(LIB)
    lib.jet_strerror.restype = ctypes.c_char_p
    assert lib.jet_strerror(0) == b"ok"
    assert b"part" in lib.jet_strerror(-3)
