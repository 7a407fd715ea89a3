"""The C-ABI library loads on the CPU and exports every symbol include/hfci.h declares."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "hfci.h")
LIB = os.path.join(ROOT, "paper_1811_12378_amd", "libhfci.so")


def declared():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(hfci_[a-z0-9_]+)\s*\(", txt)))


def test_header_declares_the_binding_surface():
    from paper_1811_12378_amd.hfci import EXPORTED
    assert sorted(EXPORTED) == declared()


@pytest.mark.skipif(not os.path.exists(LIB), reason="libhfci.so not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    for name in declared():
        assert hasattr(lib, name), name
    lib.hfci_version.restype = ctypes.c_char_p
    assert b"gfx950" in lib.hfci_version()


@pytest.mark.skipif(not os.path.exists(LIB), reason="libhfci.so not built")
def test_default_opts_without_gpu():
    from paper_1811_12378_amd import hfci
    o = hfci.default_opts()
    assert o.size == ctypes.sizeof(hfci.SolveOpts)
    assert (o.precision, o.restart, o.fp_reduce, o.precond) == (64, 30, 5.0, 1)
