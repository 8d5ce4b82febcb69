"""Host-side checks of the C ABI (no GPU needed): the built library loads and
exports every entry point that include/xtrg.h declares, and the binding
declares the same set."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_1801_00142_amd", "libxtrg.so")
HDR = os.path.join(ROOT, "include", "xtrg.h")


def declared():
    text = open(HDR).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(xtrg_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_entry_points():
    names = declared()
    for n in ("xtrg_init_rho", "xtrg_square_compress", "xtrg_observables", "xtrg_hamiltonian_xxz"):
        assert n in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    for n in declared():
        assert hasattr(lib, n), n


def test_binding_covers_header():
    from paper_1801_00142_amd.xtrg import exported_symbols
    assert sorted(exported_symbols()) == declared()


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_missing_library_fails_loudly(tmp_path):
    from paper_1801_00142_amd import xtrg as X
    with pytest.raises(X.XtrgError):
        X.load_library(str(tmp_path / "nope.so"))
