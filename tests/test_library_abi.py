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


def _header_struct(name):
    """(type, field) pairs of the typedef struct `name` in include/xtrg.h."""
    text = re.sub(r"/\*.*?\*/", "", open(HDR).read(), flags=re.S)
    m = re.search(r"typedef struct\s*\{([^{}]*)\}\s*" + name + r"\s*;", text)
    assert m, name
    out = []
    for decl in m.group(1).split(";"):
        decl = " ".join(decl.split())
        if not decl:
            continue
        typ, names = re.match(r"((?:const )?\w+\s*\**)\s*(.*)", decl).groups()
        for nm in names.split(","):
            nm = nm.strip()
            stars = len(nm) - len(nm.lstrip("*"))
            out.append((typ.replace(" ", "") + "*" * stars, nm.lstrip("*")))
    return out


@pytest.mark.parametrize("cname,pyname", [("xtrg_compress_opts", "CompressOpts"),
                                          ("xtrg_compress_info", "CompressInfo"), ("xtrg_obs", "Obs")])
def test_binding_structs_match_header(cname, pyname):
    """The ctypes structures of the binding have the header's fields in the
    header's order with matching C types (a field added on one side only
    would shift every later field across the ABI)."""
    import ctypes as C
    from paper_1801_00142_amd import xtrg as X
    ctype = {"int": C.c_int, "double": C.c_double, "double*": C.POINTER(C.c_double)}
    fields = getattr(X, pyname)._fields_
    hdr = _header_struct(cname)
    assert [n for n, _ in fields] == [n for _, n in hdr]
    for (n, t), (ht, _) in zip(fields, hdr):
        assert t == ctype[ht], (cname, n, ht)
