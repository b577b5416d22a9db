"""CPU-side checks of the native library: it builds/loads and exports every C-ABI symbol.

No compute call is made here (there is no GPU in this environment)."""

import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "pomm.h")
LIB = os.path.join(ROOT, "paper_1603_09724_amd", "libpomm.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(omm[A-Z]\w*)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        from paper_1603_09724_amd import build
        build.build(verbose=False)
    from paper_1603_09724_amd import pomm
    return pomm.library()


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("ommSetup", "ommApplyH", "ommPrecondition", "ommSolve", "ommDestroy"):
        assert required in names


def test_library_exports_every_declared_symbol(lib):
    missing = [f for f in declared_functions() if not hasattr(lib, f)]
    assert not missing, missing


def test_binding_names_match_header(lib):
    from paper_1603_09724_amd import pomm
    assert sorted(pomm.EXPORTED) == declared_functions()


def test_default_options_are_the_paper_settings(lib):
    from paper_1603_09724_amd import pomm
    o = pomm.default_options()
    assert o.npoles == 30 and o.gmres_restart == 15 and o.gmres_cycles == 5
    assert o.gmres_rtol == 1e-5 and o.maxit == 4000


def _struct_fields(name):
    src = open(os.path.join(ROOT, "include", "pomm.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    body = re.search(r"typedef struct \{([^}]*)\}\s*" + name + ";", src).group(1)
    return [(t, n) for t, n in re.findall(r"\b(int|double|long long)\s+(\w+)\s*;", body)]


@pytest.mark.parametrize("cname,pyname", [("omm_opts_t", "Options"), ("omm_info_t", "Info"),
                                          ("omm_estimate_info_t", "EstimateInfo")])
def test_struct_layouts_match_header(lib, cname, pyname):
    """The ctypes structures list the header's fields in the same order with the same types."""
    import ctypes
    from paper_1603_09724_amd import pomm
    ctype = {"int": ctypes.c_int, "double": ctypes.c_double, "long long": ctypes.c_longlong}
    want = [(n, ctype[t]) for t, n in _struct_fields(cname)]
    assert [(n, t) for n, t in getattr(pomm, pyname)._fields_] == want


def test_default_side_is_automatic(lib):
    from paper_1603_09724_amd import pomm
    assert pomm.default_options().gmres_side == pomm.SIDE_AUTO


def test_status_strings(lib):
    from paper_1603_09724_amd import pomm
    assert lib.ommStatusString(pomm.ENOCONV) == b"iteration cap reached"
    assert lib.ommStatusString(99) == b"unknown status"


def test_oracle_is_not_imported_by_the_package():
    """The product package never imports the oracle."""
    pkg = os.path.join(ROOT, "paper_1603_09724_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith(".py"):
                src = open(os.path.join(dirpath, f)).read()
                assert not re.search(r"^\s*(from|import)\s+oracle\b", src, flags=re.M), f
