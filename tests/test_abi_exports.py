"""The C-ABI library loads on the CPU and exports every entry point include/ibm.h declares."""
import ctypes
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    src = open(os.path.join(ROOT, "include", "ibm.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(ibm_[a-z0-9_]+)\s*\(", src)))


def test_header_declares_the_five_method_calls():
    names = declared_symbols()
    for n in ("ibm_tag_geometry", "ibm_build_stencils", "ibm_step", "ibm_poisson_solve", "ibm_forces"):
        assert n in names


def test_library_exports_every_declared_symbol():
    from paper_2002_06206_amd import build
    if not os.path.exists(build.LIB):
        build.build()
    lib = ctypes.CDLL(build.LIB)
    missing = [n for n in declared_symbols() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_names_match_the_header():
    from paper_2002_06206_amd import ibm
    assert sorted(ibm.EXPORTED) == declared_symbols()
