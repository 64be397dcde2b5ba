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


def test_cube_grid_sizes_checked_before_any_table():
    """ibm_bcm_create rejects, before building any table or touching a device, grids
    whose fine-cell origins or 32-bit storage and halo indices would overflow; the cube
    count used for that includes the refined cubes (8 per refined coarse cube)."""
    import numpy as np
    from paper_2002_06206_amd import build
    if not os.path.exists(build.LIB):
        build.build()
    lib = ctypes.CDLL(build.LIB)
    lib.ibm_last_error.restype = ctypes.c_char_p

    def create(K, n, refine_all):
        ref = np.full(int(np.prod(K)), 1 if refine_all else 0, dtype=np.uint8)
        out = ctypes.c_void_p()
        rc = lib.ibm_bcm_create((ctypes.c_int32 * 3)(*K), ctypes.c_int32(n), ctypes.c_double(1.0),
                                (ctypes.c_double * 3)(0.0, 0.0, 0.0), ref.ctypes.data_as(ctypes.c_void_p),
                                ctypes.byref(out))
        if rc == 0:
            lib.ibm_bcm_destroy(out)
        return rc, (lib.ibm_last_error() or b"").decode()

    rc, msg = create((1 << 20, 1, 1), 1024, False)
    assert rc == -1 and "2^31 fine cells" in msg
    rc, msg = create((100, 100, 100), 16, False)
    assert rc == -1 and "storage" in msg
    rc, msg = create((64, 32, 32), 16, True)       # 65,536 coarse cubes, all refined: 4.2e9 values
    assert rc == -1 and "exceed 2^31" in msg
    rc, msg = create((2, 2, 2), 16, True)          # small: passes the size checks
    assert rc in (0, -2), (rc, msg)
