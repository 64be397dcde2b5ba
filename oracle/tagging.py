"""ctypes wrapper around the exact-predicate tagging oracle (tag_exact.c).

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "tag_exact.c")
_LIB = os.path.join(_HERE, "liboracle_tag.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile tag_exact.c with gcc (-O2 -ffp-contract=off)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        cmd = ["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-std=c11", "-fPIC", "-shared",
               "-o", _LIB + ".tmp", _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(_LIB + ".tmp", _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        lib = ctypes.CDLL(_LIB)
        dp = ctypes.POINTER(ctypes.c_double)
        lib.oracle_tag.argtypes = [dp, ctypes.c_int64, ctypes.POINTER(ctypes.c_int32), ctypes.c_double,
                                   dp, ctypes.c_double, ctypes.POINTER(ctypes.c_uint8), dp]
        lib.oracle_tag.restype = ctypes.c_int
        lib.oracle_orient2d_sign.argtypes = [ctypes.c_double] * 6
        lib.oracle_orient2d_sign.restype = ctypes.c_int
        lib.oracle_crossing_sign.argtypes = [ctypes.c_double] * 3 + [dp, dp, dp, ctypes.c_int]
        lib.oracle_crossing_sign.restype = ctypes.c_int
        _lib = lib
    return _lib


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def tag(tri: np.ndarray, n, dx: float, origin, bary_eps: float = 0.0):
    """Returns (blocked uint8 (nz,ny,nx), theta float64 (nz,ny,nx,6)).  bary_eps: the
    ray test's tolerance in barycentric terms (0 = exact)."""
    if not (0.0 <= bary_eps <= 0.5):
        raise ValueError("bary_eps must lie in [0, 0.5]")
    lib = _load()
    tri = np.ascontiguousarray(tri, dtype=np.float64)
    nn = np.asarray(n, dtype=np.int32)
    org = np.ascontiguousarray(origin, dtype=np.float64)
    ncell = int(nn[0]) * int(nn[1]) * int(nn[2])
    blocked = np.zeros(ncell, dtype=np.uint8)
    theta = np.zeros(ncell * 6, dtype=np.float64)
    rc = lib.oracle_tag(_dp(tri), len(tri), nn.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), float(dx),
                        _dp(org), float(bary_eps), blocked.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)),
                        _dp(theta))
    if rc != 0:
        raise ValueError("oracle_tag: non-finite coordinate")
    shape = (int(nn[2]), int(nn[1]), int(nn[0]))
    return blocked.reshape(shape), theta.reshape(shape + (6,))


def orient2d_sign(pu, pv, au, av, bu, bv) -> int:
    return _load().oracle_orient2d_sign(pu, pv, au, av, bu, bv)


def crossing_sign(pu, pv, t, A, B, C, k) -> int:
    A = np.ascontiguousarray(A, dtype=np.float64)
    B = np.ascontiguousarray(B, dtype=np.float64)
    C = np.ascontiguousarray(C, dtype=np.float64)
    return _load().oracle_crossing_sign(pu, pv, t, _dp(A), _dp(B), _dp(C), int(k))
