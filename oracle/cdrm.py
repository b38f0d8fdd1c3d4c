"""Build and load oracle/cdrm.c, the plain-C evaluation of the oracle's DRM entries
(test infrastructure).  It computes the definition of oracle.drm.gaussian by the same
operations in the same order, roughly a hundred times faster than the NumPy code,
and is pinned to it bit for bit (tests/test_oracle_drm.py).  Nothing in the product
links it; gcc builds it in place as oracle/_cdrm.so."""
import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "cdrm.c")
LIB = os.path.join(HERE, "_cdrm.so")


def build():
    """Compile cdrm.c (no FMA contraction, no fast-math) into _cdrm.so."""
    tmp = LIB + ".tmp"
    cmd = ["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-shared", "-fPIC", SRC, "-o", tmp, "-lm"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"oracle C build failed: {' '.join(cmd)}\n{r.stderr}")
    os.replace(tmp, LIB)
    return LIB


_lib = None


def lib():
    """The loaded library, or None when it has not been built."""
    global _lib
    if _lib is None and os.path.exists(LIB):
        L = C.CDLL(LIB)
        L.oracle_gaussian.argtypes = [C.c_uint64, C.c_uint32, C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p]
        L.oracle_gaussian.restype = None
        L.oracle_drm_rows.argtypes = [C.c_uint64, C.c_uint32, C.c_int64, C.c_int64, C.c_int64, C.c_void_p]
        L.oracle_drm_rows.restype = None
        _lib = L
    return _lib


def gaussian(seed, tag, rows, cols):
    """G for flat index arrays (rows uint64, cols uint32, equal length) -> float64."""
    rows = np.ascontiguousarray(rows, dtype=np.uint64)
    cols = np.ascontiguousarray(cols, dtype=np.uint32)
    out = np.empty(rows.shape, dtype=np.float64)
    lib().oracle_gaussian(C.c_uint64(int(seed)), C.c_uint32(int(tag)), rows.ctypes.data, cols.ctypes.data,
                          rows.size, out.ctypes.data)
    return out


def drm_rows(seed, tag, row0, nrows, ncols):
    out = np.empty((nrows, ncols), dtype=np.float64)
    lib().oracle_drm_rows(C.c_uint64(int(seed)), C.c_uint32(int(tag)), int(row0), int(nrows), int(ncols),
                          out.ctypes.data)
    return out
