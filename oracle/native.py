"""Build and call the C direct-sum oracle (``naive.c``) -- TEST INFRASTRUCTURE ONLY."""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "naive.c")
_LIB = os.path.join(_HERE, "liboracle_naive.so")
_lib = None


def build(force=True):
    """Compile naive.c with gcc + OpenMP into oracle/liboracle_naive.so."""
    if not force and os.path.exists(_LIB) and os.path.getmtime(_LIB) >= os.path.getmtime(_SRC):
        return _LIB
    tmp = _LIB + ".tmp"
    subprocess.check_call(["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", "-Wall", "-o", tmp, _SRC])
    os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
        lib = ctypes.CDLL(_LIB)
        for name in ("oracle_moments_direct", "oracle_moments_hoisted"):
            f = getattr(lib, name)
            f.restype = ctypes.c_int
            f.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_int64, ctypes.c_int64,
                          ctypes.c_int64, ctypes.c_int, ctypes.c_void_p]
        lib.oracle_num_threads.restype = ctypes.c_int
        _lib = lib
    return _lib


def num_threads():
    return int(_load().oracle_num_threads())


def _call(fname, V, K):
    V = np.ascontiguousarray(V)
    if V.dtype not in (np.uint8, np.uint16):
        raise ValueError("uint8 or uint16 volume expected")
    N, M, L = V.shape
    nm = (K + 1) * (K + 2) * (K + 3) // 6
    out = np.zeros(2 * nm, dtype=np.uint64)
    rc = getattr(_load(), fname)(V.ctypes.data, V.itemsize, L, M, N, K, out.ctypes.data)
    if rc == -2:
        raise OverflowError("moments may exceed a signed 128-bit integer")
    if rc != 0:
        raise ValueError(f"{fname} failed ({rc})")
    res = []
    for i in range(nm):
        u = int(out[2 * i]) | (int(out[2 * i + 1]) << 64)
        if u >= 1 << 127:
            u -= 1 << 128
        res.append(u)
    return res


def moments_direct(V, K):
    """Per-voxel direct sum of eq. (2) (exact int128); graded order."""
    return _call("oracle_moments_direct", V, K)


def moments_hoisted(V, K):
    """Eq. (2) with hoisted powers (exact int128); graded order."""
    return _call("oracle_moments_hoisted", V, K)
