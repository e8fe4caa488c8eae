"""ctypes loader for the oracle's C cluster enumerator (builds it on demand)."""

from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "enum_clusters.c")
_LIB = os.path.join(_HERE, "liboracle_enum.so")
_lib = None


def build(force: bool = False) -> str:
    """Compile the enumerator with gcc (plain C, -O2)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + f".tmp{os.getpid()}"
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-shared", "-fPIC", _SRC, "-o", tmp])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        build()
        lib = ctypes.CDLL(_LIB)
        f = lib.oracle_enum_clusters
        f.restype = ctypes.c_longlong
        f.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p,
                      ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p, ctypes.c_longlong,
                      ctypes.c_void_p, ctypes.c_longlong, ctypes.POINTER(ctypes.c_longlong)]
        _lib = lib
    return _lib


def enum_clusters(n_sites: int, bu, bv, exempt, K: int):
    """Return a list of clusters, each a tuple of ascending bond ids."""
    lib = _load()
    bu = np.ascontiguousarray(bu, dtype=np.int32)
    bv = np.ascontiguousarray(bv, dtype=np.int32)
    ex = np.ascontiguousarray(exempt, dtype=np.uint8)
    nb = int(bu.shape[0])
    entries = ctypes.c_longlong(0)
    n = lib.oracle_enum_clusters(n_sites, nb, bu.ctypes.data, bv.ctypes.data, ex.ctypes.data,
                                 int(K), None, 0, None, 0, ctypes.byref(entries))
    if n <= 0:
        return []
    out_b = np.zeros(max(1, entries.value), np.int32)
    out_s = np.zeros(n, np.int32)
    m = lib.oracle_enum_clusters(n_sites, nb, bu.ctypes.data, bv.ctypes.data, ex.ctypes.data,
                                 int(K), out_b.ctypes.data, entries.value, out_s.ctypes.data, n,
                                 ctypes.byref(entries))
    if m != n:
        raise RuntimeError("oracle enumerator: inconsistent second pass")
    res = []
    pos = 0
    for s in out_s:
        res.append(tuple(int(x) for x in out_b[pos:pos + s]))
        pos += s
    return res
