"""ctypes loader for the oracle's plain-C parts (``ssp.c``, ``coloring.c``).

ORACLE: test infrastructure only.  The shared object is built with gcc at
-O2 -ffp-contract=off (no fused multiply-add, so every rounding step is the
one written in the source).
"""
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "liboracle.so")
_SRC = [os.path.join(_HERE, "ssp.c"), os.path.join(_HERE, "coloring.c")]
_lib = None


def build(force=True):
    if force or not os.path.exists(_SO):
        cmd = ["gcc", "-O2", "-std=c99", "-ffp-contract=off", "-fPIC", "-shared",
               "-o", _SO] + _SRC + ["-lm"]
        subprocess.run(cmd, check=True)
    return _SO


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            build()
        L = ctypes.CDLL(_SO)
        ip = np.ctypeslib.ndpointer(dtype=np.int32, flags="C_CONTIGUOUS")
        dp = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")
        L.oracle_ssp_level.argtypes = [ctypes.c_int, dp, ctypes.c_int, ip, ctypes.c_int,
                                       ctypes.c_int, ctypes.POINTER(ctypes.c_int), dp,
                                       ctypes.POINTER(ctypes.c_int), ip, ip, dp, dp]
        L.oracle_ssp_level.restype = ctypes.c_int
        L.oracle_color.argtypes = [ctypes.c_int, ip, ip, ip]
        L.oracle_color.restype = ctypes.c_int
        _lib = L
    return _lib


def ssp_level(V, F, target, interior_only=False):
    """One decimation level.  Returns (Vc, Fc, Pcols (n,3), Pw (n,3), stats)."""
    V = np.ascontiguousarray(V, dtype=np.float64)
    F = np.ascontiguousarray(F, dtype=np.int32)
    n, m = len(V), len(F)
    Xc = np.zeros(3 * n, dtype=np.float64)
    Fc = np.zeros(3 * m, dtype=np.int32)
    Pc = np.zeros(3 * n, dtype=np.int32)
    Pw = np.zeros(3 * n, dtype=np.float64)
    st = np.zeros(8, dtype=np.float64)
    nc = ctypes.c_int(0)
    mc = ctypes.c_int(0)
    rc = lib().oracle_ssp_level(n, V.ravel(), m, F.ravel(), int(target), int(bool(interior_only)),
                                ctypes.byref(nc), Xc, ctypes.byref(mc), Fc, Pc, Pw, st)
    if rc != 0:
        raise RuntimeError(f"oracle SSP failed with code {rc}")
    stats = dict(collapses=int(st[0]), fails=int(st[1]), interior=int(st[2]),
                 one_boundary=int(st[3]), b_case1=int(st[4]), b_case2=int(st[5]),
                 b_case3=int(st[6]), max_clamp=float(st[7]))
    return (Xc[:3 * nc.value].reshape(-1, 3).copy(), Fc[:3 * mc.value].reshape(-1, 3).copy(),
            Pc.reshape(-1, 3), Pw.reshape(-1, 3), stats)


def color(rowptr, cols):
    rowptr = np.ascontiguousarray(rowptr, dtype=np.int32)
    cols = np.ascontiguousarray(cols, dtype=np.int32)
    n = len(rowptr) - 1
    out = np.zeros(max(n, 1), dtype=np.int32)
    nc = lib().oracle_color(n, rowptr, cols, out)
    return out[:n].copy(), int(nc)
