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
        L.oracle_ssp_level_probe.argtypes = L.oracle_ssp_level.argtypes + [
            dp, ctypes.c_int, ctypes.POINTER(ctypes.c_int), dp]
        L.oracle_ssp_level_probe.restype = ctypes.c_int
        L.oracle_color.argtypes = [ctypes.c_int, ip, ip, ip]
        L.oracle_color.restype = ctypes.c_int
        _lib = L
    return _lib


# collapse sets of oracle_ssp_level: the method, and two test restrictions
# with a closed form on a flat disc (interior edges only; interior edges plus
# boundary edges on straight boundary runs, no one-boundary collapse)
COLLAPSES = {"all": 0, "interior": 1, "straight": 2}

# probe record layout (ssp.c): header, ring ids, before faces, three cases
MAXD = MAXF = 96
PR_HDR = 10
PR_RING = PR_HDR
PR_FACE = PR_RING + MAXD
PR_CASE0 = PR_FACE + 3 * MAXF
PR_CASE_SIZE = 2 + 2 * MAXD + 6
PR_SIZE = PR_CASE0 + 3 * PR_CASE_SIZE


def _level_call(V, F, target, collapses, probe_cap):
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
    args = (n, V.ravel(), m, F.ravel(), int(target), COLLAPSES[collapses],
            ctypes.byref(nc), Xc, ctypes.byref(mc), Fc, Pc, Pw, st)
    probe = None
    if probe_cap:
        rec = np.zeros(probe_cap * PR_SIZE, dtype=np.float64)
        Xall = np.zeros(3 * (2 * n + 8), dtype=np.float64)
        npr = ctypes.c_int(0)
        rc = lib().oracle_ssp_level_probe(*args, rec, int(probe_cap), ctypes.byref(npr), Xall)
        probe = (rec[:npr.value * PR_SIZE].reshape(-1, PR_SIZE).copy(), Xall.reshape(-1, 3))
    else:
        rc = lib().oracle_ssp_level(*args)
    if rc != 0:
        raise RuntimeError(f"oracle SSP failed with code {rc}")
    stats = dict(collapses=int(st[0]), fails=int(st[1]), interior=int(st[2]),
                 one_boundary=int(st[3]), b_case1=int(st[4]), b_case2=int(st[5]),
                 b_case3=int(st[6]), max_clamp=float(st[7]))
    out = (Xc[:3 * nc.value].reshape(-1, 3).copy(), Fc[:3 * mc.value].reshape(-1, 3).copy(),
           Pc.reshape(-1, 3), Pw.reshape(-1, 3), stats)
    return out, probe


def ssp_level(V, F, target, collapses="all"):
    """One decimation level.  Returns (Vc, Fc, Pcols (n,3), Pw (n,3), stats)."""
    return _level_call(V, F, target, collapses, 0)[0]


def ssp_level_probe(V, F, target, collapses="all", cap=4096):
    """As ssp_level, plus the probe: a list of dicts, one per committed
    collapse (at most ``cap``), with the labels the oracle gave it (kind,
    i, j, p, q, k), its ring and before faces, and per flattening case the
    status, energy and UV positions; and the positions of every vertex the
    level created (new ids continue after the input's)."""
    out, (rec, Xall) = _level_call(V, F, target, collapses, cap)
    recs = []
    for r in rec:
        nr, nfb, ncase = int(r[7]), int(r[8]), int(r[9])
        cases = []
        for cs in range(ncase):
            c = r[PR_CASE0 + cs * PR_CASE_SIZE: PR_CASE0 + (cs + 1) * PR_CASE_SIZE]
            tail = c[2 + 2 * MAXD:]
            cases.append(dict(status=c[0], energy=c[1], ring_uv=c[2:2 + 2 * nr].reshape(nr, 2).copy(),
                              uv_i=tail[0:2].copy(), uv_j=tail[2:4].copy(), uv_k=tail[4:6].copy()))
        recs.append(dict(kind=int(r[0]), chosen=int(r[1]), i=int(r[2]), j=int(r[3]),
                         p=int(r[4]), q=int(r[5]), k=int(r[6]),
                         ring=r[PR_RING:PR_RING + nr].astype(np.int64),
                         faces=r[PR_FACE:PR_FACE + 3 * nfb].reshape(nfb, 3).astype(np.int64),
                         cases=cases))
    return out, recs, Xall


def color(rowptr, cols):
    rowptr = np.ascontiguousarray(rowptr, dtype=np.int32)
    cols = np.ascontiguousarray(cols, dtype=np.int32)
    n = len(rowptr) - 1
    out = np.zeros(max(n, 1), dtype=np.int32)
    nc = lib().oracle_color(n, rowptr, cols, out)
    return out[:n].copy(), int(nc)
