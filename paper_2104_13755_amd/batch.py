"""Batched solves of many meshes in one persistent launch (libsmg batch API)."""
import ctypes

import torch

from . import _lib as L
from .solver import PRECISION, _dev_f64, _stream

_c = ctypes.c_void_p


class BatchSolver:
    """Solve many (mesh, right-hand sides) systems at once.  ``solvers`` are
    paper_2104_13755_amd.solver.Solver objects with values set; they must
    outlive the batch."""

    def __init__(self, solvers, threads=0, lanes_level0=0, lanes_coarse=0, team_max=0, cache_file=None,
                 device_teams=False, balance=False):
        """device_teams: teams anywhere on the device with device-scope
        barriers, instead of each team on one XCD with barriers in its L2.
        balance: workgroups per mesh by level-0 entries x the last solve's
        cycles (from the second solve on) instead of by entries."""
        self._lib = L.load()
        self.solvers = list(solvers)
        arr = (_c * len(self.solvers))(*[s._s for s in self.solvers])
        self._cache = cache_file.encode() if cache_file else None
        o = L.BatchOpts(int(threads), int(lanes_level0), int(lanes_coarse), int(team_max), self._cache,
                        int(bool(device_teams)), int(bool(balance)))
        h = _c()
        L.check(self._lib.smg_batch_create(arr, len(self.solvers), ctypes.byref(o), ctypes.byref(h)), "batch_create")
        self._b = h

    def __del__(self):
        if getattr(self, "_b", None):
            self._lib.smg_batch_destroy(self._b)
            self._b = None

    def solve(self, bs, rtol=1e-8, max_cycles=200, precision="fp32ir", raise_on_error=True):
        bs = [_dev_f64(b if b.dim() == 2 else b.unsqueeze(1)) for b in bs]
        xs = [torch.empty_like(b) for b in bs]
        n = len(bs)
        pb = (_c * n)(*[_c(b.data_ptr()) for b in bs])
        px = (_c * n)(*[_c(x.data_ptr()) for x in xs])
        ks = (ctypes.c_int32 * n)(*[b.shape[1] for b in bs])
        p = L.SolveParams(float(rtol), int(max_cycles), PRECISION[precision], 0, 0)
        infos = (L.SolveInfo * n)()
        st = self._lib.smg_batch_solve(self._b, pb, px, ks, ctypes.byref(p), infos, _stream())
        if raise_on_error:
            L.check(st, "batch_solve")
        out = [dict(cycles=i.cycles, rel_res=list(i.rel_res)[:i.k], ms=i.ms) for i in infos]
        return xs, out, st

    def autotune(self, budget_ms=2000):
        L.check(self._lib.smg_batch_autotune(self._b, int(budget_ms), _stream()), "batch_autotune")
        return self.shape()

    def shape(self):
        s = (ctypes.c_int32 * 5)()
        L.check(self._lib.smg_batch_shape(self._b, s), "batch_shape")
        return dict(threads=s[0], lanes_level0=s[1], lanes_coarse=s[2], team_max=s[3], balance=s[4])
