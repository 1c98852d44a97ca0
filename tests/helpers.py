"""Shared test helpers: build the same seeded problem on the oracle side and
hand the oracle's prolongations and A_0 values to the library."""
import numpy as np

import synth
from oracle import assemble as AS, hierarchy as OH, vcycle as OV


def gpu_available():
    try:
        import torch
        return torch.cuda.is_available()
    except Exception:
        return False


def ell3(P):
    """scipy CSR prolongation (1-3 entries per row) -> ELL-3 (cols, w)."""
    P = P.tocsr()
    n = P.shape[0]
    cols = -np.ones((n, 3), dtype=np.int32)
    w = np.zeros((n, 3))
    cnt = np.diff(P.indptr)
    assert cnt.max() <= 3
    for s in range(3):
        m = cnt > s
        idx = P.indptr[:-1][m] + s
        cols[m, s] = P.indices[idx]
        w[m, s] = P.data[idx]
    return cols, w


def mesh_case(name):
    rng = np.random.default_rng(17)
    if name == "icosphere-L5":
        w = synth.workload_c1()
        return w["V"], w["F"], w["t"], w["n_levels"]
    if name == "disc-41x37":
        V, F = synth.flat_disc(41, 37, seed=3, jitter=0.1)
        return V, F, 1e-2, 4
    if name == "torus-96x40":
        V, F = synth.torus_grid(96, 40, 1.0, 0.3, rng, jitter=0.2)
        return V, F, 1e-2, 5
    if name == "heightfield-70x66":
        V, F = synth.disc_grid(70, 66, rng, 0.1, height=lambda x, y: 0.1 * np.sin(3 * x) * np.cos(2 * y))
        return V, F, 3e-2, 4
    raise KeyError(name)


class Problem:
    """Oracle hierarchy + oracle A_0 for a named mesh."""

    def __init__(self, name, n_levels=None):
        V, F, t, nl = mesh_case(name)
        self.name, self.V, self.F, self.t = name, V, F, t
        self.n_levels = nl if n_levels is None else n_levels
        self.A, self.L, self.m = AS.system(V, F, t)
        self.Ps, self.meshes, _ = OH.prolongations(V, F, n_levels=self.n_levels)
        self.oracle = OV.Solver(self.Ps, self.A)
        self.sizes = [len(V)] + [P.shape[1] for P in self.Ps]

    def gpu_solver(self, mu_pre=2, mu_post=2, faces=False, **kw):
        import torch
        from paper_2104_13755_amd.solver import Hierarchy, Solver
        ells = [ell3(P) for P in self.Ps]
        h = Hierarchy.from_prolongations(self.sizes, [e[0] for e in ells], [e[1] for e in ells])
        S = Solver(h, self.A.indptr, self.A.indices, mu_pre=mu_pre, mu_post=mu_post,
                   faces=self.F if faces else None, **kw)
        S.set_values(torch.tensor(self.A.data, dtype=torch.float64, device="cuda"))
        return S


def rel(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    den = np.abs(b).max()
    return float(np.abs(a - b).max() / (den if den > 0 else 1.0))
