"""ORACLE (test infrastructure only): the multigrid hierarchy.

* prolongations P_l from successive self-parameterization (paper Sec. 4,
  Alg. "Galerkin Surface Multigrid Solver": P_1..P_H are precomputed from the
  mesh alone), one mid-point decimation level at a time with coarsening ratio
  0.25 (Sec. 5 defaults), then zero-column removal (App. B, last paragraph);
* Galerkin coarse operators A_{l+1} = P_l^T A_l P_l (Eq. gca with R = P^T),
  values on the structural pattern of the symbolic product;
* greedy multicolor ordering of every smoothed level (App. A, Alg. "Graph
  Coloring").

Level-count reading: with ``n_levels`` given, exactly n_levels - 1
decimations; with ``n_levels = 0``, keep decimating while the next target
floor(n/4 + 1/2) is at least ``min_coarse`` (500).
"""
import numpy as np
import scipy.sparse as sp

from . import native


def next_target(n):
    return int(np.floor(n / 4.0 + 0.5))


def level_count(n0, min_coarse=500):
    nl, n = 1, n0
    while next_target(n) >= min_coarse:
        n = next_target(n)
        nl += 1
    return nl


def prolongations(V, F, n_levels=0, min_coarse=500, collapses="all"):
    """Returns (P list of scipy CSR n_l x n_{l+1}, meshes list, stats list)."""
    if n_levels <= 0:
        n_levels = level_count(len(V), min_coarse)
    meshes = [(np.asarray(V, dtype=np.float64), np.asarray(F, dtype=np.int32))]
    Ps, stats = [], []
    for _ in range(n_levels - 1):
        Vl, Fl = meshes[-1]
        Vc, Fc, Pc, Pw, st = native.ssp_level(Vl, Fl, next_target(len(Vl)), collapses)
        n = len(Vl)
        mask = Pw > 0
        rows = np.repeat(np.arange(n), 3).reshape(n, 3)[mask]
        P = sp.csr_matrix((Pw[mask], (rows, Pc[mask])), shape=(n, len(Vc)))
        P.sort_indices()
        Ps.append(P)
        meshes.append((Vc, Fc))
        stats.append(st)
    Ps = remove_zero_columns(Ps)
    return Ps, meshes, stats


def remove_zero_columns(Ps):
    """Drop columns of P_l whose largest weight is 0 together with the matching
    rows of P_{l+1}."""
    out = []
    keep_rows = None
    for P in Ps:
        if keep_rows is not None:
            P = P[keep_rows]
        colmax = np.asarray(P.max(axis=0).todense()).ravel()
        keep = np.flatnonzero(colmax > 0)
        if len(keep) < P.shape[1]:
            P = P[:, keep]
        out.append(P.tocsr())
        keep_rows = keep
    return out


def spones(S):
    T = S.tocsr().copy()
    T.data = np.ones_like(T.data)
    return T


def on_pattern(C, S):
    """Values of C placed on the structural pattern S (C's nonzeros are a subset)."""
    n = S.shape[1]
    S = S.tocsr()
    S.sort_indices()
    Sc = S.tocoo()
    ks = Sc.row.astype(np.int64) * n + Sc.col
    Cc = C.tocoo()
    kc = Cc.row.astype(np.int64) * n + Cc.col
    pos = np.searchsorted(ks, kc)
    assert np.all(ks[pos] == kc), "numeric entry outside the structural pattern"
    data = np.zeros(len(ks))
    np.add.at(data, pos, Cc.data)
    out = S.copy()
    out.data = data
    return out


def galerkin(A, P):
    """A_c = P^T A P: numeric product placed on the symbolic product's pattern
    (explicit zeros from cancellation keep their place)."""
    S = spones(P).T @ spones(A) @ spones(P)
    C = (P.T @ A) @ P
    return on_pattern(C, S)


def coloring(A):
    """Alg. "Graph Coloring" on the off-diagonal structure of A.
    Returns (color per row, number of colors)."""
    A = A.tocsr()
    return native.color(A.indptr.astype(np.int32), A.indices.astype(np.int32))
