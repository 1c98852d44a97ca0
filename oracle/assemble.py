"""ORACLE (test infrastructure only): system matrix A = M + t L of the paper's
examples (Sec. 6 "Applications": cotangent Laplacian, mass matrix; App. E
writes the data-smoothing system as alpha Q + (1 - alpha) M).

The paper uses L and M without defining them; the reading taken here is the
standard one:
  L_ij = -1/2 (cot alpha_ij + cot beta_ij) for every mesh edge (i, j), with one
         term on boundary edges (natural Neumann boundary),
  L_ii = -sum_{j != i} L_ij  (positive semi-definite sign convention),
  M_ii = sum over faces f containing i of area(f) / 3  (lumped barycentric).
Optional per-edge weights w scale the off-diagonal entries of L (the diagonal
stays minus the row sum) and per-vertex scales s multiply M.

Every matrix returned has the structural pattern {diagonal} U {mesh edges},
columns sorted, explicit zeros kept.
"""
import numpy as np
import scipy.sparse as sp


def edge_list(F):
    """Unique undirected edges (i < j), sorted lexicographically."""
    E = np.concatenate([F[:, [0, 1]], F[:, [1, 2]], F[:, [2, 0]]], axis=0).astype(np.int64)
    E.sort(axis=1)
    n1 = int(E.max()) + 1
    key = np.unique(E[:, 0] * n1 + E[:, 1])
    return np.stack([key // n1, key % n1], axis=1)


def face_areas(V, F):
    e1 = V[F[:, 1]] - V[F[:, 0]]
    e2 = V[F[:, 2]] - V[F[:, 0]]
    return 0.5 * np.linalg.norm(np.cross(e1, e2), axis=1)


def cotan_weights(V, F):
    """For every face and corner c, cot of the angle at corner c; that angle is
    opposite the edge (F[:, c+1], F[:, c+2])."""
    cots = np.empty((len(F), 3))
    for c in range(3):
        a, b, o = F[:, (c + 1) % 3], F[:, (c + 2) % 3], F[:, c]
        u = V[a] - V[o]
        v = V[b] - V[o]
        cots[:, c] = (u * v).sum(1) / np.linalg.norm(np.cross(u, v), axis=1)
    return cots


def pattern(n, F):
    """CSR pattern {diag} U {edges}: (indptr, indices)."""
    E = edge_list(F)
    r = np.concatenate([np.arange(n), E[:, 0], E[:, 1]])
    c = np.concatenate([np.arange(n), E[:, 1], E[:, 0]])
    S = sp.csr_matrix((np.ones(len(r)), (r, c)), shape=(n, n))
    S.sort_indices()
    return S.indptr.astype(np.int64), S.indices.astype(np.int64)


def _on_pattern(n, F, rows, cols, vals):
    """Sum (rows, cols, vals) onto the full structural pattern."""
    indptr, indices = pattern(n, F)
    A = sp.csr_matrix((np.zeros(len(indices)), indices, indptr), shape=(n, n))
    V = sp.csr_matrix((vals, (rows, cols)), shape=(n, n))
    V.sum_duplicates()
    V.sort_indices()
    # scatter V into A's pattern (V's pattern is a subset of A's)
    out = A.copy()
    Acoo = A.tocoo()
    key_a = Acoo.row.astype(np.int64) * n + Acoo.col
    Vcoo = V.tocoo()
    key_v = Vcoo.row.astype(np.int64) * n + Vcoo.col
    pos = np.searchsorted(key_a, key_v)
    assert np.all(key_a[pos] == key_v)
    data = np.zeros(len(key_a))
    np.add.at(data, pos, Vcoo.data)
    out.data = data
    return out


def laplacian(V, F, edge_weights=None, edges=None):
    """Cotangent Laplacian (PSD convention).  ``edge_weights`` (optional) are
    given per edge of ``edges`` (default: ``edge_list(F)``)."""
    n = len(V)
    cots = cotan_weights(V, F)
    rows, cols, vals = [], [], []
    for c in range(3):
        a, b = F[:, (c + 1) % 3], F[:, (c + 2) % 3]
        w = -0.5 * cots[:, c]
        rows += [a, b]
        cols += [b, a]
        vals += [w, w]
    rows = np.concatenate(rows)
    cols = np.concatenate(cols)
    vals = np.concatenate(vals)
    if edge_weights is not None:
        E = edge_list(F) if edges is None else edges
        lo = np.minimum(rows, cols)
        hi = np.maximum(rows, cols)
        n1 = n + 1
        ekey = E[:, 0].astype(np.int64) * n1 + E[:, 1]
        pos = np.searchsorted(ekey, lo.astype(np.int64) * n1 + hi)
        assert np.all(ekey[pos] == lo.astype(np.int64) * n1 + hi)
        vals = vals * np.asarray(edge_weights)[pos]
    offsum = np.zeros(n)
    np.add.at(offsum, rows, vals)
    rows = np.concatenate([rows, np.arange(n)])
    cols = np.concatenate([cols, np.arange(n)])
    vals = np.concatenate([vals, -offsum])
    return _on_pattern(n, F, rows, cols, vals)


def mass(V, F):
    """Lumped barycentric mass: one third of the incident face areas."""
    n = len(V)
    m = np.zeros(n)
    ar = face_areas(V, F) / 3.0
    for c in range(3):
        np.add.at(m, F[:, c], ar)
    return m


def system(V, F, t, mass_scale=None, edge_weights=None, edges=None):
    """A = diag(s * m) + t L on the structural pattern; returns (A, L, m)."""
    L = laplacian(V, F, edge_weights, edges)
    m = mass(V, F)
    mm = m if mass_scale is None else m * np.asarray(mass_scale)
    A = L.copy()
    A.data = t * L.data
    A = A + sp.diags(mm, format="csr")
    A = _same_pattern(A, L)
    return A, L, m


def _same_pattern(A, ref):
    """Return A's values on ref's structural pattern (A's pattern is a subset)."""
    n = ref.shape[0]
    A = A.tocsr()
    A.sort_indices()
    R = ref.tocoo()
    key_r = R.row.astype(np.int64) * n + R.col
    C = A.tocoo()
    key_c = C.row.astype(np.int64) * n + C.col
    pos = np.searchsorted(key_r, key_c)
    assert np.all(key_r[pos] == key_c)
    data = np.zeros(len(key_r))
    data[pos] = C.data
    out = ref.copy()
    out.data = data
    return out
