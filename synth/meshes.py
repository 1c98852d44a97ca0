"""Seeded triangle-mesh generators (geometry and connectivity only).

All meshes are manifold, consistently oriented (counter-clockwise seen from the
outward / upward side) and returned as ``V`` (n x 3 float64) and ``F``
(m x 3 int32, 0-based).  Quads of the grid generators are split along the
diagonal whose two opposite 3D angles sum to at most pi (the local Delaunay
choice), so every cotangent weight of the resulting mesh is non-negative up to
the jitter.
"""
import numpy as np

_PHI = (1.0 + 5.0 ** 0.5) / 2.0


def _icosahedron():
    V = np.array([[-1, _PHI, 0], [1, _PHI, 0], [-1, -_PHI, 0], [1, -_PHI, 0],
                  [0, -1, _PHI], [0, 1, _PHI], [0, -1, -_PHI], [0, 1, -_PHI],
                  [_PHI, 0, -1], [_PHI, 0, 1], [-_PHI, 0, -1], [-_PHI, 0, 1]],
                 dtype=np.float64)
    V /= np.linalg.norm(V, axis=1, keepdims=True)
    F = np.array([[0, 11, 5], [0, 5, 1], [0, 1, 7], [0, 7, 10], [0, 10, 11],
                  [1, 5, 9], [5, 11, 4], [11, 10, 2], [10, 7, 6], [7, 1, 8],
                  [3, 9, 4], [3, 4, 2], [3, 2, 6], [3, 6, 8], [3, 8, 9],
                  [4, 9, 5], [2, 4, 11], [6, 2, 10], [8, 6, 7], [9, 8, 1]],
                 dtype=np.int64)
    # orient every face outward
    c = V[F].mean(axis=1)
    nrm = np.cross(V[F[:, 1]] - V[F[:, 0]], V[F[:, 2]] - V[F[:, 0]])
    flip = (nrm * c).sum(axis=1) < 0
    F[flip] = F[flip][:, [0, 2, 1]]
    return V, F


def icosphere_subdiv(level):
    """Icosahedron refined ``level`` times by 1:4 midpoint subdivision, each new
    midpoint projected to the unit sphere (10*4^level + 2 vertices).  Old
    vertices keep their ids; midpoints are numbered in order of creation."""
    V, F = _icosahedron()
    Vl = [v for v in V]
    for _ in range(level):
        emap = {}
        nf = np.empty((4 * len(F), 3), dtype=np.int64)

        def mid(a, b):
            key = (a, b) if a < b else (b, a)
            idx = emap.get(key)
            if idx is None:
                p = Vl[a] + Vl[b]
                p = p / np.linalg.norm(p)
                idx = len(Vl)
                Vl.append(p)
                emap[key] = idx
            return idx

        for f, (a, b, c) in enumerate(F):
            ab, bc, ca = mid(a, b), mid(b, c), mid(c, a)
            nf[4 * f + 0] = (a, ab, ca)
            nf[4 * f + 1] = (b, bc, ab)
            nf[4 * f + 2] = (c, ca, bc)
            nf[4 * f + 3] = (ab, bc, ca)
        F = nf
    return np.array(Vl, dtype=np.float64), F.astype(np.int32)


def icosphere_freq(nu):
    """Class-I geodesic sphere of frequency ``nu`` (10*nu^2 + 2 vertices): each
    icosahedron face carries a nu x nu triangular lattice, projected to the unit
    sphere.  Shared edge and corner points are created once, keyed canonically."""
    V0, F0 = _icosahedron()
    ids = {}
    pts = []

    def vid(key, pos):
        i = ids.get(key)
        if i is None:
            i = len(pts)
            ids[key] = i
            pts.append(pos / np.linalg.norm(pos))
        return i

    def point(A, B, C, i, j):
        # lattice point A + i/nu (B-A) + j/nu (C-A) with a canonical key
        k = nu - i - j
        corners = ((A, k), (B, i), (C, j))
        nz = [(v, w) for v, w in corners if w > 0]
        if len(nz) == 1:
            v = nz[0][0]
            return vid(("v", v), V0[v].copy())
        if len(nz) == 2:
            (va, wa), (vb, wb) = nz
            if va > vb:
                (va, wa), (vb, wb) = (vb, wb), (va, wa)
            pos = (wa * V0[va] + wb * V0[vb]) / nu
            return vid(("e", va, vb, wb), pos)
        pos = (k * V0[A] + i * V0[B] + j * V0[C]) / nu
        return vid(("f", A, B, C, i, j), pos)

    faces = []
    for (A, B, C) in F0:
        grid = {}
        for i in range(nu + 1):
            for j in range(nu + 1 - i):
                grid[(i, j)] = point(A, B, C, i, j)
        for i in range(nu):
            for j in range(nu - i):
                faces.append((grid[(i, j)], grid[(i + 1, j)], grid[(i, j + 1)]))
                if i + j + 2 <= nu:
                    faces.append((grid[(i + 1, j)], grid[(i + 1, j + 1)],
                                  grid[(i, j + 1)]))
    return np.array(pts, dtype=np.float64), np.array(faces, dtype=np.int32)


def _angle(P, a, b, c):
    """Angle at vertex a of triangle (a, b, c), vectorised over index arrays."""
    u = P[b] - P[a]
    v = P[c] - P[a]
    cs = (u * v).sum(1) / (np.linalg.norm(u, axis=1) * np.linalg.norm(v, axis=1))
    return np.arccos(np.clip(cs, -1.0, 1.0))


def _split_quads(P, q00, q10, q11, q01):
    """Split quads (q00,q10,q11,q01) (counter-clockwise) along the locally
    Delaunay diagonal and return the (2*nq) x 3 face array."""
    # diagonal q00-q11: opposite angles at q10 (tri q00,q10,q11) and q01
    s = _angle(P, q10, q11, q00) + _angle(P, q01, q00, q11)
    use_d1 = s <= np.pi
    f1 = np.where(use_d1[:, None], np.stack([q00, q10, q11], 1),
                  np.stack([q00, q10, q01], 1))
    f2 = np.where(use_d1[:, None], np.stack([q00, q11, q01], 1),
                  np.stack([q10, q11, q01], 1))
    F = np.empty((2 * len(q00), 3), dtype=np.int64)
    F[0::2] = f1
    F[1::2] = f2
    return F.astype(np.int32)


def torus_grid(a, b, R, r, rng=None, jitter=0.0):
    """a x b torus parametric grid (u along the major circle, index i*b + j),
    both directions periodic.  ``jitter`` is the standard deviation of the
    parameter-space noise in units of the grid spacing."""
    i, j = np.meshgrid(np.arange(a), np.arange(b), indexing="ij")
    di = np.zeros((a, b))
    dj = np.zeros((a, b))
    if jitter > 0:
        di = rng.normal(0.0, jitter, size=(a, b))
        dj = rng.normal(0.0, jitter, size=(a, b))
    u = 2 * np.pi * (i + di) / a
    v = 2 * np.pi * (j + dj) / b
    P = np.stack([(R + r * np.cos(v)) * np.cos(u), (R + r * np.cos(v)) * np.sin(u),
                  r * np.sin(v)], axis=-1).reshape(-1, 3)
    idx = (i * b + j)
    ip = ((i + 1) % a) * b + j
    jp = i * b + (j + 1) % b
    ijp = ((i + 1) % a) * b + (j + 1) % b
    F = _split_quads(P, idx.ravel(), ip.ravel(), ijp.ravel(), jp.ravel())
    return P.astype(np.float64), F


def disc_grid(nx, ny, rng=None, jitter=0.0, height=None):
    """nx x ny grid on the square [-1,1]^2 (index i*ny + j, i along x).  Interior
    vertices are jittered in both directions, boundary vertices only along the
    boundary, corners not at all.  ``height(x, y)`` gives z (default 0)."""
    hx = 2.0 / (nx - 1)
    hy = 2.0 / (ny - 1)
    i, j = np.meshgrid(np.arange(nx), np.arange(ny), indexing="ij")
    x = -1.0 + hx * i
    y = -1.0 + hy * j
    if jitter > 0:
        dx = rng.normal(0.0, jitter * hx, size=(nx, ny))
        dy = rng.normal(0.0, jitter * hy, size=(nx, ny))
        bx = (i == 0) | (i == nx - 1)
        by = (j == 0) | (j == ny - 1)
        dx[bx] = 0.0
        dy[by] = 0.0
        x = x + dx
        y = y + dy
    z = np.zeros_like(x) if height is None else height(x, y)
    P = np.stack([x, y, z], axis=-1).reshape(-1, 3)
    ii, jj = np.meshgrid(np.arange(nx - 1), np.arange(ny - 1), indexing="ij")
    q00 = (ii * ny + jj).ravel()
    q10 = ((ii + 1) * ny + jj).ravel()
    q11 = ((ii + 1) * ny + jj + 1).ravel()
    q01 = (ii * ny + jj + 1).ravel()
    F = _split_quads(P, q00, q10, q11, q01)
    return P.astype(np.float64), F


def edges_of(F):
    """Unique undirected edges (i < j), sorted lexicographically."""
    E = np.concatenate([F[:, [0, 1]], F[:, [1, 2]], F[:, [2, 0]]], axis=0).astype(np.int64)
    E.sort(axis=1)
    key = np.unique(E[:, 0] * (int(E.max()) + 1) + E[:, 1])
    n1 = int(E.max()) + 1
    return np.stack([key // n1, key % n1], axis=1)


def mean_edge_length(V, F):
    E = edges_of(F)
    return float(np.linalg.norm(V[E[:, 0]] - V[E[:, 1]], axis=1).mean())
