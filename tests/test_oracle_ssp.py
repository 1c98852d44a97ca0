"""Pins of the oracle's successive self-parameterization (paper Sec. 4)."""
import numpy as np
import pytest

import synth
from oracle import hierarchy as H, native


def _dense_rows(Pc, Pw, nc):
    n = len(Pc)
    D = np.zeros((n, nc))
    for c in range(3):
        m = Pw[:, c] > 0
        np.add.at(D, (np.flatnonzero(m), Pc[m, c]), Pw[m, c])
    return D


def _planar_bary(p, A, B, C):
    def cr(u, v, w):
        return (v[0] - u[0]) * (w[1] - u[1]) - (v[1] - u[1]) * (w[0] - u[0])
    T = cr(A, B, C)
    return np.array([cr(p, B, C), cr(A, p, C), cr(A, B, p)]) / T


def test_flat_closed_form_interior_collapses():
    """On a flat disc with only interior collapses, the joint LSCM minimum is the
    planar embedding (zero conformal energy), so every row of P must be the
    planar barycentric coordinates of the fine vertex in the coarse triangle
    that contains it (found here by brute force) and P reproduces linear
    functions exactly."""
    V, F = synth.flat_disc(32, seed=11, jitter=0.1)
    n = len(V)
    Vc, Fc, Pc, Pw, st = native.ssp_level(V, F, H.next_target(n), "interior")
    assert st["collapses"] > 0 and st["one_boundary"] == 0
    D = _dense_rows(Pc, Pw, len(Vc))
    # linear reproduction
    assert abs(D @ Vc[:, :2] - V[:, :2]).max() < 1e-13
    # brute-force point location in the coarse mesh
    for v in range(n):
        p = V[v, :2]
        best, bb = -np.inf, None
        for f in Fc:
            lam = _planar_bary(p, Vc[f[0], :2], Vc[f[1], :2], Vc[f[2], :2])
            if lam.min() > best:
                best, bb, bf = lam.min(), lam, f
        assert best > -1e-12
        ref = np.zeros(len(Vc))
        ref[bf] = np.clip(bb, 0, None) / np.clip(bb, 0, None).sum()
        assert abs(D[v] - ref).max() < 1e-10, v


def test_flat_closed_form_in_a_tilted_plane():
    """The parameterization is intrinsic (Sec. 4 flattens by edge lengths and
    angles), so the flat-disc closed form must hold unchanged once the disc is
    moved rigidly into a general plane of R^3: dropping the z coordinate, or
    any other use of raw coordinates, breaks it."""
    V, F = synth.flat_disc(32, seed=11, jitter=0.1)
    rng = np.random.default_rng(3)
    Q, _ = np.linalg.qr(rng.normal(size=(3, 3)))
    off = np.array([0.3, -1.7, 2.2])
    n = len(V)
    Vc, Fc, Pc, Pw, st = native.ssp_level(V @ Q.T + off, F, H.next_target(n), "interior")
    assert st["collapses"] > 0
    D = _dense_rows(Pc, Pw, len(Vc))
    Uc = ((Vc - off) @ Q)[:, :2]          # coarse vertices back in the disc's plane
    U = V[:, :2]
    assert abs(D @ Uc - U).max() < 1e-13
    for v in range(n):
        best = -np.inf
        for f in Fc:
            lam = _planar_bary(U[v], Uc[f[0]], Uc[f[1]], Uc[f[2]])
            if lam.min() > best:
                best, bb, bf = lam.min(), lam, f
        assert best > -1e-12
        ref = np.zeros(len(Vc))
        ref[bf] = np.clip(bb, 0, None) / np.clip(bb, 0, None).sum()
        assert abs(D[v] - ref).max() < 1e-10, v


def test_similarity_invariance():
    """Every quantity the hierarchy depends on (quadric costs, edge lengths,
    angles) is invariant under rigid motion, and a power-of-two scale changes
    them by exact factors: scaling gives bitwise the same operators, a rigid
    motion the same sparsity with values equal to rounding."""
    rng = np.random.default_rng(5)
    V, F = synth.torus_grid(60, 24, 1.0, 0.3, rng, jitter=0.2)
    Ps, _, _ = H.prolongations(V, F, n_levels=3)
    Ps_scaled, _, _ = H.prolongations(4.0 * V, F, n_levels=3)
    for a, b in zip(Ps, Ps_scaled):
        assert a.shape == b.shape and (a != b).nnz == 0
    Q, _ = np.linalg.qr(rng.normal(size=(3, 3)))
    Ps_moved, _, _ = H.prolongations(V @ Q.T + np.array([0.5, -0.25, 1.0]), F, n_levels=3)
    for a, b in zip(Ps, Ps_moved):
        assert a.shape == b.shape
        assert (a.indptr == b.indptr).all() and (a.indices == b.indices).all()
        assert abs(a - b).max() < 1e-12


@pytest.mark.parametrize("mesh", ["icosphere", "torus", "disc", "heightfield"])
def test_prolongation_invariants(mesh):
    rng = np.random.default_rng(5)
    if mesh == "icosphere":
        V, F = synth.small_icosphere(4, seed=3, sigma=0.01)
    elif mesh == "torus":
        V, F = synth.torus_grid(60, 24, 1.0, 0.3, rng, jitter=0.2)
    elif mesh == "disc":
        V, F = synth.flat_disc(40, seed=4, jitter=0.1)
    else:
        V, F = synth.disc_grid(40, 38, rng, 0.1, height=lambda x, y: 0.1 * np.sin(3 * x) * np.cos(2 * y))
    chi = len(V) - len(synth.edges_of(F)) + len(F)
    Ps, meshes, stats = H.prolongations(V, F, n_levels=3)
    for l, P in enumerate(Ps):
        n_f, n_c = P.shape
        assert n_f == len(meshes[l][0])
        assert P.data.min() > 0
        rs = np.asarray(P.sum(axis=1)).ravel()
        assert abs(rs - 1).max() < 1e-14
        nnz = np.diff(P.indptr)
        assert nnz.min() >= 1 and nnz.max() <= 3
        assert np.asarray(P.max(axis=0).todense()).min() > 0     # no zero column
        Vc, Fc = meshes[l + 1]
        assert len(Vc) - len(synth.edges_of(Fc)) + len(Fc) == chi   # topology kept
        assert stats[l]["max_clamp"] < 1e-8
    if mesh in ("disc", "heightfield"):
        s = stats[0]
        assert s["one_boundary"] > 0 and s["b_case1"] + s["b_case2"] + s["b_case3"] > 0


def test_targets_and_determinism():
    V, F = synth.small_icosphere(4, seed=9)
    Ps1, m1, _ = H.prolongations(V, F, n_levels=3)
    Ps2, m2, _ = H.prolongations(V, F, n_levels=3)
    assert [P.shape for P in Ps1] == [(2562, 641), (641, 160)]
    for a, b in zip(Ps1, Ps2):
        assert (a != b).nnz == 0
    assert H.level_count(10242) == 3 and H.level_count(655362) == 6


# ---------------------------------------------------------------------------
# Boundary collapses (Sec. 4.3 "Boundary Edges", Eq. jointEnergy).


def _patch_area(X, faces):
    e1 = X[faces[:, 1]] - X[faces[:, 0]]
    e2 = X[faces[:, 2]] - X[faces[:, 0]]
    return 0.5 * np.linalg.norm(np.cross(e1, e2), axis=1).sum()


@pytest.mark.parametrize("tilted", [False, True])
def test_straight_boundary_closed_form(tilted):
    """With boundary-edge collapses allowed on straight boundary runs (p, i,
    j, q on one line) next to the interior ones, a flat disc whose sides are
    exactly straight still has a zero-energy joint flattening for every
    collapse: for a boundary edge it is the third case (k on the line through
    i and j, every colinearity constraint met by the planar embedding), while
    k on i or on j distorts the after patch (k sits at the 3D midpoint).  So
    every boundary collapse must pick the third case with energy zero to
    rounding, and every row of P must be the planar barycentric coordinates
    of its fine vertex, found by brute force."""
    V, F = synth.flat_disc(32, seed=11, jitter=0.1)
    n = len(V)
    if tilted:
        rng = np.random.default_rng(3)
        Q, _ = np.linalg.qr(rng.normal(size=(3, 3)))
        off = np.array([0.3, -1.7, 2.2])
        Vin = V @ Q.T + off
    else:
        Vin = V
    (Vc, Fc, Pc, Pw, st), recs, Xall = native.ssp_level_probe(Vin, F, H.next_target(n), "straight")
    assert st["b_case3"] > 20 and st["interior"] > 0
    assert st["b_case1"] == st["b_case2"] == st["one_boundary"] == 0
    nb = 0
    for r in recs:
        area = _patch_area(Xall, r["faces"])
        if r["kind"] == 2:
            nb += 1
            assert r["chosen"] == 2
            e = [c["energy"] for c in r["cases"]]
            assert e[2] <= 1e-20 * area, e
            assert min(e[0], e[1]) > 1e-8 * area, e
        else:
            assert r["kind"] == 0 and r["cases"][0]["energy"] <= 1e-20 * area
    assert nb == st["b_case3"]
    Uc = ((Vc - off) @ Q)[:, :2] if tilted else Vc[:, :2]
    U = V[:, :2]
    D = _dense_rows(Pc, Pw, len(Vc))
    assert abs(D @ Uc - U).max() < 1e-13
    for v in range(n):
        best = -np.inf
        for f in Fc:
            lam = _planar_bary(U[v], Uc[f[0]], Uc[f[1]], Uc[f[2]])
            if lam.min() > best:
                best, bb, bf = lam.min(), lam, f
        assert best > -1e-12
        ref = np.zeros(len(Vc))
        ref[bf] = np.clip(bb, 0, None) / np.clip(bb, 0, None).sum()
        assert abs(D[v] - ref).max() < 1e-10, v


def _conformal_rows(P):
    """Rows r(u, v) = sqrt(area) (grad v - n x grad u) of one 3D triangle P
    (3 x 3), as a 3 x 6 matrix acting on (u0, u1, u2, v0, v1, v2); |r|^2 is
    the triangle's conformal (LSCM) energy area * |grad v - n x grad u|^2,
    written with 3D gradients of the hat functions (no local frame)."""
    c = np.cross(P[1] - P[0], P[2] - P[0])
    A2 = np.linalg.norm(c)
    nrm = c / A2
    G = np.array([np.cross(nrm, P[(t + 2) % 3] - P[(t + 1) % 3]) / A2 for t in range(3)])  # grad of hat t
    NG = np.cross(nrm, G)                                                                   # n x grad
    return np.sqrt(0.5 * A2) * np.hstack([-NG.T, G.T])


def _labels(faces, i_or_a, j_or_b):
    """Boundary status and orientation from the before patch alone: every face
    at the two endpoints is in it, so an edge at an endpoint is a boundary edge
    iff exactly one patch face has it."""
    def count(u, w):
        return sum(1 for f in faces if u in f and w in f)

    def bnd_nbrs(v):
        nb = {w for f in faces if v in f for w in f if w != v}
        return sorted(w for w in nb if count(v, w) == 1)
    a, b = i_or_a, j_or_b
    if count(a, b) == 1:
        f = next(f for f in faces if a in f and b in f)
        fl = list(f)
        ia = fl.index(a)
        i, j = (a, b) if fl[(ia + 1) % 3] == b else (b, a)
        p = [w for w in bnd_nbrs(i) if w != j]
        q = [w for w in bnd_nbrs(j) if w != i]
        assert len(p) == 1 and len(q) == 1
        return 2, i, j, p[0], q[0]
    ba, bb = bool(bnd_nbrs(a)), bool(bnd_nbrs(b))
    assert not (ba and bb)
    if ba:
        return 1, b, a, -1, -1
    if bb:
        return 1, a, b, -1, -1
    return 0, a, b, -1, -1


def _independent_flattening(X, faces, kind, i, j, p, q, k, case):
    """Joint conformal flattening of the edge 1-ring before the collapse and
    the vertex 1-ring after it (Eq. jointEnergy), for the joint variable of
    the given case: interior edge (k its own unknown), one boundary endpoint j
    (k shares j's UV), boundary edge with k on i (case 0), k on j (case 1) or
    k on the line through i and j (case 2), with v = 0 on the colinear
    vertices and the first / last of them at u = 0 / the 3D chain length.
    Interior and one-boundary collapses fix the two ring vertices farthest
    apart in 3D (lowest ids on ties) at (0, 0) and (d, 0).  Solved with
    numpy least squares over the free coordinates.  Returns
    (energy, {vertex: uv} for ring, i, j in the before patch and k in the
    after patch, scale, min signed area over both patches)."""
    ring = sorted({w for f in faces for w in f} - {i, j})
    var = {w: s for s, w in enumerate(ring)}
    var[i] = len(ring)
    var[j] = len(ring) + 1
    if kind == 0 or (kind == 2 and case == 2):
        var[k] = len(ring) + 2
    elif kind == 1 or case == 1:
        var[k] = var[j]
    else:
        var[k] = var[i]
    nv = max(var.values()) + 1
    before = [tuple(f) for f in faces]
    after = [tuple(k if w in (i, j) else w for w in f) for f in faces if not (i in f and j in f)]
    Xk = X[k]
    rows = []
    for tri in before + after:
        P = np.array([Xk if w == k else X[w] for w in tri])
        Rt = _conformal_rows(P)
        M = np.zeros((3, 2 * nv))
        for t, w in enumerate(tri):
            M[:, var[w]] += Rt[:, t]
            M[:, nv + var[w]] += Rt[:, 3 + t]
        rows.append(M)
    R = np.vstack(rows)
    fix = {}
    dist = lambda a, b: float(np.linalg.norm(X[a] - X[b]))
    if kind != 2:
        best, pair = -1.0, None
        for s in range(len(ring)):
            for r in range(s + 1, len(ring)):
                d2 = float(((X[ring[s]] - X[ring[r]]) ** 2).sum())
                if d2 > best:
                    best, pair = d2, (ring[s], ring[r])
        scale = np.sqrt(best)
        fix[var[pair[0]]] = 0.0
        fix[nv + var[pair[0]]] = 0.0
        fix[var[pair[1]]] = scale
        fix[nv + var[pair[1]]] = 0.0
    else:
        line = [[i, j, q], [p, i, j], [p, i, k, j, q]][case]
        for w in line:
            fix[nv + var[w]] = 0.0
        chain = [[i, j, q], [p, i, j], [p, i, j, q]][case]
        scale = sum(dist(a, b) for a, b in zip(chain[:-1], chain[1:]))
        fix[var[line[0]]] = 0.0
        fix[var[line[-1]]] = scale
    z = np.zeros(2 * nv)
    fixed_cols = np.array(sorted(fix))
    z[fixed_cols] = [fix[c] for c in fixed_cols]
    free = np.array([c for c in range(2 * nv) if c not in fix])
    sol = np.linalg.lstsq(R[:, free], -R[:, fixed_cols] @ z[fixed_cols], rcond=None)[0]
    z[free] = sol
    energy = float(((R @ z) ** 2).sum())
    uv = {w: np.array([z[var[w]], z[nv + var[w]]]) for w in ring + [i, j, k]}
    uvk = uv[k]

    def sarea(tri, which):
        P = [uvk if (w == k and which == "a") else uv[w] for w in tri]
        return 0.5 * ((P[1][0] - P[0][0]) * (P[2][1] - P[0][1]) - (P[1][1] - P[0][1]) * (P[2][0] - P[0][0]))
    amin = min([sarea(t, "b") for t in before] + [sarea(t, "a") for t in after])
    return energy, uv, scale, amin


@pytest.mark.parametrize("mesh", ["flat", "heightfield"])
def test_collapses_match_an_independent_joint_flattening(mesh):
    """Every collapse of one level, on discs whose boundary is bent in 3D
    (height field) or has corners (flat square): the oracle's labels (kind,
    i -> j along the boundary face, previous p and next q boundary vertex), its
    per-case energies, its UV positions and its validity decision must equal
    an independent solve of Eq. jointEnergy for each joint variable of Sec.
    4.3, and the chosen boundary case must be the one of least energy (ties
    to the lower case).  Covers interior, one-boundary (snap of k to the
    boundary endpoint j) and all three boundary-edge cases."""
    rng = np.random.default_rng(7)
    if mesh == "flat":
        V, F = synth.flat_disc(40, seed=4, jitter=0.1)
    else:
        V, F = synth.disc_grid(24, 22, rng, 0.1, height=lambda x, y: 0.3 * np.sin(3 * x) * np.cos(2 * y))
    (Vc, Fc, Pc, Pw, st), recs, Xall = native.ssp_level_probe(V, F, H.next_target(len(V)), "all")
    assert len(recs) == st["collapses"]
    seen = {"interior": 0, "one": 0, "case": [0, 0, 0]}
    for r in recs:
        faces = r["faces"]
        kind, i, j, p, q = _labels([tuple(f) for f in faces], min(r["i"], r["j"]), max(r["i"], r["j"]))
        assert (kind, i, j) == (r["kind"], r["i"], r["j"]), r
        if kind == 2:
            assert (p, q) == (r["p"], r["q"])
        assert list(r["ring"]) == sorted({w for f in faces for w in f} - {i, j})
        energies, valid = [], []
        for cs, c in enumerate(r["cases"]):
            E, uv, scale, amin = _independent_flattening(Xall, faces, kind, i, j, p, q, r["k"], cs)
            ok = amin > 1e-12 * scale * scale
            assert (c["status"] == 0) == ok, (r, cs, amin)
            assert abs(c["energy"] - E) <= 1e-8 * E + 1e-12 * scale * scale, (c["energy"], E)
            got = {w: c["ring_uv"][s] for s, w in enumerate(r["ring"])}
            got.update({i: c["uv_i"], j: c["uv_j"]})
            for w, g in got.items():
                assert abs(g - uv[w]).max() <= 1e-9 * scale, (w, g, uv[w])
            assert abs(c["uv_k"] - uv[r["k"]]).max() <= 1e-9 * scale
            energies.append(E if ok else np.inf)
        if kind == 2:
            order = np.argsort(energies, kind="stable")
            e0, e1 = energies[order[0]], energies[order[1]]
            assert r["chosen"] == order[0] or abs(e1 - e0) <= 1e-9 * e0, (r["chosen"], energies)
            seen["case"][r["chosen"]] += 1
        elif kind == 1:
            seen["one"] += 1
        else:
            seen["interior"] += 1
    assert seen["interior"] > 0 and seen["one"] > 0
    assert seen["case"][2] > 0 and seen["case"][0] + seen["case"][1] > 0, seen
