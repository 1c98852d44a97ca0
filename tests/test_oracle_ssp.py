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
    Vc, Fc, Pc, Pw, st = native.ssp_level(V, F, H.next_target(n), interior_only=True)
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
    Vc, Fc, Pc, Pw, st = native.ssp_level(V @ Q.T + off, F, H.next_target(n), interior_only=True)
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
