"""Pins of the oracle's Galerkin operators and V-cycle (paper Sec. 3, Sec. 5,
App. A, App. E)."""
import numpy as np
import pytest
import scipy.linalg as sla
import scipy.sparse as sp

import synth
from oracle import assemble as AS, hierarchy as H, vcycle as VC


@pytest.fixture(scope="module")
def ico3():
    V, F = synth.small_icosphere(3, seed=21, sigma=0.02)
    A, L, m = AS.system(V, F, 1e-2)
    Ps, meshes, _ = H.prolongations(V, F, n_levels=3)
    return V, F, A, L, m, Ps


def test_galerkin_invariants(ico3):
    V, F, A, L, m, Ps = ico3
    Al, Ll, Ml = A, L, sp.diags(m, format="csr")
    for P in Ps:
        Ac = H.galerkin(Al, P)
        Lc = H.galerkin(Ll, P)
        Mc = H.galerkin(Ml, P)
        assert abs(Ac - Ac.T).max() <= 1e-14 * abs(Ac).max()
        np.linalg.cholesky(Ac.toarray())                         # SPD
        assert abs(Lc @ np.ones(Lc.shape[0])).max() < 1e-13      # L_c 1 = 0
        assert abs(Ac.sum() - Al.sum()) < 1e-12 * abs(Al.sum())  # 1^T A 1 kept
        # brute force: dense triple product
        dense = P.toarray().T @ Al.toarray() @ P.toarray()
        assert abs(Ac.toarray() - dense).max() < 1e-14 * abs(dense).max()
        # App. E: P^T (a Q + b M) P = a P^T Q P + b P^T M P
        lin = 0.3 * Lc + 0.7 * Mc
        assert abs(H.galerkin(0.3 * Ll + 0.7 * Ml, P) - lin).max() < 1e-14 * abs(lin).max()
        Al, Ll, Ml = Ac, Lc, Mc


def test_one_level_is_direct_solve(ico3):
    V, F, A, L, m, Ps = ico3
    S = VC.Solver([], A)
    b = np.random.default_rng(0).uniform(-1, 1, (A.shape[0], 2))
    x, cyc, hist = S.solve(b, 1e-14)
    xs = np.linalg.solve(A.toarray(), b)
    assert cyc == 1 and abs(x - xs).max() < 1e-13 * abs(xs).max()


def _forward_gs_colormajor(A, colors, x, b, sweeps):
    """Textbook forward Gauss-Seidel (D + L_strict)^{-1}(b - U x) on the matrix
    permuted to color-major order (rows sorted by (color, index))."""
    order = np.lexsort((np.arange(len(colors)), colors))
    Ap = A.toarray()[np.ix_(order, order)]
    Lo = np.tril(Ap)
    Up = np.triu(Ap, 1)
    xp = x[order].copy()
    for _ in range(sweeps):
        xp = sla.solve_triangular(Lo, b[order] - Up @ xp, lower=True)
    out = np.empty_like(x)
    out[order] = xp
    return out


def test_two_grid_textbook(ico3):
    V, F, A, L, m, Ps = ico3
    S = VC.Solver(Ps[:1], A)
    col, _ = S.colors[0]
    rng = np.random.default_rng(1)
    b = rng.uniform(-1, 1, (A.shape[0], 3))
    x0 = rng.uniform(-1, 1, (A.shape[0], 3))
    got = S.vcycle(0, x0.copy(), b)
    P = Ps[0].toarray()
    Ac = P.T @ A.toarray() @ P
    x1 = _forward_gs_colormajor(A, col, x0, b, 2)
    x2 = x1 + P @ np.linalg.solve(Ac, P.T @ (b - A @ x1))
    ref = _forward_gs_colormajor(A, col, x2, b, 2)
    assert abs(got - ref).max() < 1e-12 * abs(ref).max()


def test_three_level_converges_to_direct(ico3):
    V, F, A, L, m, Ps = ico3
    S = VC.Solver(Ps, A)
    rng = np.random.default_rng(2)
    b = rng.uniform(-1, 1, (A.shape[0], 1))
    x, cyc, hist = S.solve(b, 1e-14, max_cycles=60)
    xs = np.linalg.solve(A.toarray(), b)
    assert np.linalg.norm(x - xs) / np.linalg.norm(xs) < 1e-13
    assert hist[-1].max() <= 1e-14


def test_energy_error_monotone(ico3):
    V, F, A, L, m, Ps = ico3
    S = VC.Solver(Ps, A)
    rng = np.random.default_rng(3)
    b = rng.uniform(-1, 1, (A.shape[0], 1))
    xs = np.linalg.solve(A.toarray(), b)
    x = np.zeros_like(b)
    prev_e, prev_r = np.inf, np.inf
    for _ in range(6):
        x = S.vcycle(0, x, b)
        e = x - xs
        ea = float((e.T @ (A @ e)).item())
        r = np.linalg.norm(b - A @ x)
        assert ea <= prev_e
        assert r <= prev_r * 1.01
        prev_e, prev_r = ea, r


def test_multicolor_equals_serial_gs(ico3):
    """App. A: a multicolor sweep equals serial Gauss-Seidel visiting the rows
    color by color (plain scalar loop, written out)."""
    V, F, A, L, m, Ps = ico3
    S = VC.Solver(Ps, A)
    col, nc = S.colors[1]
    A1 = S.A[1].tocsr()
    n = A1.shape[0]
    rng = np.random.default_rng(4)
    b = rng.uniform(-1, 1, (n, 1))
    x0 = rng.uniform(-1, 1, (n, 1))
    got = S.relax(1, x0.copy(), b, 1)
    x = x0[:, 0].copy()
    for c in range(nc):
        for i in np.flatnonzero(col == c):
            s, d = 0.0, 0.0
            for p in range(A1.indptr[i], A1.indptr[i + 1]):
                j = A1.indices[p]
                if j == i:
                    d = A1.data[p]
                else:
                    s += A1.data[p] * x[j]
            x[i] = (b[i, 0] - s) / d
    assert abs(got[:, 0] - x).max() < 1e-13


def test_zero_rhs_column_needs_no_cycle(ico3):
    V, F, A, L, m, Ps = ico3
    S = VC.Solver(Ps, A)
    x, cyc, hist = S.solve(np.zeros((A.shape[0], 1)), 1e-8)
    assert cyc == 0 and not x.any()
