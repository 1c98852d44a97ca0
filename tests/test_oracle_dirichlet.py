"""Pins of the oracle's Dirichlet reduction (App. "Dirichlet Boundary
Conditions"): the reduced solution equals the constrained minimizer computed
independently from the saddle-point (Lagrange multiplier) system, zero
columns of P_{u:} are removed when many values are known and the reduced
Galerkin matrices stay symmetric positive definite (for 60% known values on
the test disc; App. B removes zero columns only, and from ~70% known values
on, dependent columns make the coarse matrices singular), and the V-cycle solve of
the reduced system reaches the dense solution."""
import numpy as np
import scipy.sparse as sp
import pytest

import synth
from oracle import assemble as AS, hierarchy as H, vcycle as VC, dirichlet as DR


@pytest.fixture(scope="module")
def disc():
    V, F = synth.flat_disc(21, 19, seed=3, jitter=0.1)
    A, L, m = AS.system(V, F, 1e-2)
    Ps, _, _ = H.prolongations(V, F, n_levels=3)
    return V, F, A, m, Ps


def test_reduced_solution_is_the_constrained_minimizer(disc):
    V, F, A, m, Ps = disc
    n = A.shape[0]
    rng = np.random.default_rng(71)
    known = rng.uniform(size=n) < 0.2
    b = m[:, None] * rng.uniform(-1, 1, (n, 2))
    c = rng.uniform(-1, 1, (n, 2))
    Auu, rhs, u = DR.reduce(A, b, known, c)
    xu = np.linalg.solve(Auu.toarray(), rhs)
    x = DR.expand(xu, c, known)
    # saddle point: min 1/2 x'Ax - x'b subject to x_k = c_k
    kk = np.flatnonzero(known)
    E = sp.csr_matrix((np.ones(len(kk)), (np.arange(len(kk)), kk)), shape=(len(kk), n))
    K = sp.bmat([[A, E.T], [E, None]]).toarray()
    sol = np.linalg.solve(K, np.vstack([b, c[kk]]))
    assert np.abs(x - sol[:n]).max() < 1e-10 * np.abs(sol[:n]).max()
    assert np.array_equal(x[kk], c[kk])


def test_zero_columns_removed_and_levels_spd(disc):
    V, F, A, m, Ps = disc
    n = A.shape[0]
    known = np.random.default_rng(72).uniform(size=n) < 0.6    # 3 coarse vertices lose all weight
    Pr = DR.prolongations(Ps, known)
    u = np.flatnonzero(~known)
    assert Pr[0].shape[0] == len(u) and Pr[0].shape[1] < Ps[0].shape[1]   # columns were removed
    Al = DR.reduce(A, np.zeros((n, 1)), known, np.zeros((n, 1)))[0]
    for P in Pr:
        assert np.asarray(P.max(axis=0).todense()).min() > 0
        Al = H.galerkin(Al, P)
        np.linalg.cholesky(Al.toarray())


def test_multigrid_on_the_reduced_system(disc):
    V, F, A, m, Ps = disc
    n = A.shape[0]
    rng = np.random.default_rng(73)
    known = np.zeros(n, bool)
    known[np.argsort(np.linalg.norm(V[:, :2], axis=1))[-n // 8:]] = True   # the outer rim
    b = m[:, None] * rng.uniform(-1, 1, (n, 3))
    c = np.zeros((n, 3))
    c[known] = 1.0
    Auu, rhs, u = DR.reduce(A, b, known, c)
    S = VC.Solver(DR.prolongations(Ps, known), Auu)
    xu, cyc, _ = S.solve(rhs, 1e-12)
    xs = np.linalg.solve(Auu.toarray(), rhs)
    assert np.abs(xu - xs).max() < 1e-10 * np.abs(xs).max()
    x = DR.expand(xu, c, known)
    assert np.abs((A @ x - b)[u]).max() < 1e-10 * np.abs(b).max() + 1e-12
