"""Pins of the oracle's V-cycle-preconditioned conjugate gradients (the
paper's future-work combination, Sec. "Limitations & Future Work"): the
symmetric cycle is a symmetric positive definite operator, and PCG's
iterates are the A-norm-optimal points of the preconditioned Krylov spaces,
computed here by dense projection (no CG recurrence involved)."""
import numpy as np
import pytest

import synth
from oracle import assemble as AS, hierarchy as H, vcycle as VC, pcg as PCG


@pytest.fixture(scope="module")
def ico3():
    V, F = synth.small_icosphere(3, seed=21, sigma=0.02)
    A, L, m = AS.system(V, F, 1e-2)
    Ps, _, _ = H.prolongations(V, F, n_levels=3)
    S = VC.Solver(Ps, A)
    n = A.shape[0]
    eye = np.eye(n)
    Bsym = S.vcycle(0, np.zeros((n, n)), eye.copy(), symmetric=True)
    Bns = S.vcycle(0, np.zeros((n, n)), eye.copy(), symmetric=False)
    return A, m, S, Bsym, Bns


def test_symmetric_cycle_is_spd(ico3):
    A, m, S, Bsym, Bns = ico3
    nb = np.linalg.norm(Bsym)
    assert np.linalg.norm(Bsym - Bsym.T) / nb < 1e-13
    assert np.linalg.eigvalsh(0.5 * (Bsym + Bsym.T)).min() > 0
    # ascending post-relaxation is not symmetric: the pin can tell them apart
    assert np.linalg.norm(Bns - Bns.T) / np.linalg.norm(Bns) > 1e-4


def _krylov_optimum(A, B, b, m):
    """argmin over span{Bb, (BA)Bb, ...} (m vectors) of the A-norm error,
    by an orthonormal basis (modified Gram-Schmidt) and a dense projection."""
    Ad = A.toarray()
    W = []
    w = B @ b
    for _ in range(m):
        for u in W:
            w = w - (u @ w) * u
        w = w / np.linalg.norm(w)
        W.append(w)
        w = B @ (Ad @ w)
    W = np.array(W).T
    y = np.linalg.solve(W.T @ Ad @ W, W.T @ b)
    return W @ y


@pytest.mark.parametrize("which", ["vcycle", "identity"])
def test_pcg_iterates_are_krylov_optimal(ico3, which):
    A, m, S, Bsym, Bns = ico3
    n = A.shape[0]
    B = Bsym if which == "vcycle" else np.eye(n)
    rng = np.random.default_rng(3)
    b = m * rng.uniform(-1, 1, n)
    for it in (1, 2, 3, 4):
        x, its, _ = PCG.pcg(A, b, lambda r: B @ r, 0.0, fixed_iters=it)
        xo = _krylov_optimum(A, B, b, it)
        assert its == it
        assert np.linalg.norm(x[:, 0] - xo) / np.linalg.norm(xo) < 1e-8, (which, it)


def test_pcg_with_exact_inverse_takes_one_iteration(ico3):
    A, m, S, Bsym, Bns = ico3
    Ainv = np.linalg.inv(A.toarray())
    b = np.random.default_rng(4).uniform(-1, 1, (A.shape[0], 2))
    x, its, hist = PCG.pcg(A, b, lambda r: Ainv @ r, 1e-12)
    assert its == 1
    assert np.abs(x - Ainv @ b).max() < 1e-12 * np.abs(Ainv @ b).max()


def test_pcg_converges_to_dense_solution_faster_than_cycles(ico3):
    A, m, S, Bsym, Bns = ico3
    rng = np.random.default_rng(5)
    b = m[:, None] * rng.uniform(-1, 1, (A.shape[0], 3))
    xs = np.linalg.solve(A.toarray(), b)
    x, its, hist = PCG.pcg(A, b, PCG.vcycle_preconditioner(S), 1e-12)
    assert np.abs(x - xs).max() < 1e-10 * np.abs(xs).max()
    true_res = np.linalg.norm(b - A @ x, axis=0) / np.linalg.norm(b, axis=0)
    assert true_res.max() < 1e-11
    _, cycles, _ = S.solve(b, 1e-12)
    assert its < cycles


def test_columns_are_independent_runs(ico3):
    """PCG on several right-hand sides at once runs one CG per column: each
    column's iterate equals a run on that column alone."""
    A, m, S, Bsym, Bns = ico3
    rng = np.random.default_rng(6)
    b = m[:, None] * rng.uniform(-1, 1, (A.shape[0], 3))
    b[:, 2] *= 1e-3                                    # different scales, same directions
    X, _, _ = PCG.pcg(A, b, lambda r: Bsym @ r, 0.0, fixed_iters=5)
    for c in range(3):
        x1, _, _ = PCG.pcg(A, b[:, c], lambda r: Bsym @ r, 0.0, fixed_iters=5)
        assert np.abs(X[:, c] - x1[:, 0]).max() <= 1e-14 * np.abs(x1).max()
