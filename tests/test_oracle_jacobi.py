"""Pins of the oracle's damped Jacobi relaxation (the alternative smoother
of App. "Ablation Study"): the exact solution is a fixed point, on a
diagonal system a sweep scales the error by exactly 1 - omega, the V-cycle
built on it is a symmetric positive definite operator (no color order to
reverse), and the solve converges to the dense solution."""
import numpy as np
import pytest

import synth
from oracle import assemble as AS, hierarchy as H, vcycle as VC, pcg as PCG


@pytest.fixture(scope="module")
def ico3():
    V, F = synth.small_icosphere(3, seed=21, sigma=0.02)
    A, L, m = AS.system(V, F, 1e-2)
    Ps, _, _ = H.prolongations(V, F, n_levels=3)
    return V, F, A, L, m, Ps


def test_exact_solution_is_a_fixed_point(ico3):
    V, F, A, L, m, Ps = ico3
    S = VC.Solver(Ps, A, smoother="jacobi")
    rng = np.random.default_rng(6)
    b = rng.uniform(-1, 1, (A.shape[0], 2))
    xs = np.linalg.solve(A.toarray(), b)
    for l in (0,):
        x = S.relax(l, xs.copy(), b, 3)
        assert np.abs(x - xs).max() < 1e-12 * np.abs(xs).max()
    # and a sweep changes any other iterate
    x0 = xs + 1e-3 * rng.uniform(-1, 1, xs.shape)
    assert np.abs(S.relax(0, x0.copy(), b, 1) - x0).max() > 1e-6


def test_diagonal_system_error_factor(ico3):
    V, F, A, L, m, Ps = ico3
    M = AS.system(V, F, 0.0)[0]            # t = 0: A = M, diagonal
    assert abs(M - M.multiply(np.eye(M.shape[0]) != 0)).max() == 0
    rng = np.random.default_rng(7)
    b = rng.uniform(-1, 1, (M.shape[0], 1))
    xs = b / M.diagonal()[:, None]
    x0 = rng.uniform(-1, 1, b.shape)
    for om in (1.0, 0.5, 2.0 / 3.0):
        S = VC.Solver([], M, smoother="jacobi", omega=om)   # one level: relax it directly
        x1 = S.relax(0, x0.copy(), b, 1)
        assert np.abs((x1 - xs) - (1 - om) * (x0 - xs)).max() < 1e-13 * np.abs(xs).max()


def test_jacobi_cycle_is_spd_and_converges(ico3):
    V, F, A, L, m, Ps = ico3
    S = VC.Solver(Ps, A, smoother="jacobi")
    n = A.shape[0]
    B = S.vcycle(0, np.zeros((n, n)), np.eye(n))
    assert np.linalg.norm(B - B.T) / np.linalg.norm(B) < 1e-13
    assert np.linalg.eigvalsh(0.5 * (B + B.T)).min() > 0
    b = m[:, None] * np.random.default_rng(8).uniform(-1, 1, (n, 2))
    xs = np.linalg.solve(A.toarray(), b)
    x, cyc, hist = S.solve(b, 1e-12, max_cycles=300)
    assert np.abs(x - xs).max() < 1e-10 * np.abs(xs).max()
    assert np.all(np.diff(hist.max(axis=1)) < 0)       # residual falls every cycle
    xp, its, _ = PCG.pcg(A, b, lambda r: S.vcycle(0, np.zeros_like(r), r), 1e-12)
    assert np.abs(xp - xs).max() < 1e-10 * np.abs(xs).max() and its < cyc


def test_lambda_estimate_and_level_factors(ico3):
    """The power-step estimate of lambda_max(D^{-1} A) is a Rayleigh quotient
    (never above the largest eigenvalue, computed densely here) and within 10%
    of it on every level (the factor 2 / (1 + lambda) keeps omega lambda < 2
    for any estimate above lambda - 1); a diagonal matrix gives exactly 1."""
    V, F, A, L, m, Ps = ico3
    S = VC.Solver(Ps, A, smoother="jacobi")
    for l, Al in enumerate(S.A[:-1]):
        d = Al.diagonal()
        Ad = Al.toarray() / np.sqrt(np.outer(d, d))
        lam = np.linalg.eigvalsh(Ad).max()
        est = VC.jacobi_lambda(Al)
        assert est <= lam * (1 + 1e-12) and est >= 0.9 * lam, (l, est, lam)
        assert abs(S.omegas[l] - 2.0 / (1.0 + est)) < 1e-15
    M = AS.system(V, F, 0.0)[0]
    assert VC.jacobi_lambda(M) == 1.0
    assert VC.Solver([], M, smoother="jacobi").omegas == [1.0]
    assert VC.Solver(Ps, A, smoother="jacobi", omega=0.7).omegas == [0.7] * (len(Ps) + 1)
