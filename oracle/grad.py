"""ORACLE (test infrastructure only): gradients of a loss through the solve.

For A(t, s) = diag(s * m) + t L and u = A^{-1} b, a loss l(u) with
g = dl/du has, by the adjoint method (A is symmetric),
    lambda = A^{-1} g,   dl/db = lambda,   dl/dt = -lambda^T L u,
    dl/ds_i = -lambda_i m_i u_i.
Both solves use the same V-cycle hierarchy (Alg. "Galerkin Surface Multigrid
Solver"); ``dense_grads`` is the same formula with numpy.linalg.solve.
"""
import numpy as np


def mg_grads(solver, L, m, b, g, rtol, max_cycles=200):
    u, cu, _ = solver.solve(b, rtol, max_cycles)
    lam, cl, _ = solver.solve(g, rtol, max_cycles)
    u = u[:, 0]
    lam = lam[:, 0]
    return dict(u=u, db=lam, dt=-float(lam @ (L @ u)), ds=-lam * m * u, cycles=(cu, cl))


def dense_grads(A, L, m, b, g):
    Ad = A.toarray()
    u = np.linalg.solve(Ad, np.asarray(b).ravel())
    lam = np.linalg.solve(Ad, np.asarray(g).ravel())
    return dict(u=u, db=lam, dt=-float(lam @ (L @ u)), ds=-lam * m * u)
