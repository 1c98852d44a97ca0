"""ORACLE (test infrastructure only): conjugate gradients preconditioned by
one multigrid V-cycle, the solver combination the paper proposes as future
work (Sec. "Limitations & Future Work").

Textbook preconditioned CG (Hestenes-Stiefel recurrences), one independent
run per right-hand-side column, in FP64:

  x = 0, r = b, z = B r, p = z
  repeat until ||r_c|| / ||b_c|| <= eps for every column c:
      q = A p
      alpha = (r . z) / (p . q)
      x = x + alpha p
      r = r - alpha q
      z = B r
      beta = (r . z)_new / (r . z)_old
      p = z + beta p

Readings (not fixed by the paper):
  * B is one V-cycle from x = 0 with the post-relaxation in descending color
    order (the adjoint of the pre-relaxation), mu_pre = mu_post, so that B is
    symmetric positive definite as CG requires;
  * the stop test uses the recurrence residual r, tested after each update
    (and once before the first iteration), as the V-cycle solve tests its
    residual before every cycle;
  * a column whose p . q or r . z is exactly zero takes alpha = 0 or
    beta = 0 (it has converged exactly); all columns iterate until the
    worst one meets the tolerance.
"""
import numpy as np


def _cdot(u, v):
    return np.einsum("ij,ij->j", u, v)


def pcg(A, b, precond, rtol, max_iters=200, fixed_iters=None):
    """Returns (x, iterations, per-column relative residual history).
    precond(r) applies B to an n x k array."""
    b = np.asarray(b, dtype=np.float64)
    if b.ndim == 1:
        b = b[:, None]
    x = np.zeros_like(b)
    r = b.copy()
    bn = np.linalg.norm(b, axis=0)
    scale = np.where(bn > 0, bn, 1.0)
    z = precond(r)
    p = z.copy()
    rz = _cdot(r, z)
    hist = [np.linalg.norm(r, axis=0) / scale]
    it = 0
    while True:
        if fixed_iters is not None:
            if it == fixed_iters:
                break
        elif hist[-1].max() <= rtol or it >= max_iters:
            break
        q = A @ p
        pq = _cdot(p, q)
        alpha = np.divide(rz, pq, out=np.zeros_like(rz), where=pq != 0)
        x = x + alpha * p
        r = r - alpha * q
        it += 1
        hist.append(np.linalg.norm(r, axis=0) / scale)
        z = precond(r)
        rz_new = _cdot(r, z)
        beta = np.divide(rz_new, rz, out=np.zeros_like(rz), where=rz != 0)
        p = z + beta * p
        rz = rz_new
    return x, it, np.array(hist)


def vcycle_preconditioner(solver):
    """B r = one symmetric V-cycle from zero (oracle.vcycle.Solver)."""
    def apply(r):
        return solver.vcycle(0, np.zeros_like(r), r, symmetric=True)
    return apply
