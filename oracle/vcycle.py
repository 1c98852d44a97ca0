"""ORACLE (test infrastructure only): Galerkin multigrid V-cycle in FP64.

Follows Alg. "V-cycle" and Alg. "Galerkin Surface Multigrid Solver" (Sec. 5):

  Vcycle(l, x, b):
    l == H (coarsest): solve A_H x = b directly (dense Cholesky, FP64)
    otherwise:
      x' = relax(A_l, x, b, mu_pre)                 pre-relaxation
      r  = P_l^T (b - A_l x')                       restrict residual
      c  = Vcycle(l + 1, 0, r)                      coarse-grid correction
      x  = x' + P_l c                               prolong and update
      x  = relax(A_l, x, b, mu_post)                post-relaxation

  Solve: x = 0; while max_c ||b_c - A x_c|| / ||b_c|| > eps: x = Vcycle(0, x, b)

Readings (the paper is silent or inconsistent):
  * damped Jacobi (named as an alternative in App. "Ablation Study", no
    factor given) uses per level omega_l = 2 / (1 + lambda_l), lambda_l an
    estimate of the largest eigenvalue of D_l^{-1} A_l (power steps, see
    jacobi_lambda), unless one factor is set.  A single factor is not
    robust: on a jittered 200x80 torus lambda is 2.8 on levels 0-1 and 1.9
    below, 2/3 needed 39 cycles, 0.75 diverged, while the per-level rule
    needs 43 (and omega_l lambda_l < 2 even for estimates well below
    lambda_l);
  * the correction is added to the pre-relaxed iterate x' (the update line of
    the listing names the un-relaxed iterate; the residual was taken at x');
  * relaxation is multicolor Gauss-Seidel (App. A), colors in ascending
    creation order in both pre- and post-relaxation.  Rows of one color share
    no matrix entry, so updating them together equals updating them one after
    another: the sweep is serial Gauss-Seidel in color-major order;
  * the error measure is the relative residual in the 2-norm per right-hand
    side column, evaluated in FP64 before every cycle; x0 = 0.
"""
import numpy as np
import scipy.linalg as sla

from . import hierarchy as H


class Level:
    def __init__(self, A, colors=None, ncolors=0):
        self.A = A.tocsr()
        self.n = A.shape[0]
        self.diag = self.A.diagonal().copy()
        self.colors = colors
        self.ncolors = ncolors
        self._split()

    def _split(self):
        A = self.A
        off = A.copy()
        off.setdiag(0.0)          # keeps the off-diagonal structure, diag value 0
        self.off = off
        self.rows = []
        self.off_rows = []
        if self.colors is not None:
            for c in range(self.ncolors):
                rows = np.flatnonzero(self.colors == c)
                self.rows.append(rows)
                self.off_rows.append(off[rows])


JACOBI_POWER_STEPS = 20


def power_start(n):
    """Deterministic start vector: v_i = frac(0.6180339887498949 * (i + 1))
    - 1/2 (the golden-ratio sequence), for natural row index i."""
    i = np.arange(1, n + 1, dtype=np.float64)
    return np.mod(0.6180339887498949 * i, 1.0) - 0.5


def jacobi_lambda(A):
    """Estimate of the largest eigenvalue of D^{-1} A: JACOBI_POWER_STEPS
    power steps v <- D^{-1} A v from power_start (no normalization: the
    growth stays far inside FP64 range), then the Rayleigh quotient
    (v . A v) / (v . D v)."""
    d = A.diagonal()
    v = power_start(A.shape[0])
    for _ in range(JACOBI_POWER_STEPS):
        v = (A @ v) / d
    return float((v @ (A @ v)) / (v @ (d * v)))


class Solver:
    """Hierarchy (P_l, coloring) fixed at construction; values via set_values.
    smoother: "gs" (multicolor Gauss-Seidel, the paper's default) or
    "jacobi" (damped Jacobi with factor omega, the alternative App.
    "Ablation Study" names)."""

    def __init__(self, Ps, A0, mu_pre=2, mu_post=2, smoother="gs", omega=0.0):
        """omega > 0: that Jacobi factor on every level; omega <= 0: per
        level 2 / (1 + lambda_l), lambda_l estimated by jacobi_lambda."""
        self.P = [P.tocsr() for P in Ps]
        self.mu_pre, self.mu_post = mu_pre, mu_post
        self.smoother, self.omega = smoother, omega
        self.nlev = len(Ps) + 1
        self.colors = []
        self.set_values(A0, recolor=True)

    def set_values(self, A0, recolor=False):
        As = [A0.tocsr()]
        for P in self.P:
            As.append(H.galerkin(As[-1], P))
        if recolor:
            self.colors = [H.coloring(A) for A in As[:-1]]
        self.levels = [Level(A, *self.colors[l]) for l, A in enumerate(As[:-1])]
        self.levels.append(Level(As[-1]))
        self.omegas = [self.omega if self.omega > 0 else 2.0 / (1.0 + jacobi_lambda(A)) for A in As]
        dense = As[-1].toarray()
        self.G = np.linalg.cholesky(dense)          # lower, A_H = G G^T
        self.A = As

    # --- building blocks -------------------------------------------------
    def relax(self, l, x, b, sweeps, descending=False):
        """Multicolor Gauss-Seidel: for each color in ascending order (or
        descending), every row i of that color becomes
        (b_i - sum_{j != i} A_ij x_j) / A_ii.
        Damped Jacobi: every row at once, x <- x + omega D^{-1} (b - A x)
        (the color order plays no part)."""
        lv = self.levels[l]
        if self.smoother == "jacobi":
            for _ in range(sweeps):
                x = x + self.omegas[l] * (b - self.A[l] @ x) / lv.diag[:, None]
            return x
        order = list(zip(lv.rows, lv.off_rows))
        if descending:
            order = order[::-1]
        for _ in range(sweeps):
            for rows, offr in order:
                x[rows] = (b[rows] - offr @ x) / lv.diag[rows, None]
        return x

    def residual(self, l, x, b):
        return b - self.A[l] @ x

    def restrict(self, l, r):
        return self.P[l].T @ r

    def prolong(self, l, e):
        return self.P[l] @ e

    def coarse_solve(self, b):
        y = sla.solve_triangular(self.G, b, lower=True)
        return sla.solve_triangular(self.G.T, y, lower=False)

    def vcycle(self, l, x, b, symmetric=False):
        """symmetric: post-relaxation visits the colors in descending order,
        the adjoint of the pre-relaxation (with mu_pre == mu_post the cycle
        from x = 0 is then a symmetric operator in b)."""
        if l == self.nlev - 1:
            return self.coarse_solve(b)
        x = self.relax(l, x, b, self.mu_pre)
        r = self.restrict(l, self.residual(l, x, b))
        c = self.vcycle(l + 1, np.zeros_like(r), r, symmetric)
        x = x + self.prolong(l, c)
        return self.relax(l, x, b, self.mu_post, descending=symmetric)

    def solve(self, b, rtol, max_cycles=100, x0=None, fixed_cycles=None):
        """Returns (x, cycles, history of per-column relative residuals)."""
        b = np.asarray(b, dtype=np.float64)
        if b.ndim == 1:
            b = b[:, None]
        x = np.zeros_like(b) if x0 is None else np.array(x0, dtype=np.float64).reshape(b.shape)
        bn = np.linalg.norm(b, axis=0)
        scale = np.where(bn > 0, bn, 1.0)
        hist = []
        cycles = 0
        while True:
            rho = np.linalg.norm(self.residual(0, x, b), axis=0) / scale
            hist.append(rho)
            if fixed_cycles is not None:
                if cycles == fixed_cycles:
                    break
            elif rho.max() <= rtol or cycles >= max_cycles:
                break
            x = self.vcycle(0, x, b)
            cycles += 1
        return x, cycles, np.array(hist)


def build(V, F, A0, n_levels=0, mu_pre=2, mu_post=2, min_coarse=500):
    Ps, meshes, stats = H.prolongations(V, F, n_levels, min_coarse)
    return Solver(Ps, A0, mu_pre, mu_post), meshes, stats
