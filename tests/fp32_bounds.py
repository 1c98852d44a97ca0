"""Rounding-error bounds for the FP32 kernels of the inner cycles.

Each FP32 step takes FP32 inputs (FP64 values that are exactly representable
in FP32), the FP32 copy of its matrix (every entry rounded once, relative
error at most u = 2^-24), accumulates in FP32 in some order, and rounds its
result to FP32.  For a sum of N terms in any order the computed value is
within gamma_{N-1} sum |terms| (gamma_N = N u / (1 - N u)) of the exact sum,
and a product or quotient adds one rounding each.  So, first order in u and
elementwise, with m_i the stored entries of row i (diagonal included):

  residual      r_i = b_i - sum_j a_ij x_j
                |r32_i - r_i| <= (m_i + 4) u (|b_i| + sum_j |a_ij| |x_j|)
  Gauss-Seidel  x_i = (b_i - sum_{j != i} a_ij x_j) / a_ii
                |x32_i - x_i| <= (m_i + 4) u (|b_i| + sum_{j != i} |a_ij| |x_j|) / |a_ii| + 3 u |x_i|
  restriction   rc_c = sum_j P_jc r_j over the m_c entries of column c
                |rc32_c - rc_c| <= (m_c + 3) u sum_j P_jc |r_j|
  prolongation  x_i + sum_c P_ic e_c (at most three terms)
                <= 6 u (|x_i| + sum_c P_ic |e_c|)
  coarsest      x = A_H^{-1} b accumulated in FP64, rounded to FP32
                <= u |x_i| + 1e-13 sum_j |A_H^{-1}|_ij |b_j|

where x, b, r on the right are the exact (FP64) values.  Through a whole
cycle the bounds are carried as vectors: a step that reads inputs with error
bounds e applies the absolute value of its linear map to e and adds its own
local bound (running error analysis, first order).  The tests allow twice
the bound for second-order terms.
"""
import numpy as np
import scipy.sparse as sp

U = 2.0 ** -24


def _absm(M):
    M = M.tocsr().copy()
    M.data = np.abs(M.data)
    return M


def row_counts(A):
    return np.diff(A.tocsr().indptr).astype(np.float64)


def residual_bound(A, x, b, ex=None, eb=None):
    """r = b - A x and its FP32 error bound (ex, eb: input error bounds)."""
    Aa = _absm(A)
    m = row_counts(A)[:, None]
    r = b - A @ x
    e = (m + 4) * U * (np.abs(b) + Aa @ np.abs(x))
    if ex is not None:
        e = e + Aa @ ex
    if eb is not None:
        e = e + eb
    return r, e


def gs_sweep_bound(A, colors, ncolors, x, b, ex, eb, descending=False):
    """One multicolor Gauss-Seidel sweep (colors ascending, or descending)
    applied to (x, ex) with right-hand side (b, eb); returns the exact FP64
    sweep and the propagated FP32 bound."""
    A = A.tocsr()
    d = A.diagonal()
    off = A.copy()
    off.setdiag(0.0)
    off.eliminate_zeros()
    offa = _absm(off)
    m = row_counts(A)[:, None]
    x = x.copy()
    ex = ex.copy()
    order = range(ncolors - 1, -1, -1) if descending else range(ncolors)
    for c in order:
        rows = np.flatnonzero(colors == c)
        Oc, Oa = off[rows], offa[rows]
        s_abs = np.abs(b[rows]) + Oa @ np.abs(x)
        xn = (b[rows] - Oc @ x) / d[rows, None]
        en = (eb[rows] + Oa @ ex + (m[rows] + 4) * U * s_abs) / np.abs(d[rows, None]) + 3 * U * np.abs(xn)
        x[rows] = xn
        ex[rows] = en
    return x, ex


def vcycle_bound(O, l, x, ex, b, eb, symmetric=False):
    """The oracle's V-cycle from level l (its operators, coloring and color
    order) carried together with the FP32 error bound of every step."""
    if l == O.nlev - 1:
        Ainv = np.linalg.inv(O.A[l].toarray())
        xc = O.coarse_solve(b)
        e = np.abs(Ainv) @ eb + U * np.abs(xc) + 1e-13 * (np.abs(Ainv) @ np.abs(b))
        return xc, e
    lv = O.levels[l]
    A = O.A[l]
    for _ in range(O.mu_pre):
        x, ex = gs_sweep_bound(A, lv.colors, lv.ncolors, x, b, ex, eb)
    r, er = residual_bound(A, x, b, ex, eb)
    P = O.P[l]
    mc = row_counts(P.T.tocsr())[:, None]
    rc = P.T @ r
    erc = P.T @ er + (mc + 3) * U * (P.T @ np.abs(r))
    c, ec = vcycle_bound(O, l + 1, np.zeros_like(rc), np.zeros_like(rc), rc, erc, symmetric)
    pc = P @ c
    ex = ex + P @ ec + 6 * U * (np.abs(x) + P @ np.abs(c))
    x = x + pc
    for _ in range(O.mu_post):
        x, ex = gs_sweep_bound(A, lv.colors, lv.ncolors, x, b, ex, eb, descending=symmetric)
    return x, ex
