"""ORACLE (test infrastructure only): Dirichlet conditions by reduction to
the unknowns (App. "Dirichlet Boundary Conditions").

  A_uu x_u = b_u - A_uk x_k                     (the reduced system)
  P_{u:} = rows of P_0 of the unknowns          (the finest transfer)
  columns of P_{u:} whose largest weight is 0 are removed with the matching
  rows of the next prolongation (hierarchy.remove_zero_columns, level by
  level); coarser prolongations are otherwise unchanged.
"""
import numpy as np

from . import hierarchy as H


def reduce(A, b, known, xk):
    """(A_uu, b_u - A_uk x_k, unknown indices); b and xk are n x k (the known
    rows of xk are the prescribed values)."""
    known = np.asarray(known, dtype=bool)
    u = np.flatnonzero(~known)
    kk = np.flatnonzero(known)
    A = A.tocsr()
    Au = A[u]
    Auu = Au[:, u].tocsr()
    Auk = Au[:, kk].tocsr()
    b = np.asarray(b, dtype=np.float64).reshape(A.shape[0], -1)
    xk = np.asarray(xk, dtype=np.float64).reshape(A.shape[0], -1)
    return Auu, b[u] - Auk @ xk[kk], u


def prolongations(Ps, known):
    """The reduced system's prolongations: P_{u:} then the rest, zero columns
    removed."""
    if not Ps:
        return []
    u = np.flatnonzero(~np.asarray(known, dtype=bool))
    return H.remove_zero_columns([Ps[0].tocsr()[u]] + [P.tocsr() for P in Ps[1:]])


def expand(xu, xk, known):
    """Full vector from the unknowns' solution and the prescribed values."""
    x = np.array(xk, dtype=np.float64).reshape(len(known), -1)
    x[np.flatnonzero(~np.asarray(known, dtype=bool))] = np.asarray(xu).reshape(-1, x.shape[1])
    return x
