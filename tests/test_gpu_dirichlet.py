"""GPU parity of Dirichlet conditions (App. "Dirichlet Boundary Conditions")
against the oracle's reduction: the reduced hierarchy (P_{u:}, zero columns
removed) structurally identical with equal weights, the A_uu pattern and
values bitwise equal, b_u - A_uk x_k to 1e-14, and the reduced solves with
the oracle's cycle counts; the expanded solution satisfies A x = b on the
unknowns."""
import numpy as np
import pytest
import scipy.sparse as sp

from helpers import Problem, ell3, gpu_available, rel
from oracle import dirichlet as DR, vcycle as OV

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def disc():
    if not gpu_available():
        pytest.skip("no GPU")
    return Problem("disc-41x37")


def _t(a):
    import torch
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


def _np(t):
    return t.detach().cpu().numpy()


@pytest.mark.parametrize("which", ["rim", "random60"])
def test_dirichlet_reduction_and_solve(disc, which):
    from paper_2104_13755_amd.solver import DirichletSystem, Hierarchy, Solver
    p = disc
    n = p.sizes[0]
    if which == "rim":
        known = np.zeros(n, bool)
        known[np.argsort(np.linalg.norm(p.V[:, :2], axis=1))[-n // 10:]] = True
    else:
        known = np.random.default_rng(81).uniform(size=n) < 0.6
    print(f"\n[dirichlet] {which}: {known.sum()} known of {n}", flush=True)
    ells = [ell3(P) for P in p.Ps]
    h = Hierarchy.from_prolongations(p.sizes, [e[0] for e in ells], [e[1] for e in ells])
    A = p.A.tocsr()
    ds = DirichletSystem(h, A.indptr, A.indices, known)
    rng = np.random.default_rng(82)
    b = p.m[:, None] * rng.uniform(-1, 1, (n, 3))
    c = np.zeros((n, 3))
    c[known] = rng.uniform(-1, 1, (known.sum(), 3))
    Auu, rhs, u = DR.reduce(A, b, known, c)
    Pr = DR.prolongations(p.Ps, known)
    # hierarchy
    assert np.array_equal(ds.unknown, u)
    assert ds.hier.sizes == [len(u)] + [P.shape[1] for P in Pr]
    for l, P in enumerate(Pr):
        cols, w = ds.hier.prolongation(l)
        nn = len(cols)
        msk = w > 0
        Pg = sp.csr_matrix((w[msk], (np.repeat(np.arange(nn), 3).reshape(nn, 3)[msk], cols[msk])), shape=P.shape)
        assert ((Pg != 0) != (P != 0)).nnz == 0, l
        assert abs(Pg - P).max() == 0.0, l
    # reduced system
    assert np.array_equal(ds.u_rowptr, Auu.indptr) and np.array_equal(ds.u_cols, Auu.indices)
    uv, rg = ds.reduce(_t(A.data), _t(c), _t(b))
    assert np.array_equal(_np(uv), Auu.data)
    assert rel(_np(rg), rhs) < 1e-14
    # solves on the reduced system
    S = Solver(ds.hier, ds.u_rowptr, ds.u_cols)
    S.set_values(uv)
    O = OV.Solver(Pr, Auu)
    xo, co, _ = O.solve(rhs, 1e-10)
    xg, info = S.solve(rg, rtol=1e-10, precision="fp64")
    assert info["cycles"] == co
    assert np.linalg.norm(_np(xg) - xo) / np.linalg.norm(xo) < 1e-9
    x = DR.expand(_np(xg), c, known)
    assert np.abs((A @ x - b)[u]).max() <= 1e-9 * np.abs(rhs).max()
    xm, im = S.solve(rg, rtol=1e-8, precision="fp32ir")
    res = np.linalg.norm(rhs - Auu @ _np(xm), axis=0) / np.linalg.norm(rhs, axis=0)
    assert res.max() <= 1e-8 * 1.0001


def test_dirichlet_edges(disc):
    """No known value: the reduced hierarchy is the original one; every value
    known: an error."""
    from paper_2104_13755_amd.solver import DirichletSystem, Hierarchy
    from paper_2104_13755_amd._lib import SmgError
    p = disc
    n = p.sizes[0]
    ells = [ell3(P) for P in p.Ps]
    h = Hierarchy.from_prolongations(p.sizes, [e[0] for e in ells], [e[1] for e in ells])
    A = p.A.tocsr()
    ds = DirichletSystem(h, A.indptr, A.indices, np.zeros(n, bool))
    assert ds.hier.sizes == p.sizes and np.array_equal(ds.unknown, np.arange(n))
    assert np.array_equal(ds.u_rowptr, A.indptr) and np.array_equal(ds.u_cols, A.indices)
    for l in range(len(p.Ps)):
        c0, w0 = h.prolongation(l)
        c1, w1 = ds.hier.prolongation(l)
        assert np.array_equal(c0, c1) and np.array_equal(w0, w1)
    with pytest.raises(SmgError):
        DirichletSystem(h, A.indptr, A.indices, np.ones(n, bool))
