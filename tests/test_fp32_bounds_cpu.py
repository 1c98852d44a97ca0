"""The FP32 error bounds used by the GPU FP32 parity tests, checked on the
CPU: an FP32 emulation of every step (numpy float32 arithmetic, another
summation order than the GPU's) must stay inside them, the bounds must be
small enough to mean something, and a plausible mistake must break them."""
import numpy as np
import pytest
import scipy.sparse as sp

import fp32_bounds as FB
from helpers import Problem

F32 = np.float32


def _gs32(A, colors, ncolors, x, b, plant=None):
    A32 = A.astype(F32).tocsr()
    d = A32.diagonal()
    off = A32.copy()
    off.setdiag(0.0)
    off.eliminate_zeros()
    if plant == "drop":           # planted mistake: each row's first off-diagonal entry ignored
        first = off.indptr[:-1][np.diff(off.indptr) > 0]
        off.data[first] = 0.0
    x = x.astype(F32).copy()
    b = b.astype(F32)
    for c in range(ncolors - (1 if plant == "skip" else 0)):   # "skip": last color left out
        rows = np.flatnonzero(colors == c)
        x[rows] = (b[rows] - off[rows] @ x) / d[rows, None]
    return x


def _vcycle32(O, l, x, b, plant=None):
    if l == O.nlev - 1:
        Ainv = np.linalg.inv(O.A[l].toarray())
        return (Ainv @ b.astype(np.float64)).astype(F32)
    lv = O.levels[l]
    A = O.A[l]
    for _ in range(O.mu_pre):
        x = _gs32(A, lv.colors, lv.ncolors, x, b, plant if l == 0 else None)
    r = b - A.astype(F32) @ x
    P32 = O.P[l].astype(F32).tocsr()
    if plant == "p3" and l == 0:   # planted mistake: third prolongation weight left out
        full = np.flatnonzero(np.diff(P32.indptr) == 3)
        P32.data[P32.indptr[full] + 2] = 0.0
    rc = (P32.T @ r).astype(F32)
    c = _vcycle32(O, l + 1, np.zeros_like(rc), rc)
    x = x + P32 @ c
    for _ in range(O.mu_post):
        x = _gs32(A, lv.colors, lv.ncolors, x, b)
    return x


@pytest.fixture(scope="module", params=["disc-41x37", "icosphere-L5"])
def prob(request):
    return Problem(request.param)


def test_steps_inside_bounds(prob):
    O = prob.oracle
    rng = np.random.default_rng(0)
    for l in range(O.nlev - 1):
        n = prob.sizes[l]
        A = O.A[l]
        b = rng.uniform(-1, 1, (n, 3)).astype(F32).astype(np.float64)
        x = rng.uniform(-1, 1, (n, 3)).astype(F32).astype(np.float64)
        r, e = FB.residual_bound(A, x, b)
        r32 = b.astype(F32) - A.astype(F32) @ x.astype(F32)
        assert (np.abs(r32 - r) <= e).all()
        assert (e / (np.abs(b) + abs(A) @ np.abs(x))).max() < 60 * FB.U
        lv = O.levels[l]
        z = np.zeros_like(x)
        xs, es = FB.gs_sweep_bound(A, lv.colors, lv.ncolors, x, b, z, z)
        x32 = _gs32(A, lv.colors, lv.ncolors, x, b)
        assert (np.abs(x32 - xs) <= es).all()


def test_vcycle_inside_bound_and_mistakes_outside(prob):
    """The propagated bound holds for an FP32 cycle and is ~1e-4 of the
    iterate; a dropped entry per row, a skipped color or a dropped
    prolongation weight on level 0 each exceeds twice the bound by 100x+."""
    O = prob.oracle
    rng = np.random.default_rng(1)
    n = prob.sizes[0]
    b = rng.uniform(-1, 1, (n, 2)).astype(F32).astype(np.float64)
    z = np.zeros_like(b)
    x64, e = FB.vcycle_bound(O, 0, z, z, b, z)
    x32 = _vcycle32(O, 0, z.astype(F32), b.astype(F32))
    assert (np.abs(x32 - x64) <= 2 * e).all()
    assert (e / np.abs(x64).max()).max() < 1e-3
    for plant in ("drop", "skip", "p3"):
        bad = _vcycle32(O, 0, z.astype(F32), b.astype(F32), plant)
        assert (np.abs(bad - x64) / (2 * e)).max() > 100, plant
