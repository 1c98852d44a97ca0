"""GPU parity of the FP32 kernels of the inner cycles (mixed precision),
element by element against the FP64 oracle step on FP32-representable
inputs, within the rounding bounds derived in tests/fp32_bounds.py (row
length x 2^-24 x magnitudes).

For k = 1..4 on every smoothed level, through the per-color launch kernels
and through the one-workgroup tail's passes: the residual, one Gauss-Seidel
sweep (each row against its own update from the values the kernel saw:
earlier colors' new values, later colors' old ones), two sweeps, the
restriction, the prolongation and the coarsest solve.  A whole cycle
(FP64, and the FP32 refinement step with its FP64 residual, scaling down and
up) must then equal bit for bit the same cycle chained from those steps, with
and without the tail, so every step inside it is covered by the elementwise
checks.  (A first-order bound carried through a whole FP32 cycle grows far
above the real error on deep hierarchies, which is why the cycle is checked
step by step.)
"""
import numpy as np
import pytest

import fp32_bounds as FB
from helpers import Problem, gpu_available

pytestmark = pytest.mark.gpu

CASES = ["icosphere-L5", "disc-41x37", "torus-96x40", "heightfield-70x66"]
U = FB.U
F32 = np.float32


@pytest.fixture(scope="module", params=CASES)
def prob(request):
    if not gpu_available():
        pytest.skip("no GPU")
    print(f"\n[case] {request.param}", flush=True)
    p = Problem(request.param)
    p.gpu = p.gpu_solver()
    return p


def _t(a):
    import torch
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


def _np(t):
    return t.detach().cpu().numpy()


def _f32(a):
    return np.asarray(a, dtype=F32).astype(np.float64)


def _split(A):
    A = A.tocsr()
    off = A.copy()
    off.setdiag(0.0)
    off.eliminate_zeros()
    offa = off.copy()
    offa.data = np.abs(offa.data)
    return A.diagonal(), off, offa, np.diff(A.indptr).astype(np.float64)[:, None]


@pytest.mark.parametrize("k", [1, 2, 3, 4])
def test_fp32_steps(prob, k):
    S, O = prob.gpu, prob.oracle
    rng = np.random.default_rng(10 + k)
    for l in range(O.nlev - 1):
        n, A = prob.sizes[l], O.A[l]
        b = _f32(rng.uniform(-1, 1, (n, k)))
        x = _f32(rng.uniform(-1, 1, (n, k)))
        # residual
        r, e = FB.residual_bound(A, x, b)
        rg = _np(S.residual(l, _t(b), _t(x), precision="fp32ir"))
        assert np.array_equal(rg, _f32(rg))                       # an FP32 result
        assert (np.abs(rg - r) <= e).all(), (l, k, (np.abs(rg - r) / e).max())
        # one sweep, each row against its own update
        col = O.levels[l].colors
        d, off, offa, m = _split(A)
        xg = _np(S.smooth(l, _t(b), _t(x), 1, precision="fp32ir"))
        for c in range(O.levels[l].ncolors):
            rows = np.flatnonzero(col == c)
            seen = np.where((col < c)[:, None], xg, x)
            ref = (b[rows] - off[rows] @ seen) / d[rows, None]
            bnd = (m[rows] + 4) * U * (np.abs(b[rows]) + offa[rows] @ np.abs(seen)) / np.abs(d[rows, None]) \
                + 3 * U * np.abs(ref)
            assert (np.abs(xg[rows] - ref) <= bnd).all(), (l, k, c)
        # two sweeps against the FP64 oracle, propagated bound
        z = np.zeros_like(x)
        x2, e2 = FB.gs_sweep_bound(A, col, O.levels[l].ncolors, x, b, z, z)
        x2, e2 = FB.gs_sweep_bound(A, col, O.levels[l].ncolors, x2, b, e2, z)
        assert np.abs(x2 - O.relax(l, x.copy(), b, 2)).max() < 1e-12 * np.abs(x2).max()
        xg2 = _np(S.smooth(l, _t(b), _t(x), 2, precision="fp32ir"))
        assert (np.abs(xg2 - x2) <= 2 * e2).all(), (l, k)
        # restriction
        P = O.P[l]
        Pt = P.T.tocsr()
        mc = np.diff(Pt.indptr).astype(np.float64)[:, None]
        rc = O.restrict(l, b)
        rcg = _np(S.restrict(l, _t(b), precision="fp32ir"))
        assert (np.abs(rcg - rc) <= (mc + 3) * U * (Pt @ np.abs(b))).all(), (l, k)
        # prolongation
        ec = _f32(rng.uniform(-1, 1, (prob.sizes[l + 1], k)))
        xp = x + O.prolong(l, ec)
        xpg = _np(S.prolong_add(l, _t(ec), _t(x), precision="fp32ir"))
        assert (np.abs(xpg - xp) <= 6 * U * (np.abs(x) + P @ np.abs(ec))).all(), (l, k)


def _local_bounds_check(O, l, k, rng, steps, tag):
    """The four steps of level l (relax one sweep, residual, restriction,
    prolongation) from `steps` (callables taking FP64 arrays of FP32
    values) against the oracle with the FP32 local bounds."""
    n, A = O.levels[l].n, O.A[l]
    b = _f32(rng.uniform(-1, 1, (n, k)))
    x = _f32(rng.uniform(-1, 1, (n, k)))
    r, e = FB.residual_bound(A, x, b)
    rg = steps["residual"](b, x)
    assert np.array_equal(rg, _f32(rg))
    assert (np.abs(rg - r) <= e).all(), (tag, l, k)
    col = O.levels[l].colors
    d, off, offa, m = _split(A)
    xg = steps["relax"](b, x, 1)
    assert np.array_equal(xg, _f32(xg))
    for c in range(O.levels[l].ncolors):
        rows = np.flatnonzero(col == c)
        seen = np.where((col < c)[:, None], xg, x)
        ref = (b[rows] - off[rows] @ seen) / d[rows, None]
        bnd = (m[rows] + 4) * U * (np.abs(b[rows]) + offa[rows] @ np.abs(seen)) / np.abs(d[rows, None]) \
            + 3 * U * np.abs(ref)
        assert (np.abs(xg[rows] - ref) <= bnd).all(), (tag, l, k, c)
    P = O.P[l]
    Pt = P.T.tocsr()
    mc = np.diff(Pt.indptr).astype(np.float64)[:, None]
    rcg = steps["restrict"](b)
    assert (np.abs(rcg - O.restrict(l, b)) <= (mc + 3) * U * (Pt @ np.abs(b))).all(), (tag, l, k)
    ec = _f32(rng.uniform(-1, 1, (P.shape[1], k)))
    xpg = steps["prolong"](ec, x)
    assert (np.abs(xpg - (x + O.prolong(l, ec))) <= 6 * U * (np.abs(x) + P @ np.abs(ec))).all(), (tag, l, k)


def _tail_steps(S, l, prec):
    return dict(residual=lambda b, x: _np(S.tail_residual(l, _t(b), _t(x), precision=prec)),
                relax=lambda b, x, sw: _np(S.tail_relax(l, _t(b), _t(x), sw, precision=prec)),
                restrict=lambda r: _np(S.tail_restrict(l, _t(r), precision=prec)),
                prolong=lambda e, x: _np(S.tail_prolong(l, _t(e), _t(x), precision=prec)))


@pytest.mark.parametrize("k", [1, 2, 3, 4])
def test_tail_steps(prob, k):
    """Each pass type of the one-workgroup tail on every tail level: FP32
    within the local bounds, FP64 within 1e-13 of the oracle; the coarsest
    solve of the tail in both precisions."""
    S, O = prob.gpu, prob.oracle
    rng = np.random.default_rng(30 + k)
    last = O.nlev - 1
    for prec in ("fp32ir", "fp64"):
        first = S.tail_first(k, prec)
        assert first < last, "the tail covers no smoothed level"
        for l in range(first, last):
            if prec == "fp32ir":
                _local_bounds_check(O, l, k, rng, _tail_steps(S, l, prec), "tail")
                continue
            n = O.levels[l].n
            b, x = rng.uniform(-1, 1, (n, k)), rng.uniform(-1, 1, (n, k))
            rel = lambda a, c: np.abs(a - c).max() / np.abs(c).max()
            assert rel(_np(S.tail_residual(l, _t(b), _t(x))), O.residual(l, x, b)) < 1e-13
            for sw in (1, 2):
                assert rel(_np(S.tail_relax(l, _t(b), _t(x), sw)), O.relax(l, x.copy(), b, sw)) < 1e-13
            assert rel(_np(S.tail_relax(l, _t(b), _t(x), -1)), O.relax(l, x.copy(), b, 1, descending=True)) < 1e-13
            assert rel(_np(S.tail_restrict(l, _t(b))), O.restrict(l, b)) < 1e-13
            e = rng.uniform(-1, 1, (prob.sizes[l + 1], k))
            assert rel(_np(S.tail_prolong(l, _t(e), _t(x))), x + O.prolong(l, e)) < 1e-13
        bc = _f32(rng.uniform(-1, 1, (prob.sizes[-1], k)))
        xc = O.coarse_solve(bc)
        got = _np(S.tail_coarse(_t(bc), precision=prec))
        if prec == "fp64":
            assert np.abs(got - xc).max() < 1e-12 * np.abs(xc).max()
        else:
            Ainv = np.linalg.inv(O.A[last].toarray())
            assert (np.abs(got - xc) <= U * np.abs(xc) + 1e-12 * (np.abs(Ainv) @ np.abs(bc))).all()


def _cycle_by_steps(S, O, l, b, x, prec, first):
    """Alg. "V-cycle" from level l chained from the single-step calls: the
    per-color launches above `first`, the tail's steps from `first` down."""
    last = O.nlev - 1
    if l == last:
        return S.tail_coarse(b, precision=prec) if first < last else S.coarse_solve(b, precision=prec)
    tail = l >= first
    if tail:
        x = S.tail_relax(l, b, x, O.mu_pre, precision=prec)
        bc = S.tail_restrict(l, S.tail_residual(l, b, x, precision=prec), precision=prec)
    else:
        x = S.smooth(l, b, x, O.mu_pre, precision=prec)
        bc = S.restrict(l, S.residual(l, b, x, precision=prec), precision=prec)
    xc = _cycle_by_steps(S, O, l + 1, bc, np_zeros_like(bc), prec, first)
    if tail:
        x = S.tail_prolong(l, xc, x, precision=prec)
        return S.tail_relax(l, b, x, O.mu_post, precision=prec)
    x = S.prolong_add(l, xc, x, precision=prec)
    return S.smooth(l, b, x, O.mu_post, precision=prec)


def np_zeros_like(t):
    import torch
    return torch.zeros_like(t)


@pytest.mark.parametrize("tail", ["tail", "no-tail"])
def test_cycle_equals_its_steps(prob, tail):
    """One cycle of smg_vcycle equals, bit for bit, the same cycle chained
    from the single steps checked above (launch kernels above the tail, the
    tail's steps below it): FP64, and the FP32 refinement step from x = 0,
    whose result is sigma * d with d the FP32 cycle on fp32(b / sigma),
    sigma = max |b| per column (FP64 residual, scaling down and up)."""
    O = prob.oracle
    S = prob.gpu if tail == "tail" else prob.gpu_solver(tail_rows=-1)
    rng = np.random.default_rng(40)
    n = prob.sizes[0]
    for k in (1, 2, 3, 4):
        first = S.tail_first(k, "fp32ir")
        assert (first < O.nlev - 1) == (tail == "tail")
        b = prob.m[:, None] * rng.uniform(-1, 1, (n, k))
        sig = np.abs(b).max(axis=0)
        b32 = _f32(b / sig)
        d = _cycle_by_steps(S, O, 0, _t(b32), _t(np.zeros((n, k))), "fp32ir", first)
        got = _np(S.vcycle(_t(b), _t(np.zeros((n, k))), precision="fp32ir"))
        assert np.array_equal(got, sig * _np(d)), (tail, k)
        first64 = S.tail_first(k, "fp64")
        x0 = rng.uniform(-1, 1, (n, k))
        want = _cycle_by_steps(S, O, 0, _t(b), _t(x0), "fp64", first64)
        got64 = _np(S.vcycle(_t(b), _t(x0), precision="fp64"))
        assert np.array_equal(got64, _np(want)), (tail, k)


def test_refinement_update(prob):
    """From x != 0: x_new = x + sigma d with r the library's FP64 residual,
    sigma = max |r| per column and d the FP32 cycle on fp32(r / sigma), to
    the rounding of the FP64 update."""
    S, O = prob.gpu, prob.oracle
    rng = np.random.default_rng(50)
    n = prob.sizes[0]
    for k in (1, 3):
        b = prob.m[:, None] * rng.uniform(-1, 1, (n, k))
        x = rng.uniform(-1, 1, (n, k)) * 1e-2
        r = _np(S.residual(0, _t(b), _t(x)))
        assert np.abs(r - O.residual(0, x, b)).max() < 1e-13 * np.abs(r).max()
        sig = np.abs(r).max(axis=0)
        d = _np(_cycle_by_steps(S, O, 0, _t(_f32(r / sig)), _t(np.zeros((n, k))), "fp32ir", S.tail_first(k, "fp32ir")))
        got = _np(S.vcycle(_t(b), _t(x), precision="fp32ir"))
        want = x + sig * d
        assert (np.abs(got - want) <= 2.0 ** -52 * (np.abs(want) + np.abs(x))).all(), k
