"""GPU parity: every V-cycle step of libsmg against the oracle, element by
element, on seeded meshes with several slices, ragged tails and boundaries.
Tolerances: FP64 kernels 1e-13 relative (summation-order rounding only);
fixed-cycle solve 1e-8 relative solution error; mixed precision per the
stated bound (oracle FP64 residual <= rtol and 1e-6 relative to x*)."""
import numpy as np
import pytest

from helpers import Problem, gpu_available, rel

pytestmark = pytest.mark.gpu

CASES = ["icosphere-L5", "disc-41x37", "torus-96x40", "heightfield-70x66"]


@pytest.fixture(scope="module", params=CASES)
def prob(request):
    if not gpu_available():
        pytest.skip("no GPU")
    print(f"\n[case] {request.param}", flush=True)
    p = Problem(request.param)
    p.gpu = p.gpu_solver(faces=True)
    return p


def _t(a):
    import torch
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


def _np(t):
    return t.detach().cpu().numpy()


def test_galerkin_coloring_and_factor(prob):
    S, O = prob.gpu, prob.oracle
    assert S.num_levels == O.nlev
    for l in range(O.nlev):
        Ag = S.level_matrix(l)
        Ao = O.A[l]
        assert np.array_equal(Ag.indptr, Ao.indptr) and np.array_equal(Ag.indices, Ao.indices)
        assert rel(Ag.data, Ao.data) < 1e-13, l
        if l < O.nlev - 1:
            col, nc = S.colors(l)
            assert nc == O.colors[l][1] and np.array_equal(col, O.colors[l][0]), l
    G = S.coarse_factor()
    assert rel(G, O.G) < 1e-12


def test_single_steps(prob):
    S, O = prob.gpu, prob.oracle
    rng = np.random.default_rng(0)
    for k in (1, 3):
        for l in range(O.nlev - 1):
            n = prob.sizes[l]
            b = rng.uniform(-1, 1, (n, k))
            x = rng.uniform(-1, 1, (n, k))
            r = S.residual(l, _t(b), _t(x))
            assert rel(_np(r), O.residual(l, x, b)) < 1e-13
            for sweeps in (1, 2):
                xg = S.smooth(l, _t(b), _t(x), sweeps)
                xo = O.relax(l, x.copy(), b, sweeps)
                assert rel(_np(xg), xo) < 1e-13, (l, k, sweeps)
            rc = S.restrict(l, _t(b))
            assert rel(_np(rc), O.restrict(l, b)) < 1e-13
            e = rng.uniform(-1, 1, (prob.sizes[l + 1], k))
            xp = S.prolong_add(l, _t(e), _t(x))
            assert rel(_np(xp), x + O.prolong(l, e)) < 1e-13
        bc = rng.uniform(-1, 1, (prob.sizes[-1], k))
        assert rel(_np(S.coarse_solve(_t(bc))), O.coarse_solve(bc)) < 1e-12


def test_vcycle(prob):
    S, O = prob.gpu, prob.oracle
    rng = np.random.default_rng(1)
    for k in (1, 2, 4):
        n = prob.sizes[0]
        b = rng.uniform(-1, 1, (n, k))
        x0 = rng.uniform(-1, 1, (n, k))
        xg = S.vcycle(_t(b), _t(x0))
        xo = O.vcycle(0, x0.copy(), b)
        assert rel(_np(xg), xo) < 1e-12, k


def test_solve_fp64_matches_oracle(prob):
    S, O = prob.gpu, prob.oracle
    rng = np.random.default_rng(2)
    b = prob.m[:, None] * rng.uniform(-1, 1, (prob.sizes[0], 3))
    rtol = 1e-10
    xo, co, ho = O.solve(b, rtol)
    xg, info = S.solve(_t(b), rtol=rtol, precision="fp64")
    assert info["cycles"] == co
    assert max(info["rel_res"]) <= rtol
    xf, _ = S.solve(_t(b), fixed_cycles=co, precision="fp64")
    assert np.linalg.norm(_np(xf) - xo) / np.linalg.norm(xo) < 1e-8
    assert np.linalg.norm(_np(xf) - xo) / np.linalg.norm(xo) < 1e-12
    res = np.linalg.norm(b - prob.A @ _np(xg), axis=0) / np.linalg.norm(b, axis=0)
    assert res.max() <= rtol * 1.0001


def test_solve_mixed_precision(prob):
    S, O = prob.gpu, prob.oracle
    rng = np.random.default_rng(3)
    b = prob.m[:, None] * rng.uniform(-1, 1, (prob.sizes[0], 2))
    xs, _, _ = O.solve(b, 1e-13, max_cycles=200)
    rtol = 1e-8
    xg, info = S.solve(_t(b), rtol=rtol, precision="fp32ir")
    xg = _np(xg)
    res = np.linalg.norm(b - prob.A @ xg, axis=0) / np.linalg.norm(b, axis=0)
    assert res.max() <= rtol * 1.0001
    err = np.linalg.norm(xg - xs) / np.linalg.norm(xs)
    print(f"[mixed] {prob.name}: cycles={info['cycles']} res={res.max():.2e} err_vs_xstar={err:.2e}")
    assert err < 1e-6


def test_refinement_run_ahead_is_exact(prob):
    """The mixed-precision solve queues each next cycle's first part before
    its stop test; the iterate returned is still that of the reported cycle
    count (bitwise equal to a fixed-count solve, which runs no stop test), and
    a cycle cap stops it with exactly the capped count."""
    S = prob.gpu
    rng = np.random.default_rng(5)
    b = _t(prob.m[:, None] * rng.uniform(-1, 1, (prob.sizes[0], 3)))
    x1, i1 = S.solve(b, rtol=1e-9, precision="fp32ir")
    x2, i2 = S.solve(b, fixed_cycles=i1["cycles"], precision="fp32ir")
    assert np.array_equal(_np(x1), _np(x2))
    assert i2["rel_res"] == i1["rel_res"]
    cap = i1["cycles"] - 1
    x3, i3 = S.solve(b, rtol=1e-9, max_cycles=cap, precision="fp32ir", raise_on_error=False)
    x4, _ = S.solve(b, fixed_cycles=cap, precision="fp32ir")
    assert i3["status"] != 0 and i3["cycles"] == cap
    assert np.array_equal(_np(x3), _np(x4))


def test_graph_replay_and_determinism(prob):
    S = prob.gpu
    rng = np.random.default_rng(4)
    b = _t(prob.m[:, None] * rng.uniform(-1, 1, (prob.sizes[0], 3)))
    for precision in ("fp64", "fp32ir"):
        x1, i1 = S.solve(b, rtol=1e-9, precision=precision)
        x2, i2 = S.solve(b, rtol=1e-9, precision=precision, use_graph=True)
        x3, i3 = S.solve(b, rtol=1e-9, precision=precision, use_graph=True)
        x4, i4 = S.solve(b, rtol=1e-9, precision=precision)
        assert i1["cycles"] == i2["cycles"] == i3["cycles"] == i4["cycles"]
        a1 = _np(x1)
        for other in (x2, x3, x4):
            assert np.array_equal(a1, _np(other)), precision


def test_assembly_parity(prob):
    import torch
    from oracle import assemble as AS
    S = prob.gpu
    rng = np.random.default_rng(5)
    n = prob.sizes[0]
    E = AS.edge_list(prob.F)
    s = rng.uniform(0.5, 1.5, n)
    w = rng.uniform(0.5, 2.0, len(E)).astype(np.float32)
    A, L, m = AS.system(prob.V, prob.F, 0.03, mass_scale=s, edge_weights=w.astype(np.float64), edges=E)
    a, lv, mm = S.assemble(_t(prob.V), 0.03, mass_scale=_t(s),
                           edge_w=torch.tensor(w, device="cuda"), want_l=True, want_mass=True)
    assert rel(_np(a), A.data) < 1e-13
    assert rel(_np(lv), L.data) < 1e-13
    assert rel(_np(mm), m) < 1e-14
    a0, _, _ = S.assemble(_t(prob.V), prob.t)
    assert rel(_np(a0), prob.A.data) < 1e-13


@pytest.mark.parametrize("shape", [dict(tail_rows=-1, lanes_per_row=[1, 1, 1, 1, 1]),
                                   dict(tail_rows=-1, lanes_per_row=[2, 2, 2, 2, 2]),
                                   dict(tail_rows=-1, lanes_per_row=[1, 4, 8, 4, 2]),
                                   dict(tail_rows=500, lanes_per_row=[8, 8, 8, 8, 8]),
                                   dict(tail_rows=0)],
                         ids=["untailed-l1", "untailed-l2", "untailed-mixed", "tail500-l8", "default"])
def test_launch_shapes(shape):
    """Launch shape (single-workgroup tail, lanes per row) changes nothing but
    summation order: every shape matches the oracle V-cycle and solve."""
    if not gpu_available():
        pytest.skip("no GPU")
    p = _shape_problem()
    S = p.gpu_solver(**shape)
    O = p.oracle
    rng = np.random.default_rng(9)
    n = p.sizes[0]
    for k in (1, 3):
        b = rng.uniform(-1, 1, (n, k))
        x0 = rng.uniform(-1, 1, (n, k))
        assert rel(_np(S.vcycle(_t(b), _t(x0))), O.vcycle(0, x0.copy(), b)) < 1e-12
        for l in range(O.nlev - 1):
            bl = rng.uniform(-1, 1, (p.sizes[l], k))
            xl = rng.uniform(-1, 1, (p.sizes[l], k))
            assert rel(_np(S.smooth(l, _t(bl), _t(xl), 2)), O.relax(l, xl.copy(), bl, 2)) < 1e-13
            assert rel(_np(S.residual(l, _t(bl), _t(xl))), O.residual(l, xl, bl)) < 1e-13
    b = p.m[:, None] * rng.uniform(-1, 1, (n, 2))
    xo, co, _ = O.solve(b, 1e-10)
    for prec, tol in (("fp64", 1e-12), ("fp32ir", 1e-6)):
        xg, info = S.solve(_t(b), rtol=1e-10, precision=prec)
        assert max(info["rel_res"]) <= 1e-10
        assert np.linalg.norm(_np(xg) - xo) / np.linalg.norm(xo) < tol


_SHAPE_PROBLEM = []


def _shape_problem():
    if not _SHAPE_PROBLEM:
        _SHAPE_PROBLEM.append(Problem("heightfield-70x66", n_levels=5))
    return _SHAPE_PROBLEM[0]


@pytest.mark.parametrize("levels", [2, 3])
def test_coarsest_factor_many_workgroups(levels):
    """Coarsest levels of 2,561 and 640 rows take the blocked factorization
    over many workgroups (diagonal block, panel solve, trailing update on the
    FP64 matrix cores): factor within 1e-12 of numpy's Cholesky of the
    oracle's A_H, coarsest solve within 1e-12."""
    if not gpu_available():
        pytest.skip("no GPU")
    p = Problem("icosphere-L5", n_levels=levels)
    S = p.gpu_solver()
    O = p.oracle
    assert S.level_size(S.num_levels - 1) == O.A[-1].shape[0] == (2561 if levels == 2 else 640)
    assert rel(S.coarse_factor(), O.G) < 1e-12
    bc = np.random.default_rng(9).uniform(-1, 1, (O.A[-1].shape[0], 2))
    assert rel(_np(S.coarse_solve(_t(bc))), O.coarse_solve(bc)) < 1e-12


@pytest.fixture(scope="module")
def ico_matrix():
    from synth import meshes
    from oracle import assemble as AS
    if not gpu_available():
        pytest.skip("no GPU")
    V, F = meshes.icosphere_subdiv(5)
    A, _, _ = AS.system(V, F, 1e-3)
    return A.tocsr()


@pytest.mark.parametrize("n_h", [97, 100, 127, 128, 129, 161, 300])
def test_coarsest_factor_panel_edges(n_h, ico_matrix):
    """Coarsest sizes around the panel width (32) just above the one-workgroup
    limit (96): full panels, a last panel of 1 or 4 columns, several panels.
    Two levels over the icosphere L5 system with P_ic = 1 for c = i mod n_H
    (full column rank, so A_H = PᵀAP is SPD and dense); the factor and A_H⁻¹ b
    are compared with numpy's Cholesky and solve of the same A_H within
    1e-12."""
    if not gpu_available():
        pytest.skip("no GPU")
    import scipy.sparse as sp
    from helpers import ell3
    from paper_2104_13755_amd.solver import Hierarchy, Solver
    A = ico_matrix
    n0 = A.shape[0]
    P = sp.csr_matrix((np.ones(n0), (np.arange(n0), np.arange(n0) % n_h)), shape=(n0, n_h))
    c, w = ell3(P)
    h = Hierarchy.from_prolongations([n0, n_h], [c], [w])
    S = Solver(h, A.indptr, A.indices)
    S.set_values(_t(A.data))
    AH = (P.T @ A @ P).toarray()
    G = np.linalg.cholesky(AH)
    assert rel(S.coarse_factor(), G) < 1e-12
    bc = np.random.default_rng(n_h).uniform(-1, 1, (n_h, 3))
    assert rel(_np(S.coarse_solve(_t(bc))), np.linalg.solve(AH, bc)) < 1e-12


def test_team_vcycle_matches_launches():
    """The opt-in one-XCD team (smg_opts.team_level: levels >= 1 in one kernel
    whose workgroups meet at L2-local barriers) computes the same cycle as
    the per-color launches: FP64 within 1e-12 of them and of the oracle's
    cycles, FP32 cycles within 1e-7, equal cycle counts to 1e-8."""
    if not gpu_available():
        pytest.skip("no GPU")
    p = Problem("torus-96x40")
    base = p.gpu_solver(tail_rows=-1)
    team = p.gpu_solver(tail_rows=-1, team_level=1, team_size=8)
    rng = np.random.default_rng(12)
    b = p.m[:, None] * rng.uniform(-1, 1, (p.sizes[0], 3))
    xo, _, _ = p.oracle.solve(b, 0.0, fixed_cycles=3)
    for prec, tol in (("fp64", 1e-12), ("fp32ir", 1e-7)):
        x0, _ = base.solve(_t(b), fixed_cycles=3, precision=prec)
        x1, _ = team.solve(_t(b), fixed_cycles=3, precision=prec)
        assert np.linalg.norm(_np(x1) - _np(x0)) / np.linalg.norm(_np(x0)) < tol, prec
        if prec == "fp64":
            assert np.linalg.norm(_np(x1) - xo) / np.linalg.norm(xo) < 1e-12
        _, i0 = base.solve(_t(b), rtol=1e-8, precision=prec)
        _, i1 = team.solve(_t(b), rtol=1e-8, precision=prec)
        assert i0["cycles"] == i1["cycles"] and max(i1["rel_res"]) <= 1e-8, prec
