"""Split Galerkin (App. E): after smg_split_prepare(L, M), smg_split_combine
(a, b) gives the oracle's a P^T L P + b P^T M P on every level (1e-13
relative), the same levels as setting the values a L + b M directly, the same
coarsest factor (1e-12) and identical cycle counts, for several coefficient
pairs, and the errors of the entry points."""
import numpy as np
import scipy.sparse as sp
import pytest

from helpers import Problem, gpu_available, rel

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", params=["icosphere-L5", "torus-96x40"])
def prob(request):
    if not gpu_available():
        pytest.skip("no GPU")
    print(f"\n[case] {request.param}", flush=True)
    p = Problem(request.param)
    A = p.A.tocsr()
    n = A.shape[0]
    rows = np.repeat(np.arange(n), np.diff(A.indptr))
    cols = A.indices
    p.Lv = np.asarray(p.L.tocsr()[rows, cols]).ravel()
    p.Mv = np.where(rows == cols, p.m[rows], 0.0)
    return p


def _t(a):
    import torch
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


def _np(t):
    return t.detach().cpu().numpy()


def test_combine_equals_direct_values(prob):
    from paper_2104_13755_amd._lib import SmgError
    S = prob.gpu_solver()
    with pytest.raises(SmgError):
        S.split_combine(1.0, 1.0)              # nothing prepared
    S.split_prepare(_t(prob.Lv), _t(prob.Mv))
    D = prob.gpu_solver()
    # the oracle's App. E combination: a G_l(L) + c G_l(M), each Galerkin
    # chain formed once on the oracle's side from the same prolongations
    from oracle import hierarchy as OH
    A = prob.A.tocsr()
    GL = [sp.csr_matrix((prob.Lv, A.indices, A.indptr), shape=A.shape)]
    GM = [sp.csr_matrix((prob.Mv, A.indices, A.indptr), shape=A.shape)]
    for P in prob.Ps:
        GL.append(OH.galerkin(GL[-1], P))
        GM.append(OH.galerkin(GM[-1], P))
    rng = np.random.default_rng(61)
    b = prob.m[:, None] * rng.uniform(-1, 1, (prob.sizes[0], 2))
    for a, c in ((prob.t, 1.0), (3 * prob.t, 1.0), (0.1, 2.0)):
        S.split_combine(a, c)
        D.set_values(_t(a * prob.Lv + c * prob.Mv))
        for l in range(S.num_levels):
            As, Ad = S.level_matrix(l), D.level_matrix(l)
            assert np.array_equal(As.indices, Ad.indices)
            assert rel(As.data, Ad.data) < 1e-13, (a, c, l)
            assert np.array_equal(As.indptr, GL[l].indptr) and np.array_equal(As.indices, GL[l].indices)
            assert rel(As.data, a * GL[l].data + c * GM[l].data) < 1e-13, (a, c, l)
        assert rel(S.coarse_factor(), D.coarse_factor()) < 1e-12
        xs, i_s = S.solve(_t(b), rtol=1e-9, precision="fp32ir")
        xd, i_d = D.solve(_t(b), rtol=1e-9, precision="fp32ir")
        assert i_s["cycles"] == i_d["cycles"]
        assert np.linalg.norm(_np(xs) - _np(xd)) / np.linalg.norm(_np(xd)) < 1e-9
    with pytest.raises(SmgError):
        S.split_combine(float("nan"), 1.0)


def test_bilaplacian_smoothing_levels():
    """Data smoothing with the squared Laplacian energy (Sec. Applications):
    A(alpha) = alpha L M^{-1} L + (1 - alpha) M on the 2-ring pattern, levels
    by split_combine; the solve matches the oracle's V-cycle solve of the same
    matrix (cycle counts equal) and PCG reaches the tolerance."""
    if not gpu_available():
        pytest.skip("no GPU")
    import synth
    from oracle import assemble as AS, hierarchy as OH, vcycle as OV
    from paper_2104_13755_amd.solver import Hierarchy, Solver
    from helpers import ell3
    V, F = synth.small_icosphere(4, seed=21, sigma=0.01)
    _, L, m = AS.system(V, F, 1e-2)
    L = L.tocsr()
    Q = (L @ sp.diags(1.0 / m) @ L).tocsr()
    Q.sort_indices()
    n = Q.shape[0]
    rows = np.repeat(np.arange(n), np.diff(Q.indptr))
    Mv = np.where(rows == Q.indices, m[rows], 0.0)
    Ps, _, _ = OH.prolongations(V, F, n_levels=3)
    ells = [ell3(P) for P in Ps]
    sizes = [n] + [P.shape[1] for P in Ps]
    h = Hierarchy.from_prolongations(sizes, [e[0] for e in ells], [e[1] for e in ells])
    S = Solver(h, Q.indptr, Q.indices)
    S.split_prepare(_t(Q.data), _t(Mv))
    f = np.random.default_rng(63).uniform(-1, 1, (n, 1))
    for alpha in (1e-3, 1e-2):
        S.split_combine(alpha, 1.0 - alpha)
        A = sp.csr_matrix((alpha * Q.data + (1.0 - alpha) * Mv, Q.indices, Q.indptr), shape=Q.shape)
        b = (1.0 - alpha) * m[:, None] * f
        O = OV.Solver(Ps, A)
        xo, co, _ = O.solve(b, 1e-10)
        xg, info = S.solve(_t(b), rtol=1e-10, precision="fp64")
        assert info["cycles"] == co
        assert np.linalg.norm(_np(xg) - xo) / np.linalg.norm(xo) < 1e-9
        xp, ip = S.pcg(_t(b), rtol=1e-8, precision="fp32ir")
        res = np.linalg.norm(b - A @ _np(xp)) / np.linalg.norm(b)
        assert res <= 2e-8
        print(f"[bilaplacian] alpha={alpha}: {co} cycles, pcg {ip['iterations']}", flush=True)
