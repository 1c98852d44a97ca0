"""GPU parity of conjugate gradients preconditioned by one symmetric V-cycle
(smg_pcg_solve; the combination proposed in Sec. "Limitations & Future
Work") against the oracle's PCG with the same preconditioner, on seeded
meshes: fixed iteration counts element by element (FP64: rounding of the
V-cycle amplified through the CG scalars, 1e-10 relative), converged solves
with identical iteration counts, the FP32 preconditioner against the
oracle's own residual, the post-relaxation in descending color order both in
launches and in the LDS tail, and edge cases."""
import numpy as np
import pytest

from helpers import Problem, gpu_available, rel
from oracle import pcg as OP

pytestmark = pytest.mark.gpu

CASES = ["icosphere-L5", "disc-41x37", "torus-96x40", "heightfield-70x66"]


@pytest.fixture(scope="module", params=CASES)
def prob(request):
    if not gpu_available():
        pytest.skip("no GPU")
    print(f"\n[case] {request.param}", flush=True)
    p = Problem(request.param)
    p.gpu = p.gpu_solver()                    # small levels in the LDS tail
    p.gpu_launch = p.gpu_solver(tail_rows=1)  # every level on launches
    p.B = OP.vcycle_preconditioner(p.oracle)
    return p


def _t(a):
    import torch
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


def _np(t):
    return t.detach().cpu().numpy()


def _rhs(prob, k, seed):
    rng = np.random.default_rng(seed)
    return prob.m[:, None] * rng.uniform(-1, 1, (prob.sizes[0], k))


@pytest.mark.parametrize("which", ["tail", "launches"])
def test_fixed_iterations_match_oracle(prob, which):
    S = prob.gpu if which == "tail" else prob.gpu_launch
    for k in (1, 3):
        b = _rhs(prob, k, 11 + k)
        for its in (1, 3, 6):
            xg, info = S.pcg(_t(b), fixed_iters=its, precision="fp64")
            xo, io, ho = OP.pcg(prob.A, b, prob.B, 0.0, fixed_iters=its)
            assert info["iterations"] == its == io
            assert rel(_np(xg), xo) < 1e-10, (which, k, its)
            assert np.allclose(info["rel_res"], ho[-1], rtol=1e-7, atol=1e-300), (which, k, its)


def test_converged_fp64_matches_oracle(prob):
    b = _rhs(prob, 3, 21)
    rtol = 1e-10
    xo, io, ho = OP.pcg(prob.A, b, prob.B, rtol)
    xg, info = prob.gpu.pcg(_t(b), rtol=rtol, precision="fp64")
    assert info["iterations"] == io
    assert max(info["rel_res"]) <= rtol
    assert np.linalg.norm(_np(xg) - xo) / np.linalg.norm(xo) < 1e-9
    res = np.linalg.norm(b - prob.A @ _np(xg), axis=0) / np.linalg.norm(b, axis=0)
    assert res.max() <= 2 * rtol
    # fewer iterations than plain V-cycles to the same tolerance
    _, cyc = prob.gpu.solve(_t(b), rtol=rtol, precision="fp64")
    print(f"[pcg] {prob.name}: {io} iterations vs {cyc['cycles']} cycles", flush=True)
    assert io <= cyc["cycles"]


def test_fp32_preconditioner(prob):
    b = _rhs(prob, 2, 31)
    rtol = 1e-8
    x64, i64 = prob.gpu.pcg(_t(b), rtol=rtol, precision="fp64")
    x32, i32 = prob.gpu.pcg(_t(b), rtol=rtol, precision="fp32ir")
    res = np.linalg.norm(b - prob.A @ _np(x32), axis=0) / np.linalg.norm(b, axis=0)
    assert max(i32["rel_res"]) <= rtol
    assert res.max() <= 2 * rtol
    assert i32["iterations"] <= i64["iterations"] + 2
    # run ahead of the stop test: the result is that of the reported count
    xf, _ = prob.gpu.pcg(_t(b), fixed_iters=i32["iterations"], precision="fp32ir")
    assert np.array_equal(_np(xf), _np(x32))


def test_edges(prob):
    import torch
    S = prob.gpu
    n = prob.sizes[0]
    b = _rhs(prob, 3, 41)
    b[:, 1] = 0.0                                  # a zero column stays zero
    x, info = S.pcg(_t(b), rtol=1e-9, precision="fp64")
    x = _np(x)
    assert np.all(np.isfinite(x)) and np.all(x[:, 1] == 0.0) and info["rel_res"][1] == 0.0
    x0, i0 = S.pcg(_t(np.zeros((n, 2))), rtol=1e-9)
    assert i0["iterations"] == 0 and np.all(_np(x0) == 0.0)
    # a cap below the needed count reports it and returns that iterate
    full = S.pcg(_t(b), rtol=1e-9)[1]["iterations"]
    xc, ic = S.pcg(_t(b), rtol=1e-9, max_iters=full - 1, raise_on_error=False)
    xf, _ = S.pcg(_t(b), fixed_iters=full - 1)
    assert ic["status"] != 0 and ic["iterations"] == full - 1
    assert np.array_equal(_np(xc), _np(xf))
    bad = b.copy()
    bad[3, 0] = np.nan
    _, ib = S.pcg(_t(bad), raise_on_error=False)
    assert ib["status"] != 0
    # an unsymmetric cycle is refused
    S2 = prob.gpu_solver(mu_pre=2, mu_post=1)
    _, i2 = S2.pcg(_t(b), raise_on_error=False)
    assert i2["status"] != 0
    torch.cuda.synchronize()


def test_rhs_counts_and_single_level():
    """2 and 4 right-hand sides against the oracle; a one-level hierarchy is
    the direct solve."""
    if not gpu_available():
        pytest.skip("no GPU")
    p = Problem("disc-41x37")
    S = p.gpu_solver()
    B = OP.vcycle_preconditioner(p.oracle)
    for k in (2, 4):
        b = _rhs(p, k, 90 + k)
        xg, info = S.pcg(_t(b), fixed_iters=4, precision="fp64")
        xo, _, _ = OP.pcg(p.A, b, B, 0.0, fixed_iters=4)
        assert rel(_np(xg), xo) < 1e-10, k
    one = Problem("disc-41x37", n_levels=1)
    S1 = one.gpu_solver()
    b = _rhs(one, 2, 95)
    x1, i1 = S1.pcg(_t(b), rtol=1e-10)
    xs = np.linalg.solve(one.A.toarray(), b)
    assert i1["iterations"] == 1 and rel(_np(x1), xs) < 1e-12
