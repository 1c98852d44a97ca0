"""GPU parity of the damped Jacobi relaxation (App. "Ablation Study") against
the oracle's: per-level factors, single sweeps per level, one V-cycle, fixed-cycle and converged
FP64 solves (identical cycle counts), the mixed-precision solve against the
oracle's residual, PCG with the Jacobi V-cycle, switching back to
Gauss-Seidel, and argument errors."""
import numpy as np
import pytest

from helpers import Problem, gpu_available, rel
from oracle import pcg as OP, vcycle as OV

pytestmark = pytest.mark.gpu

CASES = ["icosphere-L5", "disc-41x37", "torus-96x40", "heightfield-70x66"]


@pytest.fixture(scope="module", params=CASES)
def prob(request):
    if not gpu_available():
        pytest.skip("no GPU")
    print(f"\n[case] {request.param}", flush=True)
    p = Problem(request.param)
    p.gpu = p.gpu_solver()
    p.gpu.set_smoother("jacobi")
    p.oj = OV.Solver(p.Ps, p.A, smoother="jacobi")
    return p


def _t(a):
    import torch
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


def _np(t):
    return t.detach().cpu().numpy()


def test_level_factors(prob):
    """omega_l = 2 / (1 + lambda_l) from the power-step estimate on each side;
    a set factor is used on every level."""
    S, O = prob.gpu, prob.oj
    for l in range(O.nlev - 1):
        assert abs(S.jacobi_omega(l) - O.omegas[l]) < 1e-12 * O.omegas[l], l
    S.set_smoother("jacobi", 0.6)
    try:
        Of = OV.Solver(prob.Ps, prob.A, smoother="jacobi", omega=0.6)
        rng = np.random.default_rng(50)
        b = rng.uniform(-1, 1, (prob.sizes[0], 2))
        x0 = rng.uniform(-1, 1, (prob.sizes[0], 2))
        assert all(S.jacobi_omega(l) == 0.6 for l in range(O.nlev - 1))
        assert rel(_np(S.vcycle(_t(b), _t(x0))), Of.vcycle(0, x0.copy(), b)) < 1e-12
    finally:
        S.set_smoother("jacobi")


def test_sweeps_and_cycle(prob):
    S, O = prob.gpu, prob.oj
    rng = np.random.default_rng(51)
    for l in range(O.nlev - 1):
        for k in (1, 3):
            n = prob.sizes[l]
            b = rng.uniform(-1, 1, (n, k))
            x = rng.uniform(-1, 1, (n, k))
            for sweeps in (1, 2, 3):
                xg = S.smooth(l, _t(b), _t(x), sweeps)
                assert rel(_np(xg), O.relax(l, x.copy(), b, sweeps)) < 1e-13, (l, k, sweeps)
    for k in (1, 2, 4):
        n = prob.sizes[0]
        b = rng.uniform(-1, 1, (n, k))
        x0 = rng.uniform(-1, 1, (n, k))
        assert rel(_np(S.vcycle(_t(b), _t(x0))), O.vcycle(0, x0.copy(), b)) < 1e-12, k


def test_solves(prob):
    S, O = prob.gpu, prob.oj
    rng = np.random.default_rng(52)
    b = prob.m[:, None] * rng.uniform(-1, 1, (prob.sizes[0], 3))
    rtol = 1e-10
    xo, co, _ = O.solve(b, rtol, max_cycles=300)
    xg, info = S.solve(_t(b), rtol=rtol, precision="fp64", max_cycles=300)
    assert info["cycles"] == co
    xf, _ = S.solve(_t(b), fixed_cycles=co, precision="fp64")
    assert np.linalg.norm(_np(xf) - xo) / np.linalg.norm(xo) < 1e-10
    xm, im = S.solve(_t(b), rtol=1e-8, precision="fp32ir", max_cycles=300)
    res = np.linalg.norm(b - prob.A @ _np(xm), axis=0) / np.linalg.norm(b, axis=0)
    assert res.max() <= 1e-8 * 1.0001
    # PCG with the Jacobi cycle (symmetric as it is)
    xp, ip, hp = OP.pcg(prob.A, b, lambda r: O.vcycle(0, np.zeros_like(r), r), 0.0, fixed_iters=5)
    xq, iq = S.pcg(_t(b), fixed_iters=5, precision="fp64")
    assert rel(_np(xq), xp) < 1e-10
    xc, ic = S.pcg(_t(b), rtol=1e-8, precision="fp32ir")
    res = np.linalg.norm(b - prob.A @ _np(xc), axis=0) / np.linalg.norm(b, axis=0)
    assert max(ic["rel_res"]) <= 1e-8 and res.max() <= 2e-8
    print(f"[jacobi] {prob.name}: {co} cycles (mixed {im['cycles']}), pcg {ic['iterations']}", flush=True)


def test_switch_back_and_errors(prob):
    from paper_2104_13755_amd._lib import SmgError
    S = prob.gpu
    rng = np.random.default_rng(53)
    b = _t(prob.m[:, None] * rng.uniform(-1, 1, (prob.sizes[0], 2)))
    S.set_smoother("gs")
    try:
        x1, i1 = S.solve(b, rtol=1e-9, precision="fp32ir")
        G = prob.gpu_solver()                  # a solver that never used Jacobi
        x2, i2 = G.solve(b, rtol=1e-9, precision="fp32ir")
        assert i1["cycles"] == i2["cycles"] and np.array_equal(_np(x1), _np(x2))
        for bad in (2.0, 2.5, float("nan")):
            with pytest.raises(SmgError):
                S.set_smoother("jacobi", bad)
    finally:
        S.set_smoother("jacobi")


def test_odd_sweep_counts():
    """mu_pre = 1, mu_post = 3: odd Jacobi sweep counts end in the second
    iterate and are copied back; the cycle matches the oracle's."""
    if not gpu_available():
        pytest.skip("no GPU")
    p = Problem("disc-41x37")
    S = p.gpu_solver(mu_pre=1, mu_post=3)
    S.set_smoother("jacobi")
    O = OV.Solver(p.Ps, p.A, mu_pre=1, mu_post=3, smoother="jacobi")
    rng = np.random.default_rng(54)
    b = rng.uniform(-1, 1, (p.sizes[0], 2))
    x0 = rng.uniform(-1, 1, (p.sizes[0], 2))
    assert rel(_np(S.vcycle(_t(b), _t(x0))), O.vcycle(0, x0.copy(), b)) < 1e-12
    xo, co, _ = O.solve(b, 1e-10, max_cycles=300)
    xg, info = S.solve(_t(b), rtol=1e-10, precision="fp64", max_cycles=300)
    assert info["cycles"] == co and rel(_np(xg), xo) < 1e-9


def test_graph_replay_with_jacobi(prob):
    """Cycles captured into a graph with the Jacobi smoother replay to the
    same iterates as eager launches (several replays in a row)."""
    S = prob.gpu
    rng = np.random.default_rng(55)
    b = _t(prob.m[:, None] * rng.uniform(-1, 1, (prob.sizes[0], 2)))
    for precision in ("fp64", "fp32ir"):
        x1, i1 = S.solve(b, rtol=1e-9, precision=precision, max_cycles=300)
        for _ in range(3):
            x2, i2 = S.solve(b, rtol=1e-9, precision=precision, max_cycles=300, use_graph=True)
            assert i1["cycles"] == i2["cycles"] and np.array_equal(_np(x1), _np(x2)), precision
