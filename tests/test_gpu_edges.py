"""GPU edge cases and error paths of the C ABI (all forced from the host;
no kernel is made to fault)."""
import numpy as np
import pytest

from helpers import Problem, gpu_available, rel

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def prob():
    if not gpu_available():
        pytest.skip("no GPU")
    p = Problem("disc-41x37")
    p.gpu = p.gpu_solver()
    return p


def _t(a):
    import torch
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


def test_single_level_is_direct_solve():
    if not gpu_available():
        pytest.skip("no GPU")
    import torch
    from paper_2104_13755_amd.solver import Hierarchy, Solver
    from oracle import assemble as AS
    import synth
    V, F = synth.flat_disc(20, 19, seed=2)
    A, _, m = AS.system(V, F, 1e-2)
    h = Hierarchy.from_prolongations([len(V)], [], [])
    S = Solver(h, A.indptr, A.indices)
    S.set_values(_t(A.data))
    b = np.random.default_rng(0).uniform(-1, 1, (len(V), 2))
    x, info = S.solve(_t(b), rtol=1e-12)
    assert info["cycles"] == 1
    assert rel(x.cpu().numpy(), np.linalg.solve(A.toarray(), b)) < 1e-12


def test_zero_rhs_column(prob):
    b = np.zeros((prob.sizes[0], 2))
    b[:, 1] = prob.m
    x, info = prob.gpu.solve(_t(b), rtol=1e-10)
    x = x.cpu().numpy()
    assert not x[:, 0].any()
    assert info["rel_res"][0] == 0.0 and info["rel_res"][1] <= 1e-10


def test_nonfinite_rhs(prob):
    from paper_2104_13755_amd._lib import SmgError
    b = np.ones((prob.sizes[0], 1))
    b[7, 0] = np.nan
    with pytest.raises(SmgError) as e:
        prob.gpu.solve(_t(b), rtol=1e-8)
    assert e.value.status == -6


def test_cycle_cap(prob):
    x, info = prob.gpu.solve(_t(prob.m[:, None]), rtol=1e-14, max_cycles=1, raise_on_error=False)
    assert info["status"] == -5 and info["cycles"] == 1
    assert np.isfinite(x.cpu().numpy()).all()


def test_not_spd():
    if not gpu_available():
        pytest.skip("no GPU")
    from paper_2104_13755_amd._lib import SmgError
    p = Problem("disc-41x37")
    S = p.gpu_solver()
    from oracle import assemble as AS
    A, _, _ = AS.system(p.V, p.F, -5.0)
    with pytest.raises(SmgError) as e:
        S.set_values(_t(A.data))
    assert e.value.status == -4
    with pytest.raises(SmgError) as e2:
        S.solve(_t(p.m[:, None]), rtol=1e-8)
    assert e2.value.status == -7


def test_nonfinite_matrix():
    if not gpu_available():
        pytest.skip("no GPU")
    from paper_2104_13755_amd._lib import SmgError
    p = Problem("disc-41x37")
    S = p.gpu_solver()
    vals = p.A.data.copy()
    vals[3] = np.inf
    with pytest.raises(SmgError) as e:
        S.set_values(_t(vals))
    assert e.value.status == -6


def test_bad_arguments(prob):
    """k = 5 and a residual on the coarsest level: the binding refuses them
    before the library, and the library itself returns INVALID_ARG."""
    import ctypes
    import torch
    from paper_2104_13755_amd import _lib as L
    S = prob.gpu
    b = _t(np.ones((prob.sizes[0], 5)))
    with pytest.raises(ValueError):
        S.solve(b, rtol=1e-8)
    x = torch.empty_like(b)
    p = L.SolveParams(1e-8, 100, L.SMG_FP64, 0, 0)
    st = S._lib.smg_solve(S._s, b.data_ptr(), x.data_ptr(), 5, ctypes.byref(p), None, None)
    assert st == -1
    last = S.num_levels - 1
    bc = _t(np.ones((prob.sizes[-1], 1)))
    with pytest.raises(ValueError):
        S.residual(last, bc, bc)
    rc = torch.empty_like(bc)
    assert S._lib.smg_residual(S._s, last, L.SMG_FP64, bc.data_ptr(), bc.data_ptr(), rc.data_ptr(), 1, None) == -1
