"""The C-ABI boundary: a caller allocator (smg_ctx_create, here torch's
caching allocator) receives every device buffer of a solver and a batch and
gets all of them back at destruction; after creation no solve, cycle, PCG
solve, smoother switch or value refresh takes memory; a saved and reloaded
hierarchy gives the same solver; a timed solve reports per-phase times that
add up to its device time."""
import numpy as np
import pytest

from helpers import Problem, gpu_available

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def prob():
    if not gpu_available():
        pytest.skip("no GPU")
    return Problem("torus-96x40")


def _t(a):
    import torch
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


def test_torch_allocator_context(prob):
    import gc
    import torch
    from helpers import ell3
    from paper_2104_13755_amd.batch import BatchSolver
    from paper_2104_13755_amd.solver import Hierarchy, Solver, TorchAllocator
    ells = [ell3(P) for P in prob.Ps]
    h = Hierarchy.from_prolongations(prob.sizes, [e[0] for e in ells], [e[1] for e in ells])
    alloc = TorchAllocator(0)
    torch.cuda.synchronize()
    before = torch.cuda.memory_allocated()
    S = Solver(h, prob.A.indptr, prob.A.indices, allocator=alloc)
    taken = alloc.bytes_in_use
    assert taken > 0 and len(alloc.live) > 20
    assert torch.cuda.memory_allocated() - before >= taken      # visible to torch
    S.set_values(_t(prob.A.data))
    b = prob.m[:, None] * np.random.default_rng(3).uniform(-1, 1, (prob.sizes[0], 2))
    x, info = S.solve(_t(b), rtol=1e-8, precision="fp32ir")
    # the same solve as a solver with the library's own allocations
    R = prob.gpu_solver()
    xr, ir = R.solve(_t(b), rtol=1e-8, precision="fp32ir")
    assert info["cycles"] == ir["cycles"] and bool((x == xr).all())
    n_live = len(alloc.live)
    S.pcg(_t(b), rtol=1e-8)
    S.set_smoother("jacobi")
    S.solve(_t(b), rtol=1e-8, max_cycles=400, raise_on_error=False)
    S.set_smoother("gs")
    S.set_values(_t(prob.A.data))
    S.vcycle(_t(b), _t(np.zeros_like(b)), precision="fp32ir")
    assert len(alloc.live) == n_live                              # nothing taken after creation
    B = BatchSolver([S, S])
    assert len(alloc.live) > n_live                               # the batch takes from the same allocator
    del B
    gc.collect()
    assert len(alloc.live) == n_live
    del S
    gc.collect()
    torch.cuda.synchronize()
    assert len(alloc.live) == 0 and alloc.bytes_in_use == 0


def test_saved_hierarchy_gives_the_same_solver(prob, tmp_path):
    import synth
    from paper_2104_13755_amd.solver import Hierarchy, Solver, mesh_pattern
    V, F = prob.V, prob.F
    h = Hierarchy.build(V, F, n_levels=prob.n_levels)
    h.save(tmp_path / "t.smg")
    g = Hierarchy.load(tmp_path / "t.smg")
    rp, ci = mesh_pattern(len(V), F)
    S1 = Solver(h, rp, ci)
    S2 = Solver(g, rp, ci)
    S1.set_values(_t(prob.A.data))
    S2.set_values(_t(prob.A.data))
    for l in range(S1.num_levels - 1):
        c1, n1 = S1.colors(l)
        c2, n2 = S2.colors(l)
        assert n1 == n2 and np.array_equal(c1, c2)
    b = prob.m[:, None] * np.random.default_rng(4).uniform(-1, 1, (len(V), 3))
    x1, i1 = S1.solve(_t(b), rtol=1e-8, precision="fp32ir")
    x2, i2 = S2.solve(_t(b), rtol=1e-8, precision="fp32ir")
    assert i1["cycles"] == i2["cycles"] and bool((x1 == x2).all())     # same layout, same arithmetic


def test_timed_solve_reports_phases(prob):
    S = prob.gpu_solver(tail_rows=-1)       # per-color launches on every level (this mesh fits the tail)
    b = prob.m[:, None] * np.random.default_rng(5).uniform(-1, 1, (prob.sizes[0], 3))
    x0, i0 = S.solve(_t(b), rtol=1e-8, precision="fp32ir")
    x1, i1 = S.solve(_t(b), rtol=1e-8, precision="fp32ir", timed=True)
    assert bool((x0 == x1).all()) and i0["cycles"] == i1["cycles"]    # timing changes nothing
    ph = i1["ms_phase"]
    assert ph["prepare"] > 0 and ph["relax"] > 0 and ph["transfer"] > 0 and ph["norm"] > 0 and ph["other"] > 0
    assert ph["relax"] > ph["transfer"]
    total = sum(v for k, v in ph.items() if k != "prepare")
    assert total <= i1["ms"] * 1.05                      # device time inside the wall time of the solve
    assert i0["ms_phase"]["relax"] == 0.0 and i0["ms_phase"]["prepare"] == ph["prepare"]


def test_profile_counts_every_relaxation_launch(prob):
    """smg_profile_enable / smg_profile_read: one event pair per relaxation
    launch (or per relaxation call with "gs_group"), every launch counted, and
    the byte rule z (s + 4) + 4 (n + 1) + 3 k n s per sweep (z = entries incl.
    the diagonal), summed over the colors of the sweep."""
    S = prob.gpu_solver(tail_rows=-1)
    k, cycles = 3, 2
    b = _t(prob.m[:, None] * np.random.default_rng(6).uniform(-1, 1, (prob.sizes[0], k)))
    for prec, sb in (("fp64", 8), ("fp32ir", 4)):
        for level, kind in ((-1, "gs"), (1, "gs"), (-1, "gs_group"), (1, "gs_group")):
            S.profile_enable(kind, level)
            x, info = S.solve(b, fixed_cycles=cycles, precision=prec)
            p = S.profile_read()
            S.profile_enable(None)
            levels = range(S.num_levels - 1) if level < 0 else [level]
            launches = cycles * sum(4 * S.colors(l)[1] for l in levels)
            want = cycles * sum(4 * (S.level_nnz(l) * (sb + 4) + 4 * (S.level_size(l) + 1)
                                     + 3 * k * S.level_size(l) * sb) for l in levels)
            assert p["launches"] == launches, (prec, level, kind)
            assert abs(p["bytes"] - want) <= 1e-12 * want, (prec, level, kind)
            assert 0 < p["ms"] < info["ms"] * 1.05
    x1, _ = S.solve(b, fixed_cycles=cycles, precision="fp32ir")
    S.profile_enable("gs", -1)
    x2, _ = S.solve(b, fixed_cycles=cycles, precision="fp32ir")
    S.profile_enable(None)
    assert bool((x1 == x2).all())                     # profiling changes no result


def test_launch_floor(prob):
    from paper_2104_13755_amd._lib import SmgError
    S = prob.gpu_solver(tail_rows=-1)
    for kind in ("empty", "chain", "chain_rw"):
        for level in range(S.num_levels - 1):
            us, per = S.launch_floor(kind, level, launches=200)
            assert 0.0 < us < 1e3 and 0.0 < per < 1e3, (kind, level, us, per)
    with pytest.raises(SmgError):
        S.launch_floor("chain", S.num_levels - 1)          # the coarsest level has no color launches
    with pytest.raises(SmgError):
        S.launch_floor("chain", 0, launches=0)
