"""Batching pattern: many meshes of uneven size (icospheres, tori, discs with
boundary) and 1-3 right-hand sides in ONE persistent launch replayed from a
hipGraph.  Each mesh is checked against the oracle (its own hierarchy,
assembly and tight FP64 solve) and against the library's unbatched solve."""
import os

import numpy as np
import pytest

import synth
from helpers import gpu_available

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def batch_case():
    if not gpu_available():
        pytest.skip("no GPU")
    import torch
    from oracle import assemble as AS, vcycle as OV
    from paper_2104_13755_amd.solver import Hierarchy, Solver, mesh_pattern
    meshes = synth.workload_c3(count=6, nmin=2500, nmax=14000, seed=31)
    out = []
    for w in meshes:
        V, F = w["V"], w["F"]
        h = Hierarchy.build(V, F, n_levels=0)
        rp, ci = mesh_pattern(len(V), F)
        S = Solver(h, rp, ci, faces=F)
        a, _, _ = S.assemble(torch.tensor(V, device="cuda"), w["t"])
        S.set_values(a)
        A, _, _ = AS.system(V, F, w["t"])
        Os, _, _ = OV.build(V, F, A, n_levels=0)
        xs, _, _ = Os.solve(w["b"], 1e-13, max_cycles=400)
        out.append(dict(w=w, S=S, A=A, xs=xs, b=torch.tensor(w["b"], device="cuda"), levels=len(h.sizes)))
        print(f"\n[mesh] {w['name']} n={len(V)} k={w['b'].shape[1]} t={w['t']:.2e} levels={h.sizes}", flush=True)
    return out


def _check(case, xs, infos, rtol):
    for c, x, info in zip(case, xs, infos):
        x = x.cpu().numpy()
        b = c["w"]["b"]
        res = np.linalg.norm(b - c["A"] @ x, axis=0) / np.linalg.norm(b, axis=0)
        err = np.linalg.norm(x - c["xs"]) / np.linalg.norm(c["xs"])
        assert res.max() <= rtol * 1.0001, (c["w"]["name"], res)
        assert err < 1e-6, (c["w"]["name"], err)
        assert max(info["rel_res"]) <= rtol


def test_batch_matches_oracle_and_unbatched(batch_case):
    from paper_2104_13755_amd.batch import BatchSolver
    B = BatchSolver([c["S"] for c in batch_case])
    for prec in ("fp32ir", "fp64"):
        xs, infos, st = B.solve([c["b"] for c in batch_case], rtol=1e-8, precision=prec)
        _check(batch_case, xs, infos, 1e-8)
        for c, x, info in zip(batch_case, xs, infos):
            xu, iu = c["S"].solve(c["b"], rtol=1e-8, precision=prec)
            assert iu["cycles"] == info["cycles"], (c["w"]["name"], prec, iu["cycles"], info["cycles"])
            rel = float((x - xu).norm() / xu.norm())
            assert rel < (1e-12 if prec == "fp64" else 1e-6), (c["w"]["name"], prec, rel)
        # replay of the captured graph: bitwise identical
        xs2, infos2, _ = B.solve([c["b"] for c in batch_case], rtol=1e-8, precision=prec)
        for x, x2 in zip(xs, xs2):
            assert bool((x == x2).all())


def test_batch_autotune_and_cache(batch_case, tmp_path):
    from paper_2104_13755_amd.batch import BatchSolver
    cache = str(tmp_path / "smg_tune.txt")
    B = BatchSolver([c["S"] for c in batch_case], cache_file=cache)
    B.solve([c["b"] for c in batch_case], rtol=1e-8)
    shape = B.autotune(budget_ms=20000)
    assert shape["threads"] in (256, 512, 1024)
    assert os.path.exists(cache)
    xs, infos, _ = B.solve([c["b"] for c in batch_case], rtol=1e-8)
    _check(batch_case, xs, infos, 1e-8)
    B2 = BatchSolver([c["S"] for c in batch_case], cache_file=cache)
    assert B2.shape() == shape


def test_batch_rejects_single_level():
    if not gpu_available():
        pytest.skip("no GPU")
    from paper_2104_13755_amd.solver import Hierarchy, Solver
    from paper_2104_13755_amd.batch import BatchSolver
    from paper_2104_13755_amd._lib import SmgError
    from oracle import assemble as AS
    V, F = synth.flat_disc(12, seed=1)
    A, _, _ = AS.system(V, F, 1e-2)
    S = Solver(Hierarchy.from_prolongations([len(V)], [], []), A.indptr, A.indices)
    with pytest.raises(SmgError):
        BatchSolver([S])


def test_batch_every_launch_shape(batch_case):
    """Every launch shape the autotuner may pick (workgroup size, lanes per
    row on level 0 and on the Galerkin levels, team size, teams on one XCD or
    spread over the device) gives an answer that meets the oracle's residual
    and takes the unbatched solve's cycle counts."""
    from paper_2104_13755_amd.batch import BatchSolver
    bs = [c["b"] for c in batch_case]
    cu = [c["S"].solve(c["b"], rtol=1e-8, precision="fp32ir")[1]["cycles"] for c in batch_case]
    for threads in (256, 512, 1024):
        for l0 in (1, 2):
            for lc in (1, 2, 4, 8):
                for tmax in (2, 8):
                    for dev in (False, True):
                        B = BatchSolver([c["S"] for c in batch_case], threads=threads, lanes_level0=l0,
                                        lanes_coarse=lc, team_max=tmax, device_teams=dev)
                        xs, infos, _ = B.solve(bs, rtol=1e-8)
                        shape = (threads, l0, lc, tmax, dev)
                        assert [i["cycles"] for i in infos] == cu, (shape, [i["cycles"] for i in infos], cu)
                        _check(batch_case, xs, infos, 1e-8)
                        del B


def test_batch_balanced_teams(batch_case):
    """Teams sized by level-0 entries x the last solve's cycles: the first
    solve lays the teams out by entries, the second by work; both meet the
    oracle's residual and take the unbatched cycle counts."""
    from paper_2104_13755_amd.batch import BatchSolver
    bs = [c["b"] for c in batch_case]
    cu = [c["S"].solve(c["b"], rtol=1e-8, precision="fp32ir")[1]["cycles"] for c in batch_case]
    for threads, tmax in ((1024, 16), (512, 32)):
        B = BatchSolver([c["S"] for c in batch_case], threads=threads, team_max=tmax, balance=True)
        assert B.shape()["balance"] == 1
        for _ in range(2):
            xs, infos, _ = B.solve(bs, rtol=1e-8)
            assert [i["cycles"] for i in infos] == cu, (threads, tmax, [i["cycles"] for i in infos], cu)
            _check(batch_case, xs, infos, 1e-8)
        del B
