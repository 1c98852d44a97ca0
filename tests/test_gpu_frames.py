"""Time-varying A: every frame the per-edge weights of L and t change; the
library re-assembles A_0, re-runs the Galerkin products over all levels and
the coarsest Cholesky on the device, then solves in FP32 cycles with FP64
refinement.  Each frame is checked against the oracle's own assembly,
Galerkin hierarchy and tight FP64 solve (same seeded frame recipe, reduced
disc)."""
import numpy as np
import pytest

import synth
from helpers import gpu_available, rel

pytestmark = pytest.mark.gpu


def test_frames_reduced_disc():
    if not gpu_available():
        pytest.skip("no GPU")
    import torch
    from oracle import assemble as AS, vcycle as OV
    from paper_2104_13755_amd.solver import Hierarchy, Solver, mesh_pattern
    mesh = synth.workload_c5_mesh(nx=141, ny=140)
    V, F = mesh["V"], mesh["F"]
    nl = 5
    h = Hierarchy.build(V, F, n_levels=nl)
    rp, ci = mesh_pattern(len(V), F)
    S = Solver(h, rp, ci, faces=F)
    Vd = torch.tensor(V, dtype=torch.float64, device="cuda")
    # oracle: its own hierarchy, the same frames
    A0, L0, m = AS.system(V, F, 1e-2)
    Os, _, _ = OV.build(V, F, A0, n_levels=nl)
    b = m[:, None] * mesh["u"]
    bd = torch.tensor(b, dtype=torch.float64, device="cuda")
    for k in range(3):
        fr = synth.workload_c5_frame(mesh, k)
        w32 = fr["w"].astype(np.float32)
        a, _, _ = S.assemble(Vd, fr["t"], edge_w=torch.tensor(w32, device="cuda"))
        S.set_values(a)
        A, _, _ = AS.system(V, F, fr["t"], edge_weights=w32.astype(np.float64), edges=mesh["edges"])
        assert rel(a.cpu().numpy(), A.data) < 1e-13
        Os.set_values(A)
        for l in range(nl):
            Ag = S.level_matrix(l)
            assert np.array_equal(Ag.indices, Os.A[l].indices)
            assert rel(Ag.data, Os.A[l].data) < 1e-12, (k, l)
        x, info = S.solve(bd, rtol=1e-8, precision="fp32ir")
        x = x.cpu().numpy()
        res = np.linalg.norm(b - A @ x) / np.linalg.norm(b)
        xs, _, _ = Os.solve(b, 1e-13, max_cycles=300)
        err = np.linalg.norm(x - xs) / np.linalg.norm(xs)
        print(f"\n[frame {k}] t={fr['t']:.3e} cycles={info['cycles']} res={res:.2e} err={err:.2e}")
        assert res <= 1e-8 * 1.0001
        assert err < 1e-6
