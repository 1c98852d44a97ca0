"""smg_spmv_dot_noalloc, the variant of smg_spmv_dot (lambda^T L u, the
adjoint helper) that allocates nothing: its partial sums live in a static
device array.  Through the C ABI it must give the same value as
smg_spmv_dot (same kernels, same summation order: bit for bit), on two calls
in a row, the second with a smaller matrix, and refuse a matrix above its
limit."""
import ctypes

import numpy as np
import pytest

from helpers import gpu_available

pytestmark = pytest.mark.gpu


def _case(nx, ny, seed):
    import torch
    import synth
    from oracle import assemble as AS
    from paper_2104_13755_amd.solver import Hierarchy, Solver, mesh_pattern
    rng = np.random.default_rng(seed)
    V, F = synth.disc_grid(nx, ny, rng, 0.1, height=lambda x, y: 0.1 * np.sin(3 * x))
    h = Hierarchy.build(V, F, n_levels=2)
    rp, ci = mesh_pattern(len(V), F)
    S = Solver(h, rp, ci, faces=F)
    _, lv, m = S.assemble(torch.tensor(V, dtype=torch.float64, device="cuda"), 1e-2, want_l=True, want_mass=True)
    lam = torch.tensor(rng.uniform(-1, 1, len(V)), dtype=torch.float64, device="cuda")
    u = torch.tensor(rng.uniform(-1, 1, len(V)), dtype=torch.float64, device="cuda")
    d_rp = torch.tensor(rp, dtype=torch.int32, device="cuda")
    d_ci = torch.tensor(ci, dtype=torch.int32, device="cuda")
    return S, lv, lam, u, d_rp, d_ci, len(V)


def test_noalloc_equals_the_allocating_entry_point():
    if not gpu_available():
        pytest.skip("no GPU")
    import torch
    from paper_2104_13755_amd import _lib as L
    lib = L.load()
    out = torch.empty(1, dtype=torch.float64, device="cuda")
    for nx, ny, seed in ((150, 140, 1), (37, 41, 2)):          # the second call is smaller
        S, lv, lam, u, d_rp, d_ci, n = _case(nx, ny, seed)
        ref = S.spmv_dot(lv, lam, u)
        out.fill_(np.nan)
        st = lib.smg_spmv_dot_noalloc(n, d_rp.data_ptr(), d_ci.data_ptr(), lv.data_ptr(), lam.data_ptr(),
                                      u.data_ptr(), out.data_ptr(), torch.cuda.current_stream().cuda_stream)
        assert st == 0
        torch.cuda.synchronize()
        assert float(out.item()) == ref, (n, float(out.item()), ref)
        # and against a plain float64 reference of lambda^T L u
        import scipy.sparse as sp
        Lc = sp.csr_matrix((lv.cpu().numpy(), d_ci.cpu().numpy(), d_rp.cpu().numpy()), shape=(n, n))
        ln, un = lam.cpu().numpy(), u.cpu().numpy()
        want = float(ln @ (Lc @ un))
        assert abs(ref - want) <= 1e-12 * float(np.abs(ln) @ (abs(Lc) @ np.abs(un)))
    # above the scratch limit: refused before any launch
    big = 1 << 25
    st = lib.smg_spmv_dot_noalloc(big, d_rp.data_ptr(), d_ci.data_ptr(), lv.data_ptr(), lam.data_ptr(),
                                  u.data_ptr(), out.data_ptr(), None)
    assert st == -1 and b"at most" in lib.smg_last_error()
