"""The Python binding checks every tensor before its pointer crosses the C
ABI (device, dtype, contiguity, shape against the level size): a wrong
argument raises before any library call that could launch a kernel."""
import numpy as np
import pytest

from helpers import Problem, gpu_available

pytestmark = pytest.mark.gpu


class _NoLaunch:
    """Library proxy: structure queries pass through, any other call fails."""

    ALLOWED = {"smg_num_levels", "smg_level_size", "smg_level_nnz"}

    def __init__(self, lib):
        self._lib = lib

    def __getattr__(self, name):
        if name in self.ALLOWED:
            return getattr(self._lib, name)

        def refuse(*args):
            raise AssertionError(f"{name} called although an argument was invalid")
        return refuse


@pytest.fixture(scope="module")
def solver():
    if not gpu_available():
        pytest.skip("no GPU")
    p = Problem("disc-41x37")
    S = p.gpu_solver(faces=True)
    return p, S


def test_invalid_arguments_raise_before_the_library(solver):
    import torch
    p, S = solver
    n, n1, nnz = S.n, S.level_size(1), S.nnz
    f = dict(dtype=torch.float64, device="cuda")
    ok = torch.zeros((n, 2), **f)
    ok1 = torch.zeros((n1, 2), **f)
    real = S._lib
    S._lib = _NoLaunch(real)
    try:
        bad = [
            lambda: S.residual(0, torch.zeros((n - 1, 2), **f), ok),               # short
            lambda: S.residual(0, ok, torch.zeros((n, 2), dtype=torch.float32, device="cuda")),
            lambda: S.residual(0, ok.cpu(), ok),                                   # host tensor
            lambda: S.residual(0, ok, torch.zeros((2, n), **f).t()),               # not contiguous
            lambda: S.residual(S.num_levels - 1, ok1, ok1),                        # coarsest
            lambda: S.residual(7, ok, ok),                                         # no such level
            lambda: S.smooth(1, ok, ok, 1),                                        # level-0 size on level 1
            lambda: S.smooth(0, torch.zeros((n, 5), **f), torch.zeros((n, 5), **f), 1),   # k = 5
            lambda: S.restrict(0, ok1),
            lambda: S.prolong_add(0, ok, ok),                                      # e of the wrong level
            lambda: S.prolong_add(0, torch.zeros((n1, 1), **f), ok),               # k mismatch
            lambda: S.vcycle(ok, torch.zeros((n, 3), **f)),
            lambda: S.coarse_solve(ok),
            lambda: S.solve(torch.zeros(n + 1, **f)),
            lambda: S.pcg(torch.zeros(n, dtype=torch.float32, device="cuda")),
            lambda: S.set_values(torch.zeros(nnz - 1, **f)),
            lambda: S.assemble(torch.zeros((n, 3), **f), 1e-2, mass_scale=torch.zeros(n - 1, **f)),
            lambda: S.assemble(torch.zeros((n, 3), **f), 1e-2, mass_scale=torch.zeros(n, dtype=torch.float32, device="cuda")),
            lambda: S.assemble(torch.zeros((n, 3), **f), 1e-2, edge_w=torch.zeros((nnz - n) // 2, **f)),
            lambda: S.assemble(torch.zeros((n, 3), **f), 1e-2,
                               edge_w=torch.zeros((nnz - n) // 2 - 1, dtype=torch.float32, device="cuda")),
            lambda: S.assemble(torch.zeros((n, 2), **f), 1e-2),
            lambda: S.split_prepare(torch.zeros(nnz, **f), torch.zeros(nnz - 1, **f)),
            lambda: S.spmv_dot(torch.zeros(nnz, **f), torch.zeros(n - 1, **f), torch.zeros(n, **f)),
            lambda: S.mass_grad(torch.zeros(n, **f), torch.zeros(n - 1, **f), torch.zeros(n, **f)),
        ]
        for i, call in enumerate(bad):
            with pytest.raises((ValueError, TypeError)):
                call()
    finally:
        S._lib = real
    # the same solver still works with valid arguments
    r = S.residual(0, ok, ok)
    assert float(r.abs().max()) == 0.0
