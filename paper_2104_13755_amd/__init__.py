"""MI355X-native surface multigrid (Galerkin V-cycle with intrinsic
prolongation) -- HIP kernels for gfx950 behind the C ABI of include/smg.h.

Importing the package does not load the library; the first use does, and it
fails loudly if libsmg.so has not been built.
"""
from ._lib import load, SmgError, LIB_PATH  # noqa: F401


def __getattr__(name):
    if name in ("Hierarchy", "Solver", "mesh_pattern"):
        from . import solver
        return getattr(solver, name)
    if name in ("HeatSolve", "HeatProblem"):
        from . import autograd
        return getattr(autograd, name)
    if name in ("BatchSolver",):
        from . import batch
        return getattr(batch, name)
    raise AttributeError(name)
