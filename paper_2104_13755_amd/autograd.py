"""Differentiable heat / screened-Poisson solve through the multigrid V-cycle.

u = A(t, s)^{-1} b with A(t, s) = diag(s * m) + t L (lumped mass m, cotan
Laplacian L; the systems of the paper's Sec. 6 examples).  The backward pass
reuses the same hierarchy and V-cycle for the adjoint solve (A is symmetric):

    lambda = A^{-1} g,  dl/db = lambda,  dl/dt = -lambda^T L u,
    dl/ds_i = -lambda_i m_i u_i.

Changing t or s only refreshes the values of the hierarchy (on-device
assembly, Galerkin A_{l+1} = P_l^T A_l P_l, coarsest Cholesky); the
prolongations are geometry-only and built once (Fig. fourSteps: the hierarchy
is reused when A changes).  All arithmetic runs in libsmg's kernels.
"""
import torch

from .solver import Hierarchy, Solver, mesh_pattern


class HeatProblem:
    """A mesh with its device-resident multigrid hierarchy."""

    def __init__(self, V, F, n_levels=0, device=0, rtol=1e-10, max_cycles=200,
                 precision="fp64", hier=None, **solver_kw):
        self.hier = hier if hier is not None else Hierarchy.build(V, F, n_levels=n_levels)
        rp, ci = mesh_pattern(len(V), F)
        self.solver = Solver(self.hier, rp, ci, device=device, faces=F, **solver_kw)
        self.V = torch.as_tensor(V, dtype=torch.float64).to(f"cuda:{device}").contiguous()
        self.n = len(V)
        self.rtol, self.max_cycles, self.precision = rtol, max_cycles, precision
        self._key = None          # (t, id of s, s version) of the current values
        self._s_ref = None        # holds s so its storage cannot be recycled
        self.l_vals = None
        self.mass = None
        self.last_info = None

    def refresh(self, t, s=None):
        """Set A = diag(s m) + t L on the device, skipped only when t and the
        very same s tensor (unmodified since) were used last time."""
        key = (float(t), None if s is None else (id(s), s._version))
        if key == self._key and s is self._s_ref:
            return
        a, lv, m = self.solver.assemble(self.V, float(t), mass_scale=s, want_l=True, want_mass=True)
        self.solver.set_values(a)
        self.l_vals, self.mass = lv, m
        self._key = key
        self._s_ref = s

    def solve(self, rhs):
        x, info = self.solver.solve(rhs.contiguous(), rtol=self.rtol, max_cycles=self.max_cycles,
                                    precision=self.precision)
        self.last_info = info
        return x


class HeatSolve(torch.autograd.Function):
    """u = HeatSolve.apply(b, t, s, problem) with b: (n,) float64 CUDA,
    t: 0-dim float64 tensor, s: (n,) float64 CUDA mass scales."""

    @staticmethod
    def forward(ctx, b, t, s, problem):
        s = s.contiguous()
        problem.refresh(t.item(), s)
        u = problem.solve(b)
        ctx.save_for_backward(u, s)
        ctx.problem = problem
        ctx.t = t.item()
        return u

    @staticmethod
    def backward(ctx, g):
        u, s = ctx.saved_tensors
        P = ctx.problem
        P.refresh(ctx.t, s)
        lam = P.solve(g.contiguous())                                   # adjoint V-cycle solve
        dt = -P.solver.spmv_dot(P.l_vals, lam, u)                       # -lambda^T L u
        ds = P.solver.mass_grad(lam, P.mass, u)                         # -lambda * m * u
        dtt = torch.tensor(dt, dtype=torch.float64, device=u.device)
        return lam, dtt, ds, None
