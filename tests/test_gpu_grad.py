"""Differentiation pattern: gradients of l = w^T u, u = (diag(s m) + t L)^{-1} b,
through HeatSolve (adjoint V-cycle) against (a) the oracle's dense-solve
gradients on the 2,562-vertex subcase and (b) central finite differences of
the library's own forward solves on the 655,362-vertex icosphere."""
import numpy as np
import pytest

import synth
from helpers import gpu_available, rel

pytestmark = pytest.mark.gpu


def _setup(level, rtol):
    import torch
    from paper_2104_13755_amd.autograd import HeatProblem
    w = synth.workload_c4(level=level)
    P = HeatProblem(w["V"], w["F"], rtol=rtol, max_cycles=400)
    dev = "cuda"
    b = torch.tensor(w["b"][:, 0], dtype=torch.float64, device=dev)
    wt = torch.tensor(w["w"], dtype=torch.float64, device=dev)
    return w, P, b, wt


def _grads(P, b, wt, t, s):
    import torch
    from paper_2104_13755_amd.autograd import HeatSolve
    bb = b.clone().requires_grad_(True)
    tt = torch.tensor(t, dtype=torch.float64, device=b.device, requires_grad=True)
    ss = s.clone().requires_grad_(True)
    u = HeatSolve.apply(bb, tt, ss, P)
    loss = (wt * u).sum()
    loss.backward()
    return float(loss.detach()), bb.grad, float(tt.grad), ss.grad


def test_refresh_sees_new_values():
    """A new s tensor must refresh A even if it reuses freed storage."""
    if not gpu_available():
        pytest.skip("no GPU")
    import torch
    w, P, b, wt = _setup(3, 1e-12)
    s = torch.ones(P.n, dtype=torch.float64, device="cuda")
    vals = []
    for scale in (1.0, 2.0, 1.0):
        P.refresh(w["t"], s * scale)
        vals.append(float((wt * P.solve(b)).sum()))
    assert vals[0] != vals[1] and abs(vals[0] - vals[2]) <= 1e-12 * abs(vals[0])


def test_dense_reference_2k():
    if not gpu_available():
        pytest.skip("no GPU")
    import torch
    from oracle import assemble as AS, grad as G
    w, P, b, wt = _setup(4, 1e-14)
    assert P.n == 2562
    s = torch.ones(P.n, dtype=torch.float64, device="cuda")
    loss, db, dt, ds = _grads(P, b, wt, w["t"], s)
    A, L, m = AS.system(w["V"], w["F"], w["t"])
    ref = G.dense_grads(A, L, m, w["b"], w["w"])
    assert abs(loss - float(w["w"] @ ref["u"])) <= 1e-11 * abs(loss)
    assert rel(db.cpu().numpy(), ref["db"]) < 1e-10
    assert abs(dt - ref["dt"]) <= 1e-10 * abs(ref["dt"])
    assert rel(ds.cpu().numpy(), ref["ds"]) < 1e-10


@pytest.mark.timeout(600)
def test_finite_differences_655k():
    if not gpu_available():
        pytest.skip("no GPU")
    import torch
    from paper_2104_13755_amd.autograd import HeatSolve
    w, P, b, wt = _setup(8, 1e-14)
    assert P.n == 655362
    t = w["t"]
    s = torch.ones(P.n, dtype=torch.float64, device="cuda")
    loss, db, dt, ds = _grads(P, b, wt, t, s)
    print(f"\n[grad] loss={loss:.6e} dt={dt:.6e} cycles={P.last_info['cycles']}", flush=True)

    def ell(tt, ss, bb=b):
        with torch.no_grad():
            tt_ = torch.tensor(tt, dtype=torch.float64, device="cuda")
            return float((wt * HeatSolve.apply(bb, tt_, ss.contiguous(), P)).sum())

    # dl/dt, relative step
    h = 1e-6 * t
    fd = (ell(t + h, s) - ell(t - h, s)) / (2 * h)
    print(f"[grad] dt fd={fd:.10e} adjoint={dt:.10e}", flush=True)
    assert abs(fd - dt) <= 1e-6 * abs(dt)
    # dl/ds_i at 8 sources (largest responses) and along a random direction.
    # Step 1e-4: the central quotient carries rounding noise ~ ulp(l) / (2h)
    # (l ~ 1e5, so ~1.4e-5 at h = 1e-6, as large as the 1e-6 relative bar on
    # dl/ds_i ~ 10); at 1e-4 the noise is 1.4e-7 and the O(h^2) truncation of
    # the smooth l(s) stays far below the bar.
    dsn = ds.cpu().numpy()
    hs = 1e-4
    for i in w["sources"][:8]:
        e = torch.zeros_like(s)
        e[int(i)] = hs
        fdi = (ell(t, s + e) - ell(t, s - e)) / (2 * hs)
        assert abs(fdi - dsn[i]) <= 1e-6 * abs(dsn[i]) + 1e-9 * np.abs(dsn).max(), (i, fdi, dsn[i])
    rng = np.random.default_rng(0)
    d = torch.tensor(rng.normal(size=P.n), dtype=torch.float64, device="cuda")
    d /= torch.linalg.norm(d)
    hd = 1e-4
    fdd = (ell(t, s + hd * d) - ell(t, s - hd * d)) / (2 * hd)
    ref = float((ds * d).sum())
    assert abs(fdd - ref) <= 1e-6 * abs(ref) + 1e-9 * float(torch.linalg.norm(ds))
    # dl/db: l is linear in b, so the directional derivative is exact
    db_dir = torch.tensor(rng.normal(size=P.n), dtype=torch.float64, device="cuda")
    fdb = (ell(t, s, b + db_dir) - ell(t, s, b - db_dir)) / 2.0
    refb = float((db * db_dir).sum())
    assert abs(fdb - refb) <= 1e-9 * abs(refb)
