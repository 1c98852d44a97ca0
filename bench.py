#!/usr/bin/env python3
"""Benchmark: surface-multigrid V-cycle solves/s at 1M vertices to relative
residual 1e-8, mixed precision (FP32 cycles inside FP64 refinement) vs FP64.

Workload: jittered torus grid 1000 x 1000 (1,000,000 vertices, 2,000,000
triangles), R = 1, r = 0.3, A = M + 1e-2 L, three right-hand sides b = M X
(vertex coordinates), 7 levels, 2 + 2 multicolor Gauss-Seidel sweeps, dense
FP64 Cholesky on the coarsest level.

One step = on-device assembly of A_0, Galerkin refresh of every level,
coarsest Cholesky, and the full solve of the 3-RHS system to 1e-8 (the
hierarchy precompute is geometry-only and runs once, untimed, as in the
paper).  Prints ONE JSON line on stdout; progress goes to stderr.

    python bench.py [--gpus 1] [--steps 5] [--warmup 2]
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def measured_traffic():
    """HBM traffic per launch of the dominant kernel (every launch level, and
    per level) from the committed counter summary, or (None, {}) when the
    kernel source changed since the counters were taken."""
    import hashlib
    import re
    path = os.path.join(ROOT, "profiles", "traffic_gs_color_f32_torus1M.md")
    src = os.path.join(ROOT, "paper_2104_13755_amd", "csrc", "kernels.hip")
    try:
        txt = open(path).read()
        sha = hashlib.sha256(open(src, "rb").read()).hexdigest()
    except OSError:
        return None, {}
    m = re.search(r"kernels_hip_sha256: ([0-9a-f]+)", txt)
    if not m or m.group(1) != sha:
        return None, {}
    a = re.search(r"traffic_bytes_per_launch_every_level: (\d+)", txt)
    per = {int(l): float(v) for l, v in re.findall(r"traffic_bytes_per_launch_level(\d+): (\d+)", txt)}
    return (float(a.group(1)) if a else None), per


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def gpu_setup(w, n_levels):
    import torch
    from paper_2104_13755_amd.solver import Hierarchy, Solver, mesh_pattern
    t0 = time.perf_counter()
    h = Hierarchy.build(w["V"], w["F"], n_levels=n_levels)
    t_pre = time.perf_counter() - t0
    log(f"hierarchy precompute {t_pre:.1f}s sizes={h.sizes}")
    rp, ci = mesh_pattern(len(w["V"]), w["F"])
    t0 = time.perf_counter()
    S = Solver(h, rp, ci, faces=w["F"])
    t_up = time.perf_counter() - t0
    log(f"device setup {t_up:.1f}s")
    Vd = torch.tensor(w["V"], dtype=torch.float64, device="cuda")
    a, _, m = S.assemble(Vd, w["t"], want_mass=True)
    S.set_values(a)
    b = (m[:, None] * torch.tensor(w["u"], dtype=torch.float64, device="cuda")).contiguous()
    return S, h, Vd, b, dict(precompute_s=t_pre, device_setup_s=t_up)


def run_steps(S, Vd, t, b, rtol, precision, steps, use_graph):
    import torch
    infos = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        a, _, _ = S.assemble(Vd, t)
        S.set_values(a)
        x, info = S.solve(b, rtol=rtol, precision=precision, use_graph=use_graph)
        infos.append(info)
    torch.cuda.synchronize()
    return time.perf_counter() - t0, infos, x


def time_solve_only(S, b, rtol, precision, steps, use_graph):
    import torch
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        x, info = S.solve(b, rtol=rtol, precision=precision, use_graph=use_graph)
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / steps, info


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def host_threads():
    """Threads this process may use: its CPU affinity, at most 16 (the share
    of one GPU's host)."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def cpu_baseline(w, n_levels, rtol):
    """The oracle, untouched, on the same workload: its own hierarchy (untimed
    setup, as the paper excludes precompute), then one timed step = assembly +
    Galerkin refresh + coarsest Cholesky + FP64 solve to rtol, once with the
    host's threads available to its numerical libraries and once with one."""
    from threadpoolctl import threadpool_limits
    from oracle import assemble as AS, vcycle as OV, hierarchy as OH
    nthr = host_threads()
    t0 = time.perf_counter()
    with threadpool_limits(limits=1):
        Ps, _, _ = OH.prolongations(w["V"], w["F"], n_levels=n_levels)
        A, L, m = AS.system(w["V"], w["F"], w["t"])
        S = OV.Solver(Ps, A)
        b = m[:, None] * w["u"]
    log(f"oracle setup {time.perf_counter() - t0:.1f}s")
    runs = {}
    for threads in (nthr, 1):
        with threadpool_limits(limits=threads):
            t1 = time.perf_counter()
            A, L, m = AS.system(w["V"], w["F"], w["t"])
            S.set_values(A)
            x, cycles, hist = S.solve(b, rtol, max_cycles=500)
            runs[threads] = (time.perf_counter() - t1, int(cycles))
        log(f"oracle step with {threads} thread(s): {runs[threads][0]:.1f}s cycles={cycles}")
    dt, cycles = runs[nthr]
    return dict(value=1.0 / dt, unit="solves/s", cores=nthr, kind="oracle",
                sample="one full step (assembly, Galerkin refresh, Cholesky, FP64 solve of the 3-RHS system to "
                       "1e-8) on the full 1M-vertex workload",
                threads_note=f"{nthr} threads allowed to the oracle's BLAS/LAPACK calls (the dense coarsest "
                             "factor and solves); its sparse products and Gauss-Seidel sweeps (scipy) run on one",
                cpu_model=cpu_model(), host_threads=nthr, step_s=dt, cycles=cycles,
                single_thread={"value": 1.0 / runs[1][0], "step_s": runs[1][0], "cycles": runs[1][1]})


def build_solvers(meshes, threads=16):
    """Hierarchies (host precompute, in parallel threads: the C ABI releases
    the interpreter lock) and device solvers for a list of workload dicts."""
    import torch
    from concurrent.futures import ThreadPoolExecutor
    from paper_2104_13755_amd.solver import Hierarchy, Solver, mesh_pattern
    t0 = time.perf_counter()
    with ThreadPoolExecutor(max_workers=threads) as ex:
        hs = list(ex.map(lambda w: Hierarchy.build(w["V"], w["F"], n_levels=w.get("n_levels", 0)), meshes))
    t_pre = time.perf_counter() - t0
    out = []
    for w, h in zip(meshes, hs):
        rp, ci = mesh_pattern(len(w["V"]), w["F"])
        S = Solver(h, rp, ci, faces=w["F"])
        Vd = torch.tensor(w["V"], dtype=torch.float64, device="cuda")
        a, _, m = S.assemble(Vd, w["t"], want_mass=True)
        S.set_values(a)
        out.append((S, h, Vd, m))
    return out, t_pre


def bench_batch(args):
    """64 meshes (20k-300k vertices, 1-3 RHS) in one persistent launch."""
    import torch
    import synth
    from paper_2104_13755_amd.batch import BatchSolver
    meshes = synth.workload_c3()
    log(f"batch: {len(meshes)} meshes, {sum(len(w['V']) for w in meshes)} vertices")
    built, t_pre = build_solvers(meshes)
    log(f"batch: hierarchies {t_pre:.1f}s")
    bs = [torch.tensor(w["b"], dtype=torch.float64, device="cuda") for w in meshes]
    # unbatched reference: the meshes one after another
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    cyc_u = []
    for (S, _, _, _), b in zip(built, bs):
        _, info = S.solve(b, rtol=1e-8, precision="fp32ir")
        cyc_u.append(info["cycles"])
    torch.cuda.synchronize()
    t_unbatched = time.perf_counter() - t0
    B = BatchSolver([s[0] for s in built], cache_file=args.tune_cache)
    B.solve(bs, rtol=1e-8)
    shape = B.autotune(budget_ms=15000) if args.autotune else B.shape()
    for _ in range(args.warmup):
        B.solve(bs, rtol=1e-8)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        xs, infos, _ = B.solve(bs, rtol=1e-8)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / args.steps
    worst = max(max(i["rel_res"]) for i in infos)
    n_tot = sum(len(w["V"]) for w in meshes)
    print(json.dumps({
        "metric": "batched V-cycle solves/s (64 meshes, 20k-300k vertices, 1-3 RHS, rel residual 1e-8, FP32+FP64 IR, one persistent launch)",
        "value": len(meshes) / dt, "unit": "solves/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": dt * 1e3, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32/f64", "data": "synthetic",
        "config": {"workload": "64 seeded meshes (icospheres, tori, discs), N~U[20k,300k], t~logU[1e-4,1e-1]",
                   "vertices": n_tot, "shape": shape},
        "unbatched_solves_per_s": len(meshes) / t_unbatched, "max_rel_res": worst,
        "cycles": [i["cycles"] for i in infos], "cycles_unbatched": cyc_u,
        "precompute_s": t_pre}), flush=True)


def bench_grad(args):
    """Forward + adjoint backward of l = w^T u through the heat step on the
    655,362-vertex icosphere."""
    import torch
    import synth
    from paper_2104_13755_amd.autograd import HeatProblem, HeatSolve
    w = synth.workload_c4(level=8)
    t0 = time.perf_counter()
    P = HeatProblem(w["V"], w["F"], rtol=1e-8)
    log(f"grad: setup {time.perf_counter() - t0:.1f}s sizes={P.hier.sizes}")
    b = torch.tensor(w["b"][:, 0], dtype=torch.float64, device="cuda")
    wt = torch.tensor(w["w"], dtype=torch.float64, device="cuda")
    s0 = torch.ones(P.n, dtype=torch.float64, device="cuda")

    def step():
        tt = torch.tensor(w["t"], dtype=torch.float64, device="cuda", requires_grad=True)
        ss = s0.clone().requires_grad_(True)
        bb = b.clone().requires_grad_(True)
        u = HeatSolve.apply(bb, tt, ss, P)
        (wt * u).sum().backward()
        return tt.grad
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        g = step()
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / args.steps
    print(json.dumps({
        "metric": "differentiable heat solve: forward + adjoint backward steps/s (655,362-vertex icosphere, rel residual 1e-8)",
        "value": 1.0 / dt, "unit": "steps/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": dt * 1e3, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64", "data": "synthetic",
        "config": {"workload": "icosphere L8, t = mean edge^2, 16 unit sources, loss w^T u",
                   "levels": P.hier.sizes}, "dl_dt": float(g)}), flush=True)


def bench_pcg(args):
    """Conjugate gradients preconditioned by one symmetric V-cycle on the
    benchmark system (1M-vertex torus, 3 RHS, 7 levels, rtol 1e-8): the same
    step as the headline (assembly + Galerkin refresh + Cholesky + solve)
    with PCG in place of plain cycles."""
    import torch
    import synth
    rtol = 1e-8
    w = synth.workload_c2(*args.size)
    S, h, Vd, b, setup = gpu_setup(w, 7)

    def step(prec):
        a, _, _ = S.assemble(Vd, w["t"])
        S.set_values(a)
        return S.pcg(b, rtol=rtol, precision=prec)
    res = {}
    for prec in ("fp32ir", "fp64"):
        for _ in range(args.warmup):
            step(prec)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            x, info = step(prec)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / args.steps
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            S.pcg(b, rtol=rtol, precision=prec)
        torch.cuda.synchronize()
        so = (time.perf_counter() - t0) / args.steps
        res[prec] = dict(value=1.0 / dt, ms_per_step=dt * 1e3, iterations=info["iterations"],
                         rel_res=info["rel_res"], solve_only_per_s=1.0 / so)
        log(f"pcg {prec}: {dt * 1e3:.2f} ms/step iterations={info['iterations']} res={max(info['rel_res']):.2e}")
    print(json.dumps({
        "metric": "V-cycle-preconditioned CG solves/s at 1M verts to rel residual 1e-8 (FP32 V-cycle preconditioner, FP64 CG)",
        "value": res["fp32ir"]["value"], "unit": "solves/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": res["fp32ir"]["ms_per_step"], "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32/f64", "data": "synthetic",
        "config": {"workload": f"{w['name']} torus R=1 r=0.3 jitter 0.2, A=M+1e-2 L, 3 RHS b=M X, "
                               "7 levels, mu 2/2 (symmetric V-cycle), rtol 1e-8 on the CG residual",
                   "vertices": len(w["V"]), "levels": h.sizes, "rhs": 3},
        "fp32_preconditioner": res["fp32ir"], "fp64_preconditioner": res["fp64"]}), flush=True)


def bench_jacobi(args):
    """Damped Jacobi relaxation (per-level factor 2 / (1 + lambda_l)) in place of multicolor
    Gauss-Seidel on the benchmark system: plain V-cycle solves and
    V-cycle-preconditioned CG, both with FP32 cycles (same step as the
    headline: assembly + Galerkin refresh + Cholesky + solve)."""
    import torch
    import synth
    rtol = 1e-8
    w = synth.workload_c2(*args.size)
    S, h, Vd, b, setup = gpu_setup(w, 7)
    S.set_smoother("jacobi")

    def step(kind):
        a, _, _ = S.assemble(Vd, w["t"])
        S.set_values(a)
        if kind == "cycles":
            x, info = S.solve(b, rtol=rtol, precision="fp32ir", max_cycles=400)
            return info["cycles"], info["rel_res"]
        x, info = S.pcg(b, rtol=rtol, precision="fp32ir", max_iters=400)
        return info["iterations"], info["rel_res"]
    res = {}
    for kind in ("cycles", "pcg"):
        for _ in range(args.warmup):
            step(kind)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            its, rr = step(kind)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / args.steps
        res[kind] = dict(value=1.0 / dt, ms_per_step=dt * 1e3, iterations=its, rel_res=rr)
        log(f"jacobi {kind}: {dt * 1e3:.2f} ms/step iterations={its} res={max(rr):.2e}")
    print(json.dumps({
        "metric": "damped-Jacobi V-cycle solves/s at 1M verts to rel residual 1e-8 (FP32 cycles + FP64 refinement)",
        "value": res["cycles"]["value"], "unit": "solves/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": res["cycles"]["ms_per_step"], "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32/f64", "data": "synthetic",
        "config": {"workload": f"{w['name']} torus R=1 r=0.3 jitter 0.2, A=M+1e-2 L, 3 RHS b=M X, "
                               "7 levels, damped Jacobi omega_l = 2/(1+lambda_l), mu 2/2, rtol 1e-8",
                   "vertices": len(w["V"]), "levels": h.sizes, "rhs": 3},
        "omega_per_level": [S.jacobi_omega(l) for l in range(len(h.sizes) - 1)],
        "cycles": res["cycles"], "pcg": res["pcg"]}), flush=True)


def bench_split(args):
    """Split Galerkin (App. E) on the benchmark mesh: a sweep of t over 10
    values in [1e-3, 1e-1] (A = M + t L), each solved to 1e-8 with FP32
    cycles; the levels of L and M are kept once, so a new t costs one axpby
    per level plus the coarsest factorization, against re-assembly and the
    Galerkin products."""
    import torch
    import synth
    rtol = 1e-8
    w = synth.workload_c2(*args.size)
    S, h, Vd, b, setup = gpu_setup(w, 7)
    _, lv, m = S.assemble(Vd, w["t"], want_l=True, want_mass=True)
    rp = torch.tensor(S.rowptr, dtype=torch.int64, device="cuda")
    ci = torch.tensor(S.cols, dtype=torch.int64, device="cuda")
    rows = torch.repeat_interleave(torch.arange(len(rp) - 1, device="cuda"), rp[1:] - rp[:-1])
    mv = torch.where(rows == ci, m[rows], torch.zeros_like(lv))
    S.split_prepare(lv, mv)
    ts = [float(x) for x in np.logspace(-3, -1, 10)]

    def sweep(split):
        cyc = 0
        for t in ts:
            if split:
                S.split_combine(t, 1.0)
            else:
                a, _, _ = S.assemble(Vd, t)
                S.set_values(a)
            x, info = S.solve(b, rtol=rtol, precision="fp32ir")
            cyc += info["cycles"]
        return cyc
    res = {}
    for split in (True, False):
        for _ in range(max(1, args.warmup // 5)):
            sweep(split)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        reps = max(1, args.steps // 10)
        for _ in range(reps):
            cyc = sweep(split)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / (reps * len(ts))
        res["split" if split else "full"] = dict(value=1.0 / dt, ms_per_step=dt * 1e3, cycles_per_sweep=cyc)
        log(f"split={split}: {dt * 1e3:.2f} ms per t, {cyc} cycles per sweep")
    # refresh cost alone
    torch.cuda.synchronize(); t0 = time.perf_counter()
    for t in ts:
        S.split_combine(t, 1.0)
    torch.cuda.synchronize(); t_comb = (time.perf_counter() - t0) / len(ts)
    t0 = time.perf_counter()
    for t in ts:
        a, _, _ = S.assemble(Vd, t)
        S.set_values(a)
    torch.cuda.synchronize(); t_full = (time.perf_counter() - t0) / len(ts)
    print(json.dumps({
        "metric": "parameter sweep solves/s at 1M verts (A = M + t L, 10 values of t, rel residual 1e-8, split Galerkin)",
        "value": res["split"]["value"], "unit": "solves/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": res["split"]["ms_per_step"], "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32/f64", "data": "synthetic",
        "config": {"workload": f"{w['name']} torus, 3 RHS b=M X, 7 levels, t in logspace(-3,-1,10), FP32 cycles",
                   "vertices": len(w["V"]), "levels": h.sizes, "rhs": 3},
        "split": res["split"], "full_refresh": res["full"],
        "refresh_ms": {"split_combine": t_comb * 1e3, "assemble_and_galerkin": t_full * 1e3}}), flush=True)


def bench_smooth(args):
    """Data smoothing with the squared Laplacian energy (Sec. Applications):
    A(alpha) = alpha L M^{-1} L + (1 - alpha) M (2-ring pattern) on the
    benchmark mesh, b = (1 - alpha) M f, a sweep over 5 values of alpha in
    [1e-4, 1e-2] with split Galerkin levels (App. E), each solved to 1e-8
    with V-cycle-preconditioned CG, and with plain FP32 cycles (capped at 200;
    the paper notes slow convergence of its prolongation on higher-order
    problems, Sec. "Limitations & Future Work").  L comes from
    the device assembly; L M^{-1} L is formed once on the host (setup)."""
    import torch
    import scipy.sparse as sp
    import synth
    from paper_2104_13755_amd.solver import Hierarchy, Solver, mesh_pattern
    rtol = 1e-8
    w = synth.workload_c2(*args.size)
    n = len(w["V"])
    t0 = time.perf_counter()
    h = Hierarchy.build(w["V"], w["F"], n_levels=7)
    rp, ci = mesh_pattern(n, w["F"])
    S1 = Solver(h, rp, ci, faces=w["F"])
    Vd = torch.tensor(w["V"], dtype=torch.float64, device="cuda")
    _, lv, m = S1.assemble(Vd, 1.0, want_l=True, want_mass=True)
    L = sp.csr_matrix((lv.cpu().numpy(), ci, rp), shape=(n, n))
    mh = m.cpu().numpy()
    Q = (L @ sp.diags(1.0 / mh) @ L).tocsr()
    Q.sort_indices()
    del S1
    rows = np.repeat(np.arange(n), np.diff(Q.indptr))
    Mv = np.where(rows == Q.indices, mh[rows], 0.0)
    S = Solver(h, Q.indptr, Q.indices)
    t_setup = time.perf_counter() - t0
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    S.split_prepare(torch.tensor(Q.data, device="cuda"), torch.tensor(Mv, device="cuda"))
    torch.cuda.synchronize()
    t_prep = time.perf_counter() - t0
    log(f"smooth: setup {t_setup:.1f}s, 2-ring nnz/row {Q.nnz / n:.1f}, split prepare {t_prep * 1e3:.1f} ms")
    f = torch.tensor(np.random.default_rng(5).uniform(-1, 1, (n, 1)), device="cuda")
    md = m[:, None]
    alphas = [float(a) for a in np.logspace(-4, -2, 5)]

    def sweep(kind):
        its = []
        for a in alphas:
            S.split_combine(a, 1.0 - a)
            b = ((1.0 - a) * md * f).contiguous()
            if kind == "cycles":
                info = S.solve(b, rtol=rtol, precision="fp32ir", max_cycles=200, raise_on_error=False)[1]
                its.append((info["cycles"], max(info["rel_res"])))
            else:
                info = S.pcg(b, rtol=rtol, precision="fp32ir", max_iters=400)[1]
                its.append((info["iterations"], max(info["rel_res"])))
        return its
    res = {}
    for kind in ("pcg", "cycles"):
        sweep(kind)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        reps = max(1, args.steps // 10)
        for _ in range(reps):
            its = sweep(kind)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / (reps * len(alphas))
        res[kind] = dict(value=1.0 / dt, ms_per_step=dt * 1e3, iterations=its)
        log(f"smooth {kind}: {dt * 1e3:.2f} ms per alpha, iterations {its}")
    print(json.dumps({
        "metric": "Bilaplacian data smoothing solves/s at 1M verts (5 values of alpha, rel residual 1e-8, V-cycle-preconditioned CG)",
        "value": res["pcg"]["value"], "unit": "solves/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": res["pcg"]["ms_per_step"], "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32/f64", "data": "synthetic",
        "config": {"workload": f"{w['name']} torus, A = alpha L M^-1 L + (1-alpha) M (2-ring), b = (1-alpha) M f, "
                               "alpha in logspace(-4,-2,5), 1 RHS, FP32 cycles",
                   "vertices": n, "levels": h.sizes, "nnz_per_row": Q.nnz / n},
        "pcg": res["pcg"], "cycles": res["cycles"], "split_prepare_ms": t_prep * 1e3}), flush=True)


def bench_frames(args):
    """Time-varying A: 2M-vertex height-field disc, per-frame edge weights and
    t, on-device re-assembly + Galerkin over 8 levels + Cholesky + FP32/FP64-IR
    solve to 1e-8."""
    import torch
    import synth
    mesh = synth.workload_c5_mesh()
    mesh["t"] = 1e-2
    built, t_pre = build_solvers([mesh])
    S, h, Vd, m = built[0]
    log(f"frames: precompute {t_pre:.1f}s sizes={h.sizes}")
    b = (m[:, None] * torch.tensor(mesh["u"], dtype=torch.float64, device="cuda")).contiguous()
    frames = [synth.workload_c5_frame(mesh, k) for k in range(args.frames)]
    ws = [torch.tensor(f["w"].astype(np.float32), device="cuda") for f in frames]

    def frame(k):
        a, _, _ = S.assemble(Vd, frames[k]["t"], edge_w=ws[k])
        S.set_values(a)
        return S.solve(b, rtol=1e-8, precision="fp32ir")[1]
    for k in range(min(args.warmup, len(frames))):
        frame(k)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    cyc = []
    for k in range(len(frames)):
        info = frame(k)
        cyc.append(info["cycles"])
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / len(frames)
    print(json.dumps({
        "metric": "time-varying A frames/s (2M-vertex disc, per-frame re-Galerkin over 8 levels + FP32/FP64-IR solve to 1e-8)",
        "value": 1.0 / dt, "unit": "frames/s", "n_gpus": 1, "steps": len(frames), "warmup": args.warmup,
        "ms_per_step": dt * 1e3, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32/f64", "data": "synthetic",
        "config": {"workload": mesh["name"] + " z=0.1 sin(3x)cos(2y), w_e in [0.5,2], t_k~logU[1e-3,1e-1]",
                   "levels": h.sizes}, "cycles": cyc}), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--size", type=int, nargs=2, default=(1000, 1000))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--graph", type=int, default=0)
    ap.add_argument("--profile-kind", default="gs")
    ap.add_argument("--workload", default="torus", choices=["torus", "batch", "grad", "frames", "pcg", "jacobi", "split", "smooth"])
    ap.add_argument("--frames", type=int, default=100)
    ap.add_argument("--autotune", type=int, default=1)
    ap.add_argument("--tune-cache", default=None)
    ap.add_argument("--pmc-probe", action="store_true",
                    help="short run for hardware counters: a 256 MiB copy (calibration), then 3 mixed cycles")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "bench.py measures one GPU; --gpus above 1 is not supported",
                          "n_gpus": args.gpus}))
        sys.exit(2)
    import torch
    import synth
    if not torch.cuda.is_available():
        print(json.dumps({"error": "no GPU visible"}))
        sys.exit(1)
    if args.workload == "batch":
        return bench_batch(args)
    if args.workload == "grad":
        return bench_grad(args)
    if args.workload == "frames":
        return bench_frames(args)
    if args.workload == "pcg":
        return bench_pcg(args)
    if args.workload == "jacobi":
        return bench_jacobi(args)
    if args.workload == "split":
        return bench_split(args)
    if args.workload == "smooth":
        return bench_smooth(args)
    rtol = 1e-8
    n_levels = 7
    w = synth.workload_c2(*args.size)
    log(f"workload {w['name']} n={len(w['V'])} faces={len(w['F'])}")
    S, h, Vd, b, setup = gpu_setup(w, n_levels)
    use_graph = bool(args.graph)
    if args.pmc_probe:
        src = torch.ones(32 * 1024 * 1024, dtype=torch.float64, device="cuda")   # 256 MiB
        dst = torch.empty_like(src)
        for _ in range(3):
            torch.mul(src, 1.0, out=dst)   # plain streaming kernel: reads and writes 256 MiB
        torch.cuda.synchronize()
        S.solve(b, fixed_cycles=3, precision="fp32ir")
        torch.cuda.synchronize()
        print(json.dumps({"pmc_probe": True, "copy_bytes_read": src.numel() * 8,
                          "copy_bytes_written": dst.numel() * 8, "cycles": 3}), flush=True)
        return

    # warmup both precisions
    for prec in ("fp32ir", "fp64"):
        run_steps(S, Vd, w["t"], b, rtol, prec, args.warmup, use_graph)
    # timed region: mixed precision, no instrumentation
    t_mixed, infos_m, x_m = run_steps(S, Vd, w["t"], b, rtol, "fp32ir", args.steps, use_graph)
    log(f"mixed: {t_mixed / args.steps * 1e3:.2f} ms/step cycles={infos_m[-1]['cycles']} res={max(infos_m[-1]['rel_res']):.2e}")
    # the same steps again with every launch of the dominant kernel timed by
    # start/stop events stamped by its own dispatch (per-level split too)
    S.profile_enable(args.profile_kind, -1)
    t_prof, _, _ = run_steps(S, Vd, w["t"], b, rtol, "fp32ir", args.steps, use_graph)
    prof = S.profile_read()
    # per level: every level relaxed by per-color launches (above the tail)
    launch_levels = list(range(S.tail_first(3, "fp32ir")))
    prof_lv = {}
    for l in launch_levels:
        S.profile_enable(args.profile_kind, l)
        run_steps(S, Vd, w["t"], b, rtol, "fp32ir", 2, use_graph)
        prof_lv[l] = S.profile_read()
    S.profile_enable(None)
    # latency bound of a launch with each level's grid: an empty kernel and a
    # kernel with the relaxation's dependent chain (index, gather, store)
    floors = {l: (S.launch_floor("empty", l), S.launch_floor("chain", l)) for l in launch_levels}
    t_fp64, infos_d, x_d = run_steps(S, Vd, w["t"], b, rtol, "fp64", args.steps, use_graph)
    log(f"fp64: {t_fp64 / args.steps * 1e3:.2f} ms/step cycles={infos_d[-1]['cycles']} res={max(infos_d[-1]['rel_res']):.2e}")
    so_m, _ = time_solve_only(S, b, rtol, "fp32ir", args.steps, use_graph)
    so_d, _ = time_solve_only(S, b, rtol, "fp64", args.steps, use_graph)
    # one more step per precision with an event at every change of phase
    # (the paper's Tab. "profile" buckets), outside the timed region
    phases = {}
    for prec in ("fp32ir", "fp64"):
        a, _, _ = S.assemble(Vd, w["t"])
        S.set_values(a)
        _, inf = S.solve(b, rtol=rtol, precision=prec, timed=True)
        phases[prec] = {k: round(v, 3) for k, v in inf["ms_phase"].items()}
        log(f"phases {prec}: {phases[prec]}")
    diff = float(torch.linalg.norm(x_m - x_d) / torch.linalg.norm(x_d))

    def summary(p):
        ach = p["bytes"] / (p["ms"] * 1e-3) / 1e9 if p["ms"] > 0 else None
        return {"achieved": ach, "frac": ach / HBM_PEAK_GBS if ach else None, "launches": p["launches"],
                "avg_launch_us": p["ms"] * 1e3 / max(1, p["launches"]),
                "algorithmic_bytes_per_launch": p["bytes"] / max(1, p["launches"])}
    traffic_all, traffic_lv = measured_traffic() if args.profile_kind == "gs" else (None, {})
    top = summary(prof)
    roofline = {"bound": "hbm", "achieved": top["achieved"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": top["frac"], "traffic": traffic_all,
                "kernel": "k_gs_color_w<3, float> / k_gs_color<3, float> (multicolor Gauss-Seidel, FP32 cycles, "
                          "every level relaxed by per-color launches)"
                          if args.profile_kind == "gs" else f"{args.profile_kind} (every level)",
                "launches": top["launches"], "avg_launch_us": top["avg_launch_us"],
                "algorithmic_bytes_per_launch": top["algorithmic_bytes_per_launch"],
                "bytes_rule": "per sweep z(s+4) + 4(n+1) + 3kns: z matrix entries incl. diagonal, n rows, "
                              "s = 4 B values, k = 3 right-hand sides, x gathers counted once; "
                              "a color launch counts its rows' share",
                "measured": "dispatch-stamped HIP events on the launch stream, every launch of the kernel "
                            "in a second pass of the same timed steps",
                "levels": {str(l): dict(summary(p), traffic=traffic_lv.get(l), floor_empty_us=floors[l][0],
                                        floor_chain_us=floors[l][1],
                                        latency_frac=floors[l][1] / summary(p)["avg_launch_us"])
                           for l, p in prof_lv.items()},
                "latency_rule": "floor_chain_us: back-to-back launches with the level's widest color grid whose "
                                "threads load an index, the value it points to, and store it; latency_frac = "
                                "that floor / the relaxation launch's average time (events)"}
    value = args.steps / t_mixed
    out = {
        "metric": "V-cycle solves/s + HBM GB/s at 1M verts to rel residual 1e-8, mixed vs FP64",
        "value": value, "unit": "solves/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": t_mixed / args.steps * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32/f64", "data": "synthetic",
        "config": {"workload": f"{w['name']} torus R=1 r=0.3 jitter 0.2, A=M+1e-2 L, 3 RHS b=M X, "
                               f"{n_levels} levels, mu 2/2, rtol 1e-8",
                   "vertices": len(w["V"]), "levels": h.sizes, "rhs": 3, "graph": use_graph},
        "fp64": {"value": args.steps / t_fp64, "ms_per_step": t_fp64 / args.steps * 1e3,
                 "cycles": infos_d[-1]["cycles"], "rel_res": infos_d[-1]["rel_res"],
                 "solve_only_per_s": 1.0 / so_d},
        "mixed": {"cycles": infos_m[-1]["cycles"], "rel_res": infos_m[-1]["rel_res"],
                  "solve_only_per_s": 1.0 / so_m, "rel_diff_vs_fp64": diff},
        "setup": setup,
        "phases_ms": dict(phases, buckets="prepare = Galerkin levels + coarsest factor (the value refresh); "
                                           "relax = Gauss-Seidel launches + one-workgroup tail; transfer = "
                                           "residuals feeding restriction, restriction, prolongation; norm = "
                                           "level-0 FP64 residual + column norms; other = refinement glue, "
                                           "set-up of the solve"),
        "roofline": roofline,
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(w, n_levels, rtol)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
