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
import math
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


# ------------------------------------------------------------------
# Summaries of rocprofv3 output (run on the machine that profiled, the
# markdown goes to profiles/).  The dominant kernel's launches are told apart
# by their position: every FP32 cycle launches, per relaxed level l in order,
# mu_pre * colors_l pre-relaxation launches, then the post-relaxation ones in
# reverse level order; a step may end with the run-ahead prefix of one more
# cycle (level-0 pre-relaxation launches only).
DOMINANT = r"k_gs_color(_w)?<3, float>"


def _cycle_levels(colors, mu_pre=2, mu_post=2):
    """Level of each dominant launch of one cycle, in launch order."""
    seq = []
    for l, c in enumerate(colors):
        seq += [l] * (mu_pre * c)
    for l in reversed(range(len(colors))):
        seq += [l] * (mu_post * colors[l])
    return seq


def _step_levels(n, colors):
    """Levels of the n dominant launches of one step (whole cycles, then a
    pre-relaxation prefix)."""
    cyc = _cycle_levels(colors)
    full, rest = divmod(n, len(cyc))
    return cyc * full + cyc[:rest]


def _step_groups(n, colors):
    """Relaxation call (one level's pre- or post-relaxation of one cycle) of
    each of the n dominant launches of one step, numbered in launch order."""
    cyc, g = [], 0
    for l, c in enumerate(colors):
        cyc += [g] * (2 * c)
        g += 1
    for l in reversed(range(len(colors))):
        cyc += [g] * (2 * colors[l])
        g += 1
    full, rest = divmod(n, len(cyc))
    return [x + 2 * len(colors) * (i // len(cyc)) for i, x in enumerate(cyc * full + cyc[:rest])]


def _read_csv(path):
    import csv
    with open(path, newline="") as f:
        return list(csv.DictReader(f))


def kernel_table(d, top=24):
    """Markdown table of the kernels of a rocprofv3 --stats run (directory d)."""
    import re
    stats = _read_csv(os.path.join(d, "run_kernel_stats.csv"))
    tot = sum(float(r["TotalDurationNs"]) for r in stats)
    out = [f"Total kernel time: {tot / 1e6:.1f} ms over {sum(int(r['Calls']) for r in stats)} dispatches.", "",
           "| kernel | calls | total ms | avg us | min us | max us | % |", "|---|---|---|---|---|---|---|"]
    for r in sorted(stats, key=lambda r: -float(r["TotalDurationNs"]))[:top]:
        name = re.sub(r"^(void )?smg::\(anonymous namespace\)::", "", r["Name"]).split("(")[0]
        out.append(f"| `{name}` | {r['Calls']} | {float(r['TotalDurationNs']) / 1e6:.2f} | "
                   f"{float(r['AverageNs']) / 1e3:.2f} | {float(r['MinNs']) / 1e3:.2f} | "
                   f"{float(r['MaxNs']) / 1e3:.2f} | {float(r['TotalDurationNs']) / tot * 100:.1f} |")
    return "\n".join(out)


def trace_summary(d, bench_json):
    """Markdown summary of `rocprofv3 --kernel-trace --stats` of a bench run
    (directory d, files run_*) next to the JSON line of a plain run with the
    same --steps / --warmup: per-kernel table, the dominant kernel's average
    per pass of the bench, and per level its kernel time and its time per
    launch inside each relaxation call (first start to last end of the call's
    back-to-back launches / launches: what the bench's events measure)."""
    import re
    b = json.loads(open(bench_json).read().strip().splitlines()[-1])
    if b.get("config", {}).get("launch_mode_ms_per_step"):
        raise ValueError("the launch mode was chosen by timing (extra steps): profile with --graph 0")
    roof = b["roofline"]
    steps, warm = b["steps"], b["warmup"]
    colors = [roof["levels"][str(l)]["colors"] for l in range(len(roof["levels"]))]
    tr = _read_csv(os.path.join(d, "run_kernel_trace.csv"))
    tr.sort(key=lambda r: int(r["Start_Timestamp"]))
    dom = [(int(r["Start_Timestamp"]), int(r["End_Timestamp"])) for r in tr if re.search(DOMINANT, r["Kernel_Name"])]
    per_step = roof["launches"] // steps
    passes = [("warmup (FP32 cycles)", warm), ("timed steps (no instrumentation)", steps),
              ("event-timed pass (the bench line's figure)", steps)]
    passes += [(f"level-{l} event pass", 2) for l in range(len(colors))]
    passes += [("solve-only timing", steps), ("phase-timed step", 1)]

    def per_level(seg, k):
        acc = {}
        for st in range(k):
            part = seg[st * per_step:(st + 1) * per_step]
            lv, gr = _step_levels(len(part), colors), _step_groups(len(part), colors)
            calls = {}
            for (t0, t1), l, g in zip(part, lv, gr):
                a = acc.setdefault(l, [0.0, 0, 0.0, 0])
                a[0] += (t1 - t0) * 1e-3
                a[1] += 1
                c = calls.setdefault(g, [l, t0, t1, 0])
                c[2] = t1
                c[3] += 1
            for l, t0, t1, n in calls.values():
                acc[l][2] += (t1 - t0) * 1e-3
                acc[l][3] += n
        return acc

    rows, i, lev = [], 0, {}
    for name, k in passes:
        seg = dom[i:i + k * per_step]
        if not seg:
            break
        avg = sum(t1 - t0 for t0, t1 in seg) * 1e-3 / len(seg)
        rows.append(f"| {name} | {k} | {len(seg)} | {avg:.3f} |")
        if name.startswith("timed") or name.startswith("event-timed"):
            lev[name.split(" ")[0]] = (per_level(seg, k), avg)
        i += k * per_step
    lines = [kernel_table(d)]
    lines += ["", f"Dominant kernel (`{DOMINANT}`, {per_step} launches per step) by pass of the bench, "
              "in trace order:", "", "| pass | steps | launches | avg kernel us |", "|---|---|---|---|"]
    lines += rows
    lines += ["", "Per level: kernel time per launch, and time per launch inside each relaxation call (first "
              "start to last end / launches), from the trace; the plain run's event figure beside them:", "",
              "| level | colors | pass | launches | kernel us | per launch in calls us | plain run's events us | "
              "algorithmic MB/launch | GB/s (per launch in calls) | frac |", "|---|---|---|---|---|---|---|---|---|---|"]
    for key, (acc, _) in lev.items():
        for l in sorted(acc):
            s_us, n, c_us, cn = acc[l]
            lv = roof["levels"][str(l)]
            by = lv["algorithmic_bytes_per_launch"]
            gbs = by / (c_us / cn * 1e-6) / 1e9
            lines.append(f"| {l} | {colors[l]} | {key} | {n} | {s_us / n:.3f} | {c_us / cn:.3f} | "
                         f"{lv['avg_launch_us']:.3f} | {by / 1e6:.3f} | {gbs:.0f} | {gbs / HBM_PEAK_GBS:.4f} |")
    ab = roof["algorithmic_bytes_per_launch"]
    for key, (acc, avg) in lev.items():
        c_us = sum(a[2] for a in acc.values()) / sum(a[3] for a in acc.values())
        lines.append("")
        lines.append(f"Every level, {key} pass: kernel {avg:.3f} us per launch, {c_us:.3f} us per launch inside "
                     f"relaxation calls -> {ab / (c_us * 1e-6) / 1e9:.0f} GB/s = "
                     f"{ab / (c_us * 1e-6) / 1e9 / HBM_PEAK_GBS:.4f} of 8 TB/s.")
    lines += ["", f"Plain run's bench line: {roof['avg_launch_us']:.3f} us per launch, {roof['achieved']:.0f} GB/s, "
              f"frac {roof['frac']:.4f}."]
    return "\n".join(lines)


def pmc_summary(fetch_dir, write_dir, colors):
    """HBM traffic per dominant launch from two `rocprofv3 --pmc` runs of
    `bench.py --pmc-probe` (FETCH_SIZE, then WRITE_SIZE), each scaled by what
    the counter reads for the probe's three 256 MiB streaming multiplies."""
    import re

    def per_dispatch(d, counter):
        rows = _read_csv(os.path.join(d, "run_counter_collection.csv"))
        acc = {}
        for r in rows:
            if r["Counter_Name"] != counter:
                continue
            k = int(r["Dispatch_Id"])
            acc.setdefault(k, [r["Kernel_Name"], 0.0])[1] += float(r["Counter_Value"])
        return [acc[k] for k in sorted(acc)]

    res = {}
    for counter, d in (("FETCH_SIZE", fetch_dir), ("WRITE_SIZE", write_dir)):
        disp = per_dispatch(d, counter)
        copies = [v for n, v in disp if "elementwise" in n][-3:]
        scale = 262144.0 / (sum(copies) / len(copies))          # KiB moved per copy / KiB counted
        dom = [v for n, v in disp if re.search(DOMINANT, n)]
        res[counter] = (scale, sum(copies) / len(copies), dom)
    nd = len(res["FETCH_SIZE"][2])
    levels = _step_levels(nd, colors)
    tot = [res["FETCH_SIZE"][0] * f + res["WRITE_SIZE"][0] * w
           for f, w in zip(res["FETCH_SIZE"][2], res["WRITE_SIZE"][2])]
    out = {"scale_fetch": res["FETCH_SIZE"][0], "scale_write": res["WRITE_SIZE"][0],
           "copy_fetch_kib": res["FETCH_SIZE"][1], "copy_write_kib": res["WRITE_SIZE"][1], "launches": nd,
           "all": {"fetch_kib": sum(res["FETCH_SIZE"][2]) / nd, "write_kib": sum(res["WRITE_SIZE"][2]) / nd,
                   "bytes": sum(tot) / nd * 1024}}
    for l in sorted(set(levels)):
        idx = [i for i, x in enumerate(levels) if x == l]
        out[l] = {"launches": len(idx), "fetch_kib": sum(res["FETCH_SIZE"][2][i] for i in idx) / len(idx),
                  "write_kib": sum(res["WRITE_SIZE"][2][i] for i in idx) / len(idx),
                  "bytes": sum(tot[i] for i in idx) / len(idx) * 1024}
    return out


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


def copy_bandwidth(nbytes=1 << 30, reps=10):
    """GB/s of a plain device-to-device copy (bytes read + bytes written per
    second), timed with events on torch's stream: the measured ceiling the
    roofline fractions are also quoted against."""
    import torch
    src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        dst.copy_(src)
    e1.record()
    e1.synchronize()
    gbs = 2.0 * nbytes * reps / (e0.elapsed_time(e1) * 1e-3) / 1e9
    del src, dst
    return gbs


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


def cycle_bytes(S, k, sweeps=4, s=4):
    """Algorithmic bytes of one V-cycle with FP32 values (s = 4) for k
    right-hand sides: every relaxation sweep and residual by the CSR rule
    z(s+4) + 4(n+1) + 3kns, a transfer as P's three columns and weights per
    row plus the vectors it reads and writes, the coarsest dense apply, and
    the refinement's level-0 FP64 residual."""
    L = S.num_levels
    relax = resid = transfer = 0.0
    for l in range(L - 1):
        n, z, nc = S.level_size(l), S.level_nnz(l), S.level_size(l + 1)
        csr = z * (s + 4) + 4 * (n + 1) + 3 * k * n * s
        relax += sweeps * csr
        resid += csr
        transfer += 2 * 3 * n * (4 + s) + (k * n * s + k * nc * s) + (k * nc * s + 2 * k * n * s)
    nH = S.level_size(L - 1)
    z0, n0 = S.level_nnz(0), S.level_size(0)
    return dict(relax=relax, residual=resid, transfer=transfer, coarse=nH * nH * 8.0 + 2 * k * nH * s,
                ir=z0 * (8 + 4) + 4 * (n0 + 1) + 3 * k * n0 * 8.0)


def bench_coarse(args):
    """Coarsest-level value refresh at a chosen coarsest size n_H (Galerkin
    product into it, dense Cholesky, A_H^{-1}): a two-level hierarchy of a
    jittered torus grid with about 4 n_H vertices.  Run it under rocprofv3
    --kernel-trace --stats and divide the factor and inverse kernels' time by
    the refreshes this prints."""
    import torch
    from paper_2104_13755_amd.solver import Hierarchy, Solver, mesh_pattern
    from synth.meshes import torus_grid
    a = max(8, int(round(math.sqrt(4 * args.coarse_n))))
    V, F = torus_grid(a, a, 1.0, 0.3, np.random.default_rng(3), jitter=0.2)
    h = Hierarchy.build(V, F, n_levels=2)
    rp, ci = mesh_pattern(len(V), F)
    S = Solver(h, rp, ci, faces=F)
    Vd = torch.tensor(V, dtype=torch.float64, device="cuda")
    vals, _, _ = S.assemble(Vd, 1e-2)
    refreshes = 0
    for _ in range(args.warmup):
        S.set_values(vals)
        refreshes += 1
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        S.set_values(vals)
        refreshes += 1
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / args.steps
    nH = h.sizes[-1]
    print(json.dumps({"workload": f"torus-{a}x{a}, 2 levels", "sizes": h.sizes, "n_H": nH,
                      "refreshes": refreshes, "refresh_ms": dt * 1e3,
                      "factor_flop": nH ** 3 / 3.0, "inverse_flop": 2 * nH ** 3 / 3.0}), flush=True)


def coarse_summary(runs):
    """Markdown table from rocprofv3 --stats runs of --workload coarse: list
    of (rocprof dir, JSON file) pairs."""
    factor = ("k_chol_panel", "k_chol_update", "k_zero_upper", "k_cholesky_blocked", "k_cholesky(")
    inverse = ("k_identity", "k_trinv_rows", "k_trinv_update", "k_inv_syrk", "k_tri_inverse_cols",
               "k_tri_inverse(", "k_inverse_product")
    out = ["| n_H | refreshes | factor us | factor TFLOP/s (n^3/3) | frac of 78.6 | inverse us | "
           "inverse TFLOP/s (2n^3/3) | refresh ms (wall) | factor kernels |",
           "|---|---|---|---|---|---|---|---|---|"]
    for d, js in runs:
        j = json.loads(open(js).read().strip().splitlines()[-1])
        stats = _read_csv(os.path.join(d, "run_kernel_stats.csv"))
        tf = sum(float(r["TotalDurationNs"]) for r in stats if any(k in r["Name"] for k in factor))
        ti = sum(float(r["TotalDurationNs"]) for r in stats if any(k in r["Name"] for k in inverse))
        names = sorted({r["Name"].split("::")[-1].split("(")[0] for r in stats if any(k in r["Name"] for k in factor)})
        f_us, i_us = tf / j["refreshes"] / 1e3, ti / j["refreshes"] / 1e3
        out.append(f"| {j['n_H']} | {j['refreshes']} | {f_us:.1f} | {j['factor_flop'] / f_us / 1e6:.2f} | "
                   f"{j['factor_flop'] / f_us / 1e6 / 78.6:.4f} | {i_us:.1f} | "
                   f"{j['inverse_flop'] / i_us / 1e6:.2f} | {j['refresh_ms']:.3f} | {', '.join(names)} |")
    return "\n".join(out)


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
    # roofline of the one dispatch: smoother + SpMV bytes of every cycle of
    # every mesh over the whole dispatch's time (a lower bound for those
    # kernels' own rate: the dispatch also holds transfers, coarsest solves
    # and team barriers)
    sm = tot_all = 0.0
    for (S, _, _, _), b, inf in zip(built, bs, infos):
        cb = cycle_bytes(S, b.shape[1] if b.dim() > 1 else 1)
        sm += inf["cycles"] * (cb["relax"] + cb["residual"] + cb["ir"])
        tot_all += inf["cycles"] * sum(cb.values())
    copy_gbs = copy_bandwidth()
    roof = {"bound": "hbm", "achieved": sm / dt / 1e9, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": sm / dt / 1e9 / HBM_PEAK_GBS, "traffic": None, "copy_gbs": copy_gbs,
            "frac_of_copy": sm / dt / 1e9 / copy_gbs,
            "kernel": "k_batch_solve (one persistent dispatch: every cycle of every mesh)",
            "bytes_per_batch": sm, "bytes_per_batch_all_steps": tot_all,
            "all_steps_frac": tot_all / dt / 1e9 / HBM_PEAK_GBS,
            "bytes_rule": "per cycle: 4 relaxation sweeps + 1 residual per level above the coarsest, each "
                          "z(s+4) + 4(n+1) + 3kns with s = 4, plus the level-0 FP64 residual z 12 + 4(n+1) + 24kn "
                          "of the refinement; all_steps adds transfers (P: 3 columns + weights per row, vectors) "
                          "and the coarsest dense apply n_H^2 8"}
    print(json.dumps({
        "metric": "batched V-cycle solves/s (64 meshes, 20k-300k vertices, 1-3 RHS, rel residual 1e-8, FP32+FP64 IR, one persistent launch)",
        "value": len(meshes) / dt, "unit": "solves/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": dt * 1e3, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32/f64", "data": "synthetic",
        "config": {"workload": "64 seeded meshes (icospheres, tori, discs), N~U[20k,300k], t~logU[1e-4,1e-1]",
                   "vertices": n_tot, "shape": shape},
        "unbatched_solves_per_s": len(meshes) / t_unbatched, "max_rel_res": worst,
        "cycles": [i["cycles"] for i in infos], "cycles_unbatched": cyc_u,
        "precompute_s": t_pre, "roofline": roof}), flush=True)


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
        "omega_rule": "the paper names damped Jacobi without a factor: omega_l = 2/(1 + lambda_l), lambda_l the "
                      "Rayleigh quotient of D^-1 A after 20 power steps from a fixed golden-ratio start vector "
                      "(a fixed 2/3 diverged on this torus, whose levels have lambda 1.9 to 2.8)",
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
    ap.add_argument("--graph", type=int, default=-1,
                    help="1: replay each cycle from a captured hipGraph, 0: eager launches, -1: the faster of the two")
    ap.add_argument("--profile-kind", default="gs_group")
    ap.add_argument("--workload", default="torus",
                    choices=["torus", "batch", "grad", "frames", "pcg", "jacobi", "split", "smooth", "coarse"])
    ap.add_argument("--coarse-n", type=int, default=1960, help="coarsest size of --workload coarse")
    ap.add_argument("--coarse-summary", nargs="+", metavar="DIR=JSON",
                    help="print the table of rocprofv3 --stats runs of --workload coarse")
    ap.add_argument("--frames", type=int, default=100)
    ap.add_argument("--autotune", type=int, default=1)
    ap.add_argument("--tune-cache", default=None)
    ap.add_argument("--stats-table", metavar="ROCPROF_DIR",
                    help="print the kernel table of a rocprofv3 --stats run")
    ap.add_argument("--trace-summary", nargs=2, metavar=("ROCPROF_DIR", "BENCH_JSON"),
                    help="print the markdown summary of a rocprofv3 --kernel-trace --stats run of this bench")
    ap.add_argument("--pmc-summary", nargs=3, metavar=("FETCH_DIR", "WRITE_DIR", "PROBE_JSON"),
                    help="print the traffic summary of two rocprofv3 --pmc runs of --pmc-probe")
    ap.add_argument("--pmc-probe", action="store_true",
                    help="short run for hardware counters: a 256 MiB copy (calibration), then 3 mixed cycles")
    args = ap.parse_args()
    if args.stats_table:
        print(kernel_table(args.stats_table))
        return
    if args.coarse_summary:
        print(coarse_summary([tuple(x.split("=", 1)) for x in args.coarse_summary]))
        return
    if args.trace_summary:
        print(trace_summary(*args.trace_summary))
        return
    if args.pmc_summary:
        import hashlib
        probe = json.loads(open(args.pmc_summary[2]).read().strip().splitlines()[-1])
        r = pmc_summary(args.pmc_summary[0], args.pmc_summary[1], probe["colors"])
        src = os.path.join(ROOT, "paper_2104_13755_amd", "csrc", "kernels.hip")
        lines = [f"Calibration on the multiply: FETCH_SIZE reads {r['copy_fetch_kib']:.0f} KiB for 262144 KiB read "
                 f"(scale {r['scale_fetch']:.4f}); WRITE_SIZE reads {r['copy_write_kib']:.0f} KiB for 262144 KiB "
                 f"written (scale {r['scale_write']:.4f}).  Traffic = scale_fetch * FETCH_SIZE + scale_write * "
                 "WRITE_SIZE.", "",
                 f"Colors per relaxed level: {probe['colors']}; {r['launches']} dominant launches in "
                 f"{probe['cycles']} cycles.", "",
                 "| launches | count | FETCH_SIZE KiB/launch | WRITE_SIZE KiB/launch | traffic MB/launch |",
                 "|---|---|---|---|---|",
                 f"| every level | {r['launches']} | {r['all']['fetch_kib']:.1f} | {r['all']['write_kib']:.1f} | "
                 f"{r['all']['bytes'] / 1e6:.3f} |"]
        for l in range(len(probe["colors"])):
            lines.append(f"| level {l} | {r[l]['launches']} | {r[l]['fetch_kib']:.1f} | {r[l]['write_kib']:.1f} | "
                         f"{r[l]['bytes'] / 1e6:.3f} |")
        lines += ["", f"traffic_bytes_per_launch_every_level: {r['all']['bytes']:.0f}"]
        lines += [f"traffic_bytes_per_launch_level{l}: {r[l]['bytes']:.0f}" for l in range(len(probe["colors"]))]
        lines.append("kernels_hip_sha256: " + hashlib.sha256(open(src, "rb").read()).hexdigest())
        print("\n".join(lines))
        return
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
    if args.workload == "coarse":
        return bench_coarse(args)
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
                          "copy_bytes_written": dst.numel() * 8, "cycles": 3,
                          "colors": [S.colors(l)[1] for l in range(S.tail_first(3, "fp32ir"))]}), flush=True)
        return

    # warmup both precisions
    for prec in ("fp32ir", "fp64"):
        run_steps(S, Vd, w["t"], b, rtol, prec, args.warmup, use_graph)
    # Launch mode per precision: eager launches, or every cycle replayed from
    # a captured hipGraph (the same iterates bit for bit).  --graph -1 times
    # both after the warmup and keeps the faster: the host's cost to enqueue
    # one launch (2.3-3.3 us) differs between machines, a replay's does not.
    graph, mode_ms = {}, {}
    for prec in ("fp32ir", "fp64"):
        if args.graph >= 0:
            graph[prec] = bool(args.graph)
            continue
        run_steps(S, Vd, w["t"], b, rtol, prec, 1, True)
        te = tg = 0.0
        for _ in range(2):
            te += run_steps(S, Vd, w["t"], b, rtol, prec, 2, False)[0]
            tg += run_steps(S, Vd, w["t"], b, rtol, prec, 2, True)[0]
        graph[prec] = tg < te
        mode_ms[prec] = {"eager": te / 4 * 1e3, "graph": tg / 4 * 1e3}
        log(f"launch mode {prec}: eager {te / 4 * 1e3:.2f} ms/step, graph {tg / 4 * 1e3:.2f} ms/step")
    use_graph = graph["fp32ir"]
    # timed region: mixed precision, no instrumentation
    t_mixed, infos_m, x_m = run_steps(S, Vd, w["t"], b, rtol, "fp32ir", args.steps, use_graph)
    log(f"mixed: {t_mixed / args.steps * 1e3:.2f} ms/step cycles={infos_m[-1]['cycles']} res={max(infos_m[-1]['rel_res']):.2e}")
    # the same steps again with the dominant kernel's launches timed by HIP
    # events on their stream around each relaxation call (its sweeps x colors
    # launches, back to back), per level too
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
    floors = {l: (S.launch_floor("empty", l), S.launch_floor("chain", l), S.launch_floor("chain_rw", l))
              for l in launch_levels}
    t_fp64, infos_d, x_d = run_steps(S, Vd, w["t"], b, rtol, "fp64", args.steps, graph["fp64"])
    log(f"fp64: {t_fp64 / args.steps * 1e3:.2f} ms/step cycles={infos_d[-1]['cycles']} res={max(infos_d[-1]['rel_res']):.2e}")
    so_m, _ = time_solve_only(S, b, rtol, "fp32ir", args.steps, use_graph)
    so_d, _ = time_solve_only(S, b, rtol, "fp64", args.steps, graph["fp64"])
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

    copy_gbs = copy_bandwidth()
    log(f"device copy: {copy_gbs:.0f} GB/s")

    def summary(p):
        ach = p["bytes"] / (p["ms"] * 1e-3) / 1e9 if p["ms"] > 0 else None
        return {"achieved": ach, "frac": ach / HBM_PEAK_GBS if ach else None,
                "frac_of_copy": ach / copy_gbs if ach else None, "launches": p["launches"],
                "avg_launch_us": p["ms"] * 1e3 / max(1, p["launches"]),
                "algorithmic_bytes_per_launch": p["bytes"] / max(1, p["launches"])}
    traffic_all, traffic_lv = measured_traffic() if args.profile_kind.startswith("gs") else (None, {})
    top = summary(prof)
    roofline = {"bound": "hbm", "achieved": top["achieved"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": top["frac"], "traffic": traffic_all,
                "kernel": "k_gs_color_w<3, float> / k_gs_color<3, float> (multicolor Gauss-Seidel, FP32 cycles, "
                          "every level relaxed by per-color launches)"
                          if args.profile_kind.startswith("gs") else f"{args.profile_kind} (every level)",
                "launches": top["launches"], "avg_launch_us": top["avg_launch_us"],
                "algorithmic_bytes_per_launch": top["algorithmic_bytes_per_launch"],
                "bytes_rule": "per sweep z(s+4) + 4(n+1) + 3kns: z matrix entries incl. diagonal, n rows, "
                              "s = 4 B values, k = 3 right-hand sides, x gathers counted once; "
                              "a color launch counts its rows' share",
                "measured": "HIP events on the launch stream around each relaxation call (every sweep and color "
                            "of one level's pre- or post-relaxation, launched back to back) in a second pass of "
                            "the same timed steps; per launch = that time / its launches (kernel time plus the "
                            "gaps between those dependent launches)" if args.profile_kind == "gs_group" else
                            "dispatch-stamped HIP events on the launch stream, every launch of the kernel in a "
                            "second pass of the same timed steps",
                "levels": {str(l): dict(summary(p), colors=S.colors(l)[1], traffic=traffic_lv.get(l),
                                        floor_empty_us=floors[l][0][0], floor_chain_us=floors[l][1][0],
                                        floor_chain_rw_us=floors[l][2][0],
                                        host_enqueue_us=floors[l][1][1],
                                        latency_frac=floors[l][1][0] / summary(p)["avg_launch_us"])
                           for l, p in prof_lv.items()},
                "copy_gbs": copy_gbs, "frac_of_copy": top["frac_of_copy"],
                "copy_rule": "1 GiB device-to-device copy (torch copy_), bytes read + written per second",
                "latency_rule": "floor_chain_us: device launch-to-launch time of 2000 back-to-back launches, queued "
                                "ahead of the device, with the level's widest color grid whose threads load an index "
                                "(the level's column array), the value it points to, and store it (floor_empty_us: "
                                "an empty kernel; floor_chain_rw_us: the chain gathering what the previous launch "
                                "wrote, as color launches do; host_enqueue_us: host time to enqueue one such launch); "
                                "latency_frac = floor_chain_us / the level's relaxation time per launch"}
    value = args.steps / t_mixed
    out = {
        "metric": "V-cycle solves/s + HBM GB/s at 1M verts to rel residual 1e-8, mixed vs FP64",
        "value": value, "unit": "solves/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": t_mixed / args.steps * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32/f64", "data": "synthetic",
        "config": {"workload": f"{w['name']} torus R=1 r=0.3 jitter 0.2, A=M+1e-2 L, 3 RHS b=M X, "
                               f"{n_levels} levels, mu 2/2, rtol 1e-8",
                   "vertices": len(w["V"]), "levels": h.sizes, "rhs": 3, "graph": graph,
                   "launch_mode": "chosen by timing eager and graph steps after the warmup" if args.graph < 0
                   else "set by --graph", "launch_mode_ms_per_step": mode_ms},
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
