"""The measurement summaries of bench.py on synthetic rocprofv3 output: the
position rule that assigns each relaxation launch its level and relaxation
call, the trace summary's per-pass and per-level figures, and the counter
calibration of the traffic summary."""
import csv
import json
import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402

COLORS = [3, 5, 4]
DOM = "void smg::(anonymous namespace)::k_gs_color_w<3, float>(int)"


def test_cycle_order_and_calls():
    lv = bench._cycle_levels(COLORS)
    # 2 pre sweeps per level in level order, then 2 post sweeps in reverse order
    assert lv == [0] * 6 + [1] * 10 + [2] * 8 + [2] * 8 + [1] * 10 + [0] * 6
    n = len(lv)
    st = bench._step_levels(2 * n + 4, COLORS)          # two cycles and a prefix of the third
    assert st[:n] == lv and st[n:2 * n] == lv and st[2 * n:] == [0] * 4
    gr = bench._step_groups(2 * n + 4, COLORS)
    assert gr[:6] == [0] * 6 and gr[6:16] == [1] * 10 and gr[24:32] == [3] * 8
    assert gr[n:n + 6] == [6] * 6 and gr[-4:] == [12] * 4          # next cycle's calls, then the prefix's
    assert len(set(gr)) == 2 * 2 * len(COLORS) + 1


def _write(path, rows, fields):
    with open(path, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=fields)
        w.writeheader()
        w.writerows(rows)


def test_trace_summary(tmp_path):
    cyc = len(bench._cycle_levels(COLORS))
    per_step = 2 * cyc
    steps, warm = 2, 1
    total = warm + steps + steps + 2 * len(COLORS) + steps + 1
    lv = bench._step_levels(per_step, COLORS)
    rows, t = [], 0
    for _ in range(total):
        for i in range(per_step):
            dur = 1000 * (lv[i] + 1)                   # level l takes (l + 1) us
            rows.append({"Kernel_Name": DOM, "Start_Timestamp": t, "End_Timestamp": t + dur})
            t += dur + 500                             # 0.5 us between launches
        rows.append({"Kernel_Name": "k_other", "Start_Timestamp": t, "End_Timestamp": t + 100})
        t += 10000
    _write(tmp_path / "run_kernel_trace.csv", rows, ["Kernel_Name", "Start_Timestamp", "End_Timestamp"])
    _write(tmp_path / "run_kernel_stats.csv",
           [{"Name": DOM, "Calls": len(rows), "TotalDurationNs": 1, "AverageNs": 1, "MinNs": 1, "MaxNs": 1}],
           ["Name", "Calls", "TotalDurationNs", "AverageNs", "MinNs", "MaxNs"])
    levels = {str(l): {"colors": c, "algorithmic_bytes_per_launch": 1e6, "avg_launch_us": 1.0}
              for l, c in enumerate(COLORS)}
    js = {"steps": steps, "warmup": warm,
          "roofline": {"launches": per_step * steps, "levels": levels, "avg_launch_us": 2.0, "achieved": 1.0,
                       "frac": 0.1, "algorithmic_bytes_per_launch": 1e6}}
    (tmp_path / "b.json").write_text(json.dumps(js))
    out = bench.trace_summary(str(tmp_path), str(tmp_path / "b.json"))
    for l in range(len(COLORS)):
        # kernel time (l + 1) us; inside a call of m launches: ((l + 1.5) m - 0.5) / m
        m = 2 * COLORS[l]
        want = ((l + 1.5) * m - 0.5) / m
        line = [x for x in out.splitlines() if x.startswith(f"| {l} | {COLORS[l]} | timed |")][0]
        cells = [c.strip() for c in line.strip("|").split("|")]
        assert float(cells[4]) == pytest.approx(l + 1.0, abs=1e-3)
        assert float(cells[5]) == pytest.approx(want, abs=1e-3)


def test_pmc_summary_scales_by_the_copy(tmp_path):
    cyc = bench._cycle_levels(COLORS)
    for counter, d, raw in (("FETCH_SIZE", "f", 131072.0), ("WRITE_SIZE", "w", 262144.0)):
        (tmp_path / d).mkdir()
        rows, k = [], 0
        for _ in range(3):
            k += 1
            rows.append({"Dispatch_Id": k, "Kernel_Name": "vectorized_elementwise_kernel", "Counter_Name": counter,
                         "Counter_Value": raw})
        for _ in range(2):
            for l in cyc:
                k += 1
                rows.append({"Dispatch_Id": k, "Kernel_Name": DOM, "Counter_Name": counter,
                             "Counter_Value": 100.0 * (l + 1)})
        _write(tmp_path / d / "run_counter_collection.csv", rows, list(rows[0]))
    r = bench.pmc_summary(str(tmp_path / "f"), str(tmp_path / "w"), COLORS)
    assert r["scale_fetch"] == pytest.approx(2.0) and r["scale_write"] == pytest.approx(1.0)
    for l in range(len(COLORS)):
        # 100 (l + 1) KiB counted by each counter: 2x + 1x of it, in bytes
        assert r[l]["bytes"] == pytest.approx(3 * 100.0 * (l + 1) * 1024)
        assert r[l]["launches"] == 2 * 4 * COLORS[l]
