"""Host logic of the benchmark's measurement pipeline (no GPU): the
whole-step counter summary is taken over the timed dbs_step call, per step,
and scaled by the copy calibration; the step byte model adds up its stages."""
from __future__ import annotations

import csv
import os

import bench

FIELDS_T = ["Kind", "Dispatch_Id", "Kernel_Name", "Start_Timestamp", "End_Timestamp",
            "Grid_Size_X", "Grid_Size_Y", "Grid_Size_Z"]
FIELDS_C = ["Dispatch_Id", "Kernel_Name", "Grid_Size", "Counter_Value"]


def _write(path, fields, rows):
    os.makedirs(os.path.dirname(path), exist_ok=True)
    with open(path, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=fields)
        w.writeheader()
        for r in rows:
            w.writerow(r)


def _calls(step_counts):
    """Dispatches of dbs_step calls with the given step counts: per step
    k_add_time, then k_work (4 us, 1000 threads); per call k_stats_final."""
    seq = []
    for n in step_counts:
        for _ in range(n):
            seq += [("dbs::k_add_time(int)", 1, 2), ("void dbs::k_work(double*)", 1000, 4)]
        seq.append(("dbs::k_stats_final(double*)", 1024, 1))
    return seq


def test_counter_summary_is_per_step_of_the_timed_call(tmp_path):
    d = str(tmp_path)
    seq = _calls([2, 3])  # warm-up call of 2 steps, timed call of 3
    t, rows_t, rows_f, rows_w = 0, [], [], []
    for i, (name, grid, us) in enumerate(seq):
        rows_t.append({"Kind": "KERNEL_DISPATCH", "Dispatch_Id": i + 1, "Kernel_Name": name,
                       "Start_Timestamp": t, "End_Timestamp": t + us * 1000,
                       "Grid_Size_X": grid, "Grid_Size_Y": 1, "Grid_Size_Z": 1})
        t += us * 1000 + 500
        # the warm-up call's work kernels read more than the timed call's:
        # the summary must not mix them in
        kib = 4.0 if name.endswith("k_work(double*)") and i < 5 else 1.0
        rows_f.append({"Dispatch_Id": i + 1, "Kernel_Name": name, "Grid_Size": grid,
                       "Counter_Value": kib if "k_work" in name else 0.0})
        rows_w.append({"Dispatch_Id": i + 1, "Kernel_Name": name, "Grid_Size": grid,
                       "Counter_Value": 0.5 if "k_work" in name else 0.0})
    _write(f"{d}/trace/run_kernel_trace.csv", FIELDS_T, rows_t)
    _write(f"{d}/fetch/run_counter_collection.csv", FIELDS_C, rows_f)
    _write(f"{d}/write/run_counter_collection.csv", FIELDS_C, rows_w)
    # calibration: a 1 GiB copy counted as 2 GiB fetched and 1 GiB written
    for kind, kib in (("fetch", 2.0 * (1 << 20)), ("write", 1.0 * (1 << 20))):
        _write(f"{d}/c{kind}/run_counter_collection.csv", FIELDS_C,
               [{"Dispatch_Id": 1, "Kernel_Name": "__amd_rocclr_copyBuffer",
                 "Grid_Size": 1, "Counter_Value": kib}])
    out = bench.summarize_counters(d, 8, "mixed", "trace-cmd", "counter-cmd")
    assert "(3 steps" in out
    # per step: one k_add_time and one k_work, plus a third of k_stats_final
    assert "2.3 launches" in out
    row = [l for l in out.splitlines() if l.startswith("| `k_work`")][0].split("|")
    assert row[3].strip() == "1.0"   # launches per step
    assert row[4].strip() == "4.0"   # us per launch
    # fetch 1 KiB x 0.5 (calibration) + write 0.5 KiB x 1.0 per launch,
    # over 8^3 cells
    assert row[7].strip() == "2.0"   # B per cell
    recs = [l for l in out.splitlines() if l.startswith("<!-- bench-traffic")]
    assert len(recs) == 1 and '"kernel": "step"' in recs[0]
    assert '"traffic_bytes_per_launch": 1024.0' in recs[0]


def test_step_byte_model_adds_its_stages():
    B = bench.STEP_BYTES
    its = [4, 2]
    fixed = (B["alpha_face"] + B["alpha_limit_update"] + B["mom_assemble"] +
             4 * B["jacobi_sweep"] + 2 * (B["p_assembly"] + B["correct"]) +
             B["guess_first"] + B["guess_later"])
    assert bench.alg_step_bytes_per_cell("mixed", its, 4) == fixed + 6 * 160
    assert bench.alg_step_bytes_per_cell("fp64", its, 4) == fixed + 6 * 216
    # one corrector: no later-corrector guesses
    one = (B["alpha_face"] + B["alpha_limit_update"] + B["mom_assemble"] +
           4 * B["jacobi_sweep"] + B["p_assembly"] + B["correct"] + B["guess_first"])
    assert bench.alg_step_bytes_per_cell("mixed", [4], 4) == one + 4 * 160
