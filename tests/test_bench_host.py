"""Host-side logic of bench.py, without a GPU: the one-GPU refusal, the HBM
traffic table (looked up only while the row kernels' sources are unchanged),
the scaling of hardware byte counters by a copy of known size, and the
kernel-statistics summary that sets the trace's average beside the events'."""
import argparse
import csv
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert p.returncode == 2
    msg = json.loads(p.stdout.strip().splitlines()[-1])
    assert msg["n_gpus"] == 2 and "one GPU" in msg["error"]


def test_traffic_table_applies_only_to_the_sources_it_was_taken_on(monkeypatch):
    path = bench.traffic_file("c4s")
    with open(path) as fh:
        tab = json.load(fh)
    tile = next(iter(tab["tiles"]))
    r, u = (int(v) for v in tile.split("x"))
    want = tab["tiles"][tile]["update_prec"]["hbm_bytes_per_launch"]
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: tab["source_hash"])
    assert bench.measured_traffic("c4s", (r, u), "update_prec") == want
    assert bench.measured_traffic("c4s", (r + 1, u), "update_prec") is None
    assert bench.measured_traffic("no-such-workload", (r, u), "update_prec") is None
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: "0" * 16)
    assert bench.measured_traffic("c4s", (r, u), "update_prec") is None


def _counter_csv(path, counter, rows):
    os.makedirs(os.path.dirname(path), exist_ok=True)
    with open(path, "w", newline="") as fh:
        w = csv.DictWriter(fh, fieldnames=["Dispatch_Id", "Kernel_Name", "Grid_Size",
                                           "Counter_Name", "Counter_Value"])
        w.writeheader()
        for i, (name, grid, value) in enumerate(rows):
            w.writerow({"Dispatch_Id": i, "Kernel_Name": name, "Grid_Size": grid,
                        "Counter_Name": counter, "Counter_Value": value})


def test_counters_are_scaled_by_the_copy_and_taken_after_the_last_clear(tmp_path):
    # A 1 GiB copy whose FETCH_SIZE reads half of its bytes (in KiB) and whose
    # WRITE_SIZE reads all of them: fetch counts are doubled, writes kept.
    # Only launches after the last k_clear_active count (the second solve).
    upd = "void airga::k_update_prec<float, 6, 4, 1, false, true, true>(airga::SolveArgs<float>, int)"
    dsp = "void airga::k_dir_spmv<float, 6, 4, 1, false, true, true>(airga::SolveArgs<float>, int)"
    clear = "airga::k_clear_active(airga::SysDev, int)"
    copy = "__amd_rocclr_copyBuffer"
    gib_kib = 1024.0 * 1024.0
    for counter, copy_kib, scale in (("FETCH_SIZE", gib_kib / 2, 2.0), ("WRITE_SIZE", gib_kib, 1.0)):
        sub = "fetch" if counter == "FETCH_SIZE" else "write"
        rows = [(upd, 1000, 999999.0), (clear, 64, 1.0),
                (upd, 1000, 100.0), (dsp, 1000, 40.0), (upd, 1000, 300.0), (dsp, 1000, 60.0),
                (copy, 1 << 17, copy_kib), (copy, 512, 3.0)]
        _counter_csv(str(tmp_path / "pmc" / f"256x1_{sub}" / "c4s_counter_collection.csv"),
                     counter, rows)
    out = tmp_path / "table.json"
    args = argparse.Namespace(summarize_pmc=str(tmp_path / "pmc"), workload="c4s",
                              command="(test)", out=str(out))
    bench.summarize_pmc(args)
    tab = json.loads(out.read_text())
    ent = tab["tiles"]["256x1"]
    assert ent["update_prec"]["launches"] == 2 and ent["dir_spmv"]["launches"] == 2
    assert ent["update_prec"]["fetch_size_bytes_per_launch"] == int(200.0 * 1024 * 2.0)
    assert ent["update_prec"]["write_size_bytes_per_launch"] == int(200.0 * 1024 * 1.0)
    assert ent["dir_spmv"]["hbm_bytes_per_launch"] == int(50.0 * 1024 * 2.0) + int(50.0 * 1024)
    assert ent["update_prec"]["fetch_size_scale"] == pytest.approx(2.0)
    assert tab["source_hash"] == bench.kernel_source_hash()


def test_trace_summary_names_both_averages_of_the_dominant_kernel(tmp_path):
    stats = tmp_path / "c4s_kernel_stats.csv"
    upd = "void airga::k_update_prec<float, 6, 4, 1, false, true, true>(airga::SolveArgs<float>, int)"
    with open(stats, "w", newline="") as fh:
        w = csv.DictWriter(fh, fieldnames=["Name", "Calls", "TotalDurationNs", "AverageNs",
                                           "Percentage"])
        w.writeheader()
        w.writerow({"Name": "airga::k_reduce<1024>(airga::ReduceArgs, int)", "Calls": 10,
                    "TotalDurationNs": 50000, "AverageNs": 5000, "Percentage": 1.0})
        w.writerow({"Name": upd, "Calls": 32, "TotalDurationNs": 5152000, "AverageNs": 161000,
                    "Percentage": 20.0})
    line = {"value": 5500.0, "unit": "solves/s", "ms_per_step": 23.3,
            "config": {"tile": {"rows_per_wave": 256, "systems_per_group": 1}},
            "roofline": {"kernel": "update_prec", "avg_launch_us": 163.5, "achieved": 4796.6,
                         "frac": 0.5996, "peak": 8000.0}}
    bj = tmp_path / "bench.json"
    bj.write_text("[bench] log line\n" + json.dumps(line) + "\n")
    out = tmp_path / "summary.md"
    args = argparse.Namespace(summarize_trace=str(stats), bench_json=str(bj),
                              command="rocprofv3 ... (test)", out=str(out))
    bench.summarize_trace(args)
    text = out.read_text()
    rows = [x for x in text.splitlines() if x.startswith("| `")]
    assert "k_update_prec" in rows[0] and "| 32 | 5.15 | 161.0 | 20.0 |" in rows[0]
    assert "bench.py events 163.5 us" in text and "all its launches in the run: 161.0 us" in text
    assert "rocprofv3 ... (test)" in text


def test_kernel_bytes_follow_the_per_kernel_formulas():
    # one 1000-row pencil of 6000 stored entries, banded (1-byte offsets),
    # float32 inner solves: the formulas of the kernel table, term by term
    kw = dict(stored=6000, n=1000, ib=1, w=4, fw=4, m=2)
    assert bench.kernel_bytes("dir_spmv", 3, 10, 0, **kw) == 3 * 6000 * 9 + 10 * 16 * 1000
    assert bench.kernel_bytes("update_prec", 3, 10, 5, first_passes=2, **kw) == \
        3 * 6000 + 5 * 6000 * 4 + (70 - 2) * 4 * 1000
    assert bench.kernel_bytes("init_prec", 1, 4, 2, **kw) == 6000 + 2 * 6000 * 4 + 4 * 8 * 1000
    assert bench.kernel_bytes("chain", 2, 6, 3, **kw) == 2 * 6000 * 4 + 3 * 6000 * 4 + 6 * 8 * 1000
    assert bench.kernel_bytes("ir_residual", 2, 8, 0, **kw) == \
        2 * 6000 * 17 + 2 * 2 * 8 * 1000 + 8 * 12 * 1000
    # one of the two launches is a solve's first residual from X = 0 (4 systems)
    assert bench.kernel_bytes("ir_residual", 2, 8, 0, zs_launches=1, zs_sys=4, **kw) == \
        6000 * 17 + 2 * 2 * 8 * 1000 + 8 * 12 * 1000 - 4 * 8 * 1000
    assert bench.kernel_bytes("ir_update", 1, 8, 0, **kw) == 8 * 20 * 1000
    assert bench.kernel_bytes("ir_update", 2, 8, 0, assign_sys=4, **kw) == (8 * 20 - 4 * 8) * 1000
    assert bench.kernel_bytes("ir_update", 1, 8, 0, mixed=False, **kw) == 8 * 16 * 1000
    assert bench.kernel_bytes("reduce", 5, 0, 0, gp=7, red_sys=11, **kw) == 11 * 7 * 8
    # float64 solves: 8-byte vectors and factor values
    kw64 = dict(kw, w=8, fw=8)
    assert bench.kernel_bytes("update_prec", 1, 1, 1, **kw64) == 6000 + 6000 * 8 + 7 * 8 * 1000
    # 64-row slices, 4 wavefronts per block
    assert bench.row_blocks(1000, 256) == 1 and bench.row_blocks(1_000_000, 256) == 977
    rows = bench.kernel_rows({"update_prec": (2, 0.5), "reduce": (4, 0.01)},
                             {"update_prec": (4, 2), "reduce": (0, 0)}, gp=3, **kw)
    upd = next(r for r in rows if r["kernel"] == "update_prec")
    assert upd["bytes"] == 2 * 6000 + 2 * 6000 * 4 + 28 * 4 * 1000
    assert upd["gbs"] == round(upd["bytes"] / 0.5e-3 / 1e9, 1)
    red = next(r for r in rows if r["kernel"] == "reduce")
    assert red["bytes"] == 3 * 4 * 3 * 8   # 3 slots per update pass
