"""Host-side logic of bench.py (no GPU): the flop and byte tallies its rooflines use, the
profile summariser on small synthetic rocprofv3 CSV files, the traffic record's source
check, and the refusal of more than one GPU."""
import csv
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_fused_flop_tally():
    """Four residual evaluations (130), the kinematic (73), velocity (122) and momentum (48)
    stage updates, renormalisation (12), the lag stage wrenches (48), and per control step
    29 N + 2 (lag) or 14 N + 8 spread over S sub-steps."""
    assert bench.substep_flops(6, True, 16) == 4 * 130 + 73 + 122 + 48 + 12 + 48 + (29 * 6 + 2) / 16
    assert bench.substep_flops(8, True, 16) == 837.625
    assert bench.substep_flops(6, True, 16) == 834.0
    assert bench.substep_flops(6, False, 1) == 4 * 130 + 73 + 122 + 48 + 12 + 14 * 6 + 8


def test_split_flop_tally():
    """211 + 16 N per sub-step with lag, + (14 N - 6) / S per control step; the committed
    counter reading (profiles/k_split_k_task_pmc.md) is within 1 flop of it."""
    assert bench.split_substep_flops(6, True, 16) == 211 + 96 + 78 / 16
    assert bench.split_substep_flops(8, True, 16) == pytest.approx(345.625)
    assert bench.split_substep_flops(6, False, 16) == 211 + 78 / 16


def test_plain_bytes():
    """State read and write, one throttle frame and the 23 parameters per env-substep."""
    assert bench.plain_bytes(6, True) == 4 * (2 * 19 + 6 + 23) == 268
    assert bench.plain_bytes(8, True) == 292
    assert bench.plain_bytes(6, False) == 4 * (2 * 13 + 6 + 23)


def test_traffic_record_matches_only_current_sources(tmp_path, monkeypatch):
    """The committed traffic record is used only for the kernel sources it was taken on."""
    import json
    h = bench.kernel_source_hash()
    rec = {"source_hash": h, "k_step_fused_control_step": 123.0}
    (tmp_path / "profiles").mkdir()
    (tmp_path / "profiles" / "traffic.json").write_text(json.dumps(rec))
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: h)
    assert bench.load_traffic("k_step_fused_control_step") == 123.0
    rec["source_hash"] = "0" * 16
    (tmp_path / "profiles" / "traffic.json").write_text(json.dumps(rec))
    assert bench.load_traffic("k_step_fused_control_step") is None


def _write(path, rows, fields):
    with open(path, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=fields)
        w.writeheader()
        for r in rows:
            w.writerow(r)


def test_summarise_profile_unions_concurrent_launch_pairs(tmp_path):
    """Two concurrent class launches per control step: the summary reports the union of
    their busy intervals per pair, not the sum of the launches' durations."""
    d = tmp_path / "trace"
    d.mkdir()
    fields = ["Kernel_Name", "Start_Timestamp", "End_Timestamp"]
    rows = []
    t = 0
    for _ in range(3):          # pairs overlapping: [t, t+100] and [t+10, t+130]
        rows.append({"Kernel_Name": "void mg::k_step<6, true, false>(x)", "Start_Timestamp": t,
                     "End_Timestamp": t + 100_000})
        rows.append({"Kernel_Name": "void mg::k_step<8, true, false>(x)",
                     "Start_Timestamp": t + 10_000, "End_Timestamp": t + 130_000})
        t += 200_000
    _write(d / "x_kernel_trace.csv", rows, fields)
    _write(d / "x_kernel_stats.csv",
           [{"Name": "void mg::k_step<6, true, false>(x)", "Calls": 3, "AverageNs": 100000,
             "MinNs": 100000, "MaxNs": 100000, "Percentage": 50.0}],
           ["Name", "Calls", "AverageNs", "MinNs", "MaxNs", "Percentage"])
    out = bench.summarise_profile(str(tmp_path))
    assert "130.00 us per launch pair" in out
    assert "| `void mg::k_step<6, true, false>(x)` | 3 | 100.00 |" in out


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_traffic_from_counters(tmp_path):
    """traffic.json from synthetic FETCH_SIZE / WRITE_SIZE CSVs: the copy of 1 GiB that reads
    half its bytes in FETCH_SIZE calibrates fetches by 2, writes by 1; per launch the means,
    in bytes; the control step sums the two classes' fused launches."""
    rows = {"pmc_fetch": ("FETCH_SIZE", {"__amd_rocclr_copyBuffer": [524288.0, 4.0],
                                         "void mg::k_step<6, true, false>(mg::StepArgs, mg::ClassConst)": [1000.0, 1200.0],
                                         "void mg::k_step<8, true, false>(mg::StepArgs, mg::ClassConst)": [2000.0]}),
            "pmc_write": ("WRITE_SIZE", {"__amd_rocclr_copyBuffer": [1048576.0],
                                         "void mg::k_step<6, true, false>(mg::StepArgs, mg::ClassConst)": [300.0, 500.0],
                                         "void mg::k_step<8, true, false>(mg::StepArgs, mg::ClassConst)": [700.0]})}
    for sub, (counter, kern) in rows.items():
        d = tmp_path / sub / "run"
        d.mkdir(parents=True)
        with open(d / "x_counter_collection.csv", "w", newline="") as f:
            w = csv.DictWriter(f, ["Kernel_Name", "Counter_Name", "Counter_Value"])
            w.writeheader()
            for k, vals in kern.items():
                for v in vals:
                    w.writerow({"Kernel_Name": k, "Counter_Name": counter, "Counter_Value": v})
    t = bench.traffic_from_counters(str(tmp_path))
    assert t["fetch_factor"] == 2.0 and t["write_factor"] == 1.0
    assert t["per_launch"]["fused_bluerov2"] == 1024.0 * (2 * 1100.0 + 400.0)
    assert t["per_launch"]["fused_heavy"] == 1024.0 * (2 * 2000.0 + 700.0)
    assert t["k_step_fused_control_step"] == 1024.0 * (2600.0 + 4700.0)
    assert "k_step_plain_substep" not in t
    assert t["source_hash"] == bench.kernel_source_hash()
    assert t["algorithmic_fused_control_step"] == 524288 * (268 + 292)
