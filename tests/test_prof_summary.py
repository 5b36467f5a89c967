"""prof_summary.py (the script that turns rocprofv3 CSV output into the
summaries under profiles/) on synthetic CSV files: kernel names reduced to
their bare name, the mean of the last K dispatches (also with trailing
dispatches left out), HBM bytes per launch scaled by the copy calibration,
and the SQ counter ratios (per wave, VALU busy per SIMD from the busy cycles
summed over the dies)."""
import csv
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
KNAME = "(anonymous namespace)::k_persistent(nsp::KParams const*)"


def _write_csv(path, rows):
    with open(path, "w", newline="") as fh:
        w = csv.DictWriter(fh, fieldnames=list(rows[0].keys()))
        w.writeheader()
        w.writerows(rows)


def _bench_log(path, alg):
    with open(path, "w") as fh:
        fh.write("[bench] progress line\n")
        fh.write(json.dumps({"metric": "m", "value": 1.0, "unit": "u", "config": {"workload": "w"},
                             "roofline": {"avg_launch_ms": 2.0, "algorithmic_bytes_per_launch": alg}}) + "\n")


def _run(*args):
    return subprocess.run([sys.executable, os.path.join(ROOT, "prof_summary.py")] + list(args), check=True,
                          capture_output=True, text=True).stdout


def test_trace_summary(tmp_path):
    d = tmp_path / "tr"
    d.mkdir()
    _write_csv(d / "run_kernel_stats.csv", [
        {"Name": KNAME, "Calls": 3, "TotalDurationNs": 6e6, "AverageNs": 2e6, "MinNs": 1e6, "MaxNs": 3e6},
        {"Name": "__amd_rocclr_copyBuffer", "Calls": 1, "TotalDurationNs": 1e3, "AverageNs": 1e3, "MinNs": 1e3,
         "MaxNs": 1e3}])
    _write_csv(d / "run_kernel_trace.csv", [
        {"Kernel_Name": KNAME, "Dispatch_Id": i, "Start_Timestamp": 0, "End_Timestamp": int(ns)}
        for i, ns in enumerate([5e6, 1e6, 3e6])])
    _bench_log(tmp_path / "b.log", 1e9)
    out = tmp_path / "t.txt"
    _run("trace", str(d), "--last", "2", "--bench-json", str(tmp_path / "b.log"), "--cmd", "CMD", "--out", str(out))
    text = out.read_text()
    assert "k_persistent" in text and "(anonymous" not in text
    assert "timed_dispatches=2" in text
    assert "trace_avg_ms_timed=2.0000" in text   # mean of the last two: 1 ms and 3 ms


def test_traffic_summary(tmp_path):
    def counters(name, counter, values, kernel=KNAME):
        d = tmp_path / name
        d.mkdir()
        _write_csv(d / "run_counter_collection.csv", [
            {"Kernel_Name": kernel, "Dispatch_Id": i, "Counter_Name": counter, "Counter_Value": v}
            for i, v in enumerate(values)])
        return str(d)

    # the copy moves 1 GiB each way; its counters read half the fetched bytes, all written bytes (KiB)
    cf = counters("cf", "FETCH_SIZE", [524288.0], "__amd_rocclr_copyBuffer")
    cw = counters("cw", "WRITE_SIZE", [1048576.0], "__amd_rocclr_copyBuffer")
    kf = counters("kf", "FETCH_SIZE", [999.0, 1000.0, 3000.0])
    kw = counters("kw", "WRITE_SIZE", [7.0, 500.0, 1500.0])
    with open(tmp_path / "copy.log", "w") as fh:
        fh.write(json.dumps({"metric": "copy", "value": 1.0, "unit": "GB/s",
                             "config": {"bytes_read_per_launch": 1 << 30, "bytes_written_per_launch": 1 << 30}}))
    _bench_log(tmp_path / "b.log", 4096.0 * 1024)
    (tmp_path / "hash.txt").write_text("abc123\n")
    out = tmp_path / "p.txt"
    _run("traffic", "--fetch", kf, "--write", kw, "--copy-fetch", cf, "--copy-write", cw, "--bench-json",
         str(tmp_path / "b.log"), "--copy-json", str(tmp_path / "copy.log"), "--hash", str(tmp_path / "hash.txt"),
         "--last", "2", "--cmd", "CMD", "--out", str(out))
    rec = dict(line.split("=", 1) for line in out.read_text().splitlines() if "=" in line and not line.startswith("#"))
    assert float(rec["fetch_scale"]) == 2.0 and float(rec["write_scale"]) == 1.0
    # last two dispatches: fetch (1000 + 3000) / 2 KiB x 2, write (500 + 1500) / 2 KiB x 1
    assert float(rec["hbm_bytes_per_launch"]) == (4000.0 + 1000.0) * 1024
    assert abs(float(rec["traffic_over_algorithmic"]) - 5000.0 / 4096.0) < 1e-4
    assert rec["kernel_source_sha256_16"] == "abc123"
    # the same with the last dispatch left out: dispatches 0 and 1
    _run("traffic", "--fetch", kf, "--write", kw, "--copy-fetch", cf, "--copy-write", cw, "--bench-json",
         str(tmp_path / "b.log"), "--copy-json", str(tmp_path / "copy.log"), "--hash", str(tmp_path / "hash.txt"),
         "--last", "2", "--skip-last", "1", "--cmd", "CMD", "--out", str(out))
    rec = dict(line.split("=", 1) for line in out.read_text().splitlines() if "=" in line and not line.startswith("#"))
    assert float(rec["hbm_bytes_per_launch"]) == (999.0 + 1000.0 + (7.0 + 500.0) / 2) * 1024


def test_trace_summary_leaves_out_trailing_dispatches(tmp_path):
    d = tmp_path / "tr"
    d.mkdir()
    _write_csv(d / "run_kernel_stats.csv", [
        {"Name": KNAME, "Calls": 5, "TotalDurationNs": 25e6, "AverageNs": 5e6, "MinNs": 1e6, "MaxNs": 9e6}])
    _write_csv(d / "run_kernel_trace.csv", [
        {"Kernel_Name": KNAME, "Dispatch_Id": i, "Start_Timestamp": 0, "End_Timestamp": int(ns)}
        for i, ns in enumerate([1e6, 2e6, 4e6, 9e6, 9e6])])
    _bench_log(tmp_path / "b.log", 1e9)
    out = tmp_path / "t.txt"
    _run("trace", str(d), "--last", "2", "--skip-last", "2", "--bench-json", str(tmp_path / "b.log"), "--cmd",
         "CMD", "--out", str(out))
    text = out.read_text()
    assert "dispatches=5" in text and "dispatches_after_the_timed_ones=2" in text
    assert "trace_avg_ms_timed=3.0000" in text   # 2 ms and 4 ms; the two 9 ms dispatches after them left out


def test_sq_summary(tmp_path):
    d = tmp_path / "sq"
    d.mkdir()
    per = {"SQ_WAVES": 100.0, "SQ_WAVE_CYCLES": 1000.0, "SQ_WAIT_ANY": 600.0, "SQ_ACTIVE_INST_VALU": 32.0,
           "GRBM_GUI_ACTIVE": 80.0}
    # dispatch i holds (i + 1) times the values above
    _write_csv(d / "run_counter_collection.csv", [
        {"Kernel_Name": KNAME, "Dispatch_Id": i, "Counter_Name": k, "Counter_Value": v * (i + 1)}
        for i in range(3) for k, v in per.items()])
    out = tmp_path / "q.txt"
    _run("sq", str(d), "--kernel", "k_persistent", "--last", "2", "--workload", "W", "--cmd", "CMD", "--out",
         str(out), "--cus", "2", "--xcds", "2")
    rec = {k: v.split()[0] for k, v in (line.split("=", 1) for line in out.read_text().splitlines()
                                          if "=" in line and not line.startswith("#"))}
    assert float(rec["SQ_WAVES"]) == 250.0   # mean of the last two dispatches, 200 and 300
    assert float(rec["wait_fraction_of_wave_lifetime"]) == 0.6
    # 4 x ACTIVE_INST_VALU / (4 SIMDs x 2 CUs x GRBM_GUI_ACTIVE / 2 dies) = 4 x 80 / (8 x 100)
    assert float(rec["gpu_busy_cycles_per_xcd"]) == 100.0
    assert float(rec["valu_busy_per_simd"]) == 0.4
    # the last dispatch left out: dispatches 0 and 1 (100 and 200 waves)
    _run("sq", str(d), "--kernel", "k_persistent", "--last", "2", "--skip-last", "1", "--workload", "W", "--cmd",
         "CMD", "--out", str(out), "--cus", "2", "--xcds", "2")
    assert "SQ_WAVES=150.0" in out.read_text()
