#!/usr/bin/env python3
"""Turn rocprofv3 CSV output of bench.py runs into the short text summaries
kept under profiles/.

  trace:   python prof_summary.py trace DIR --kernel k_persistent --last K
               --bench-json FILE --cmd "..." --out profiles/NAME.txt
           DIR holds `rocprofv3 --kernel-trace --stats --output-format csv
           -o run` output; the summary lists the per-kernel statistics and the
           mean duration of the last K dispatches of the kernel (bench.py's
           timed launches; --skip-last N leaves out N dispatches after them)
           beside bench.py's own HIP-event figure (--bench-field, default
           roofline.avg_launch_ms).

  traffic: python prof_summary.py traffic --fetch DIR --write DIR
               --copy-fetch DIR --copy-write DIR --kernel k_persistent --last K
               [--skip-last N]
               --bench-json FILE --hash FILE --cmd "..." --out profiles/NAME.txt
           The four DIRs hold `rocprofv3 --pmc FETCH_SIZE` / `--pmc WRITE_SIZE`
           output of the benchmark and of bench.py's 1 GiB copy.  Each counter
           is scaled by what it reads for the copy (bytes moved / counter
           bytes), and the summary records HBM bytes per launch of the last K
           dispatches together with the kernel source hash, which bench.py
           checks before it reports the figure as `traffic`.

  sq:      python prof_summary.py sq DIR --kernel k_mom_adjoint --last K [--skip-last N]
               --workload "..." --cmd "..." --out profiles/NAME.txt
           DIR holds `rocprofv3 --pmc SQ_WAVES SQ_WAVE_CYCLES SQ_WAIT_ANY
           SQ_ACTIVE_INST_VALU ...` output; the summary gives each counter's
           mean per dispatch over the last K dispatches of the kernel, its
           value per wave, and the fractions of the wave lifetime spent
           waiting (SQ_WAIT_ANY / SQ_WAVE_CYCLES) and issuing VALU work
           (SQ_ACTIVE_INST_VALU / SQ_WAVE_CYCLES).  With GRBM_GUI_ACTIVE (the
           GPU's busy cycles of the dispatch, summed over the --xcds
           dies) it adds the share of the dispatch each SIMD spent issuing
           VALU work: SQ_ACTIVE_INST_VALU x 4 (the counter ticks once per 4
           cycles) / (SIMDs x GRBM_GUI_ACTIVE / xcds), with 4 SIMDs on each
           of --cus compute units.
"""
from __future__ import annotations

import argparse
import csv
import glob
import json
import os


def _csv(dirpath, suffix):
    hits = sorted(glob.glob(os.path.join(dirpath, "**", "*" + suffix), recursive=True))
    if not hits:
        raise SystemExit("no *%s under %s" % (suffix, dirpath))
    with open(hits[0], newline="") as fh:
        return list(csv.DictReader(fh))


def _bench_line(path):
    with open(path) as fh:
        for line in fh:
            line = line.strip()
            if line.startswith("{") and '"metric"' in line:
                return json.loads(line)
    raise SystemExit("no bench.py JSON line in %s" % path)


def _short(name):
    """Bare kernel name: no return type, namespaces, template or argument list."""
    name = name.replace("(anonymous namespace)", "")
    for stop in ("(", "<"):
        name = name.split(stop)[0]
    return name.split("::")[-1].split(" ")[-1].strip()


def _counter(dirpath, counter, kernel):
    """Per-dispatch values of one counter for one kernel, in dispatch order."""
    rows = [r for r in _csv(dirpath, "counter_collection.csv") if r["Counter_Name"] == counter]
    rows.sort(key=lambda r: int(r["Dispatch_Id"]))
    return [float(r["Counter_Value"]) for r in rows if _short(r["Kernel_Name"]) == kernel]


def _field(d, path):
    """d["a"]["b"] for path "a.b"; "n/a" when absent"""
    for k in path.split("."):
        if not isinstance(d, dict) or k not in d:
            return "n/a"
        d = d[k]
    return d


def cmd_trace(a):
    stats = _csv(a.dir, "kernel_stats.csv")
    trace = _csv(a.dir, "kernel_trace.csv")
    bench = _bench_line(a.bench_json)
    mine = sorted((r for r in trace if _short(r["Kernel_Name"]) == a.kernel), key=lambda r: int(r["Dispatch_Id"]))
    dur = [(int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) * 1e-6 for r in mine]
    if a.skip_last:
        dur = dur[:-a.skip_last]
    last = dur[-a.last:]
    out = ["# rocprofv3 kernel trace of: %s" % a.cmd,
           "# workload: %s" % json.dumps(bench.get("config", {})),
           "#",
           "# per-kernel statistics (all dispatches of the run)",
           "%-48s %7s %12s %12s %12s %12s" % ("kernel", "calls", "total_ms", "avg_ms", "min_ms", "max_ms")]
    for r in sorted(stats, key=lambda r: -float(r["TotalDurationNs"]))[:12]:
        out.append("%-48s %7d %12.3f %12.4f %12.4f %12.4f" % (
            _short(r["Name"])[:48], int(r["Calls"]), float(r["TotalDurationNs"]) * 1e-6,
            float(r["AverageNs"]) * 1e-6, float(r["MinNs"]) * 1e-6, float(r["MaxNs"]) * 1e-6))
    out += ["#",
            "kernel=%s" % a.kernel,
            "dispatches=%d" % (len(dur) + a.skip_last),
            "timed_dispatches=%d" % len(last),
            "dispatches_after_the_timed_ones=%d" % a.skip_last,
            "trace_avg_ms_timed=%.4f" % (sum(last) / max(len(last), 1)),
            "bench_avg_launch_ms=%s" % _field(bench, a.bench_field),
            "bench_value=%s %s" % (bench["value"], bench["unit"])]
    for k in ("cg_iters_per_step",):
        if k in bench:
            out.append("%s=%s" % (k, bench[k]))
    _write(a.out, out)


def cmd_traffic(a):
    bench = _bench_line(a.bench_json)
    copy = _bench_line(a.copy_json)
    nread = copy["config"]["bytes_read_per_launch"]
    nwrite = copy["config"]["bytes_written_per_launch"]
    cf = _counter(a.copy_fetch, "FETCH_SIZE", "__amd_rocclr_copyBuffer")
    cw = _counter(a.copy_write, "WRITE_SIZE", "__amd_rocclr_copyBuffer")
    cf, cw = cf[-1], cw[-1]
    sf = nread / (cf * 1024.0)
    sw = nwrite / (cw * 1024.0)
    f = _counter(a.fetch, "FETCH_SIZE", a.kernel)
    w = _counter(a.write, "WRITE_SIZE", a.kernel)
    if a.skip_last:
        f, w = f[:-a.skip_last], w[:-a.skip_last]
    f, w = f[-a.last:], w[-a.last:]
    rd = sf * 1024.0 * sum(f) / len(f)
    wr = sw * 1024.0 * sum(w) / len(w)
    with open(a.hash) as fh:
        h = fh.read().strip()
    alg = bench.get("roofline", {}).get("algorithmic_bytes_per_launch")
    out = ["# rocprofv3 HBM counters of: %s" % a.cmd,
           "# workload: %s" % json.dumps(bench.get("config", {})),
           "# copy calibration: bench.py --mode copy (1 GiB device copy, __amd_rocclr_copyBuffer)",
           "copy_fetch_kib=%.3f" % cf,
           "copy_write_kib=%.3f" % cw,
           "fetch_scale=%.4f" % sf,
           "write_scale=%.4f" % sw,
           "kernel=%s" % a.kernel,
           "dispatches_used=%d" % len(f),
           "dispatches_after_the_used_ones=%d" % a.skip_last,
           "fetch_kib_per_dispatch=%.1f" % (sum(f) / len(f)),
           "write_kib_per_dispatch=%.1f" % (sum(w) / len(w)),
           "hbm_read_bytes_per_launch=%.6e" % rd,
           "hbm_write_bytes_per_launch=%.6e" % wr,
           "hbm_bytes_per_launch=%.6e" % (rd + wr)]
    if alg:
        out += ["algorithmic_bytes_per_launch=%.6e" % alg,
                "traffic_over_algorithmic=%.4f" % ((rd + wr) / alg)]
    out.append("kernel_source_sha256_16=%s" % h)
    _write(a.out, out)


def _write(path, lines):
    with open(path, "w") as fh:
        fh.write("\n".join(lines) + "\n")
    print("\n".join(lines))


def cmd_sq(a):
    rows = _csv(a.dir, "counter_collection.csv")
    names = sorted({r["Counter_Name"] for r in rows})
    mean = {}
    for n in names:
        v = _counter(a.dir, n, a.kernel)
        if a.skip_last:
            v = v[:-a.skip_last]
        v = v[-a.last:]
        if not v:
            raise SystemExit("no %s dispatches of %s under %s" % (n, a.kernel, a.dir))
        mean[n] = sum(v) / len(v)
    waves = mean.get("SQ_WAVES", 0.0)
    out = ["# rocprofv3 SQ counters of: %s" % a.cmd,
           "# workload: %s" % a.workload,
           "# SQ_WAVE_CYCLES, SQ_WAIT_ANY and SQ_ACTIVE_* are summed over waves in one unit, so their ratios are "
           "fractions of the wave lifetime; per_wave = value / SQ_WAVES",
           "kernel=%s" % a.kernel,
           "dispatches_used=%d" % a.last,
           "dispatches_after_the_used_ones=%d" % a.skip_last]
    for n in names:
        pw = " per_wave=%.1f" % (mean[n] / waves) if waves else ""
        out.append("%s=%.1f%s" % (n, mean[n], pw))
    cyc = mean.get("SQ_WAVE_CYCLES")
    if cyc:
        if "SQ_WAIT_ANY" in mean:
            out.append("wait_fraction_of_wave_lifetime=%.3f" % (mean["SQ_WAIT_ANY"] / cyc))
        if "SQ_ACTIVE_INST_VALU" in mean:
            out.append("valu_active_fraction_of_wave_lifetime=%.3f" % (mean["SQ_ACTIVE_INST_VALU"] / cyc))
    gui = mean.get("GRBM_GUI_ACTIVE")
    if gui and "SQ_ACTIVE_INST_VALU" in mean:
        cycles = gui / a.xcds
        out.append("gpu_busy_cycles_per_xcd=%.0f" % cycles)
        out.append("valu_busy_per_simd=%.3f  (SQ_ACTIVE_INST_VALU x 4 / (4 x %d SIMDs x GRBM_GUI_ACTIVE / %d))"
                   % (mean["SQ_ACTIVE_INST_VALU"] * 4.0 / (4 * a.cus * cycles), a.cus, a.xcds))
    _write(a.out, out)


def main():
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd_name", required=True)
    t = sub.add_parser("trace")
    t.add_argument("dir")
    t.add_argument("--kernel", default="k_persistent")
    t.add_argument("--last", type=int, required=True)
    t.add_argument("--bench-json", required=True)
    t.add_argument("--cmd", required=True)
    t.add_argument("--out", required=True)
    t.add_argument("--skip-last", type=int, default=0,
                   help="dispatches of the kernel after the timed ones (left out)")
    t.add_argument("--bench-field", default="roofline.avg_launch_ms",
                   help="the bench.py JSON field with the kernel's own HIP-event launch time")
    p = sub.add_parser("traffic")
    for k in ("--fetch", "--write", "--copy-fetch", "--copy-write", "--bench-json", "--copy-json", "--hash", "--cmd",
              "--out"):
        p.add_argument(k, required=True)
    p.add_argument("--kernel", default="k_persistent")
    p.add_argument("--last", type=int, required=True)
    p.add_argument("--skip-last", type=int, default=0,
                   help="dispatches of the kernel after the ones to average (left out)")
    q = sub.add_parser("sq")
    q.add_argument("dir")
    q.add_argument("--kernel", default="k_persistent")
    q.add_argument("--last", type=int, required=True)
    q.add_argument("--workload", required=True)
    q.add_argument("--cmd", required=True)
    q.add_argument("--out", required=True)
    q.add_argument("--cus", type=int, default=256, help="compute units of the GPU")
    q.add_argument("--xcds", type=int, default=8, help="dies GRBM_GUI_ACTIVE is summed over")
    q.add_argument("--skip-last", type=int, default=0,
                   help="dispatches of the kernel after the ones to average (left out)")
    a = ap.parse_args()
    if a.cmd_name == "trace":
        cmd_trace(a)
    elif a.cmd_name == "sq":
        cmd_sq(a)
    else:
        cmd_traffic(a)


if __name__ == "__main__":
    main()
