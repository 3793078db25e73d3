"""Turns rocprofv3 CSV output into the short text summaries kept under
profiles/.

  python -m paper_2104_12282_amd.profile_summary stats <kernel_stats.csv> <out.md> "<command>"

`stats` lists the kernels with the largest total time and, from the kernel
trace next to the statistics file, how much of the traced span the GPU was
busy and how long it sat between kernels.
  python -m paper_2104_12282_amd.profile_summary traffic <fetch_dir> <write_dir> <bench.json> <out.json> "<commands>" [<kernel_stats.csv>]

`traffic` reads two counter runs (FETCH_SIZE, then WRITE_SIZE, in KiB per
dispatch), scales each by what the same counter reads for the plain copy of
known size that bench.py --copy-probe performs (hipMemcpy device-to-device,
kernel __amd_rocclr_copyBuffer), and stores the bytes per launch of the tiled
K*u kernel and of the coarse Chebyshev pair kernels next to the digest of the
sources it was measured on; given the
kernel statistics of a --kernel-trace run of the same sources, it also
stores each kernel's average duration there (all launches, and the launches
that did their work: the kernel trace next to the statistics file gives the
per-launch durations), and every kernel's share of the traced GPU time.
"""
from __future__ import annotations

import csv
import glob
import json
import os
import sys


def _rows(path):
    with open(path, newline="") as fh:
        return list(csv.DictReader(fh))


def stats(csv_path, out_path, command):
    rows = _rows(csv_path)
    rows.sort(key=lambda r: -float(r["TotalDurationNs"]))
    total = sum(float(r["TotalDurationNs"]) for r in rows)
    lines = ["# rocprofv3 kernel statistics", "", f"Command: `{command}`", "",
             "| kernel | calls | total ms | avg us | min us | max us | % |",
             "|---|---:|---:|---:|---:|---:|---:|"]
    for r in rows[:20]:
        name = r["Name"]
        if len(name) > 90:
            name = name[:90] + "..."
        lines.append(f"| `{name}` | {r['Calls']} | {float(r['TotalDurationNs']) / 1e6:.3f} | "
                     f"{float(r['AverageNs']) / 1e3:.2f} | {float(r['MinNs']) / 1e3:.2f} | "
                     f"{float(r['MaxNs']) / 1e3:.2f} | {100 * float(r['TotalDurationNs']) / total:.1f} |")
    lines += _timeline(os.path.dirname(csv_path))
    lines += _by_shape(os.path.dirname(csv_path))
    with open(out_path, "w") as fh:
        fh.write("\n".join(lines) + "\n")


def _timeline(run_dir, short_ns=50_000):
    """Busy time and idle gaps of the kernel trace next to the statistics:
    a gap under `short_ns` between one kernel's end and the next one's start
    is the dispatch of a queued kernel, a longer one is host work between
    launches."""
    traces = glob.glob(os.path.join(run_dir, "*kernel_trace.csv"))
    if not traces:
        return []
    spans = sorted((int(r["Start_Timestamp"]), int(r["End_Timestamp"])) for r in _rows(traces[0]))
    if len(spans) < 2:
        return []
    busy = sum(e - s for s, e in spans)
    gaps = sorted(max(0, s - e0) for (_, e0), (s, _) in zip(spans, spans[1:]))
    short = [g for g in gaps if g < short_ns]
    long_ = [g for g in gaps if g >= short_ns]
    span = spans[-1][1] - spans[0][0]
    med = short[len(short) // 2] if short else 0
    return ["", "Timeline of the kernel trace of the same run:", "",
            f"* span {span / 1e6:.3f} ms, kernels busy {busy / 1e6:.3f} ms ({100 * busy / span:.1f}%)",
            f"* {len(short)} gaps under {short_ns / 1e3:.0f} us between one kernel's end and the next "
            f"one's start (dispatch of queued work, timed under the trace): median {med / 1e3:.2f} us, "
            f"total {sum(short) / 1e6:.3f} ms",
            f"* {len(long_)} longer gaps (host work between launches): total {sum(long_) / 1e6:.3f} ms"]


def _by_shape(run_dir, top=24):
    """The kernels of the trace split by launch shape (grid size: one kernel
    runs on several multigrid levels), largest total first, with the mean
    and median durations of each."""
    traces = glob.glob(os.path.join(run_dir, "*kernel_trace.csv"))
    if not traces:
        return []
    groups = {}
    for r in _rows(traces[0]):
        name = r["Kernel_Name"].replace("void ", "").replace("(anonymous namespace)::", "").split("(")[0]
        key = (name, int(r["Grid_Size_X"]) * int(r["Grid_Size_Y"]) * int(r["Grid_Size_Z"]),
               int(r["Workgroup_Size_X"]) * int(r["Workgroup_Size_Y"]) * int(r["Workgroup_Size_Z"]))
        groups.setdefault(key, []).append((int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3)
    total = sum(sum(v) for v in groups.values())
    lines = ["", "By launch shape (work-items of the grid, workgroup size):", "",
             "| kernel | grid | workgroup | calls | total ms | mean us | median us | % |",
             "|---|---:|---:|---:|---:|---:|---:|---:|"]
    for (name, grid, wg), ds in sorted(groups.items(), key=lambda kv: -sum(kv[1]))[:top]:
        ds = sorted(ds)
        lines.append(f"| `{name[:60]}` | {grid} | {wg} | {len(ds)} | {sum(ds) / 1e3:.3f} | "
                     f"{sum(ds) / len(ds):.2f} | {ds[len(ds) // 2]:.2f} | {100 * sum(ds) / total:.1f} |")
    return lines


def _counter_by_kernel(run_dir, counter):
    files = glob.glob(os.path.join(run_dir, "**", "*counter_collection.csv"), recursive=True)
    if not files:
        raise SystemExit(f"no counter_collection.csv under {run_dir}")
    out = {}
    for r in _rows(files[0]):
        if r.get("Counter_Name") != counter:
            continue
        out.setdefault(r["Kernel_Name"], []).append(float(r["Counter_Value"]))
    return out


def traffic(fetch_dir, write_dir, bench_json, out_path, command, stats_csv=None):
    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    from paper_2104_12282_amd.build import source_digest
    probe = json.load(open(bench_json))["copy_probe"]
    fetch = _counter_by_kernel(fetch_dir, "FETCH_SIZE")
    write = _counter_by_kernel(write_dir, "WRITE_SIZE")

    def pick(d, key):
        vals = [v for k, vs in d.items() if key in k for v in vs]
        return vals

    copy_f = max(pick(fetch, "copyBuffer"))  # the probe is the largest copy
    copy_w = max(pick(write, "copyBuffer"))
    f_scale = probe["bytes"] / (copy_f * 1024.0)
    w_scale = probe["bytes"] / (copy_w * 1024.0)
    rec = {"source_digest": source_digest(), "command": command,
           "copy_probe_bytes": probe["bytes"], "copy_fetch_kib": copy_f, "copy_write_kib": copy_w,
           "fetch_scale": f_scale, "write_scale": w_scale, "kernels": {}}
    for mode_key in sorted({k for k in fetch if any(n in k for n in ("kxu_tile_kernel", "cheb3d_kernel",
                                                                    "cheb3t_kernel", "cheb2_kernel"))}):
        fk = fetch[mode_key]
        wk = write.get(mode_key, [])
        if not wk:
            continue
        # the finest grid's launches are the largest of each K*u variant (each
        # Chebyshev launch form runs on one level of the hierarchy; launches
        # that met the CG stop flag read almost nothing)
        fmax, wmax = max(fk), max(wk)
        rec["kernels"][mode_key] = {"fetch_bytes": fmax * 1024 * f_scale,
                                    "write_bytes": wmax * 1024 * w_scale,
                                    "launches_seen": len(fk)}
    if stats_csv:
        # per-launch durations from the kernel trace of the same run: the mean
        # over launches that did their work (those that met the CG stop flag
        # return at once; launches shorter than a quarter of the kernel's
        # longest are left out)
        work = {}
        traces = glob.glob(os.path.join(os.path.dirname(stats_csv), "*kernel_trace.csv"))
        if traces:
            durs = {}
            for r in _rows(traces[0]):
                durs.setdefault(r["Kernel_Name"], []).append(
                    (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3)
            for name, ds in durs.items():
                kept = [d for d in ds if d >= 0.25 * max(ds)]
                work[name] = sum(kept) / len(kept)
        rows = _rows(stats_csv)
        total = sum(float(r["TotalDurationNs"]) for r in rows)
        rec["time_shares"] = []  # every kernel of the kernel-trace run, largest total first
        for r in sorted(rows, key=lambda r: -float(r["TotalDurationNs"])):
            name = r["Name"].replace("void ", "").replace("(anonymous namespace)::", "").split("(")[0]
            rec["time_shares"].append({"kernel": name, "calls": int(r["Calls"]),
                                       "avg_us": float(r["AverageNs"]) / 1e3,
                                       "work_avg_us": work.get(r["Name"]),
                                       "share": float(r["TotalDurationNs"]) / total})
            if r["Name"] in rec["kernels"]:
                rec["kernels"][r["Name"]]["trace_avg_us"] = float(r["AverageNs"]) / 1e3
                rec["kernels"][r["Name"]]["trace_work_avg_us"] = work.get(r["Name"])
                rec["kernels"][r["Name"]]["trace_max_us"] = float(r["MaxNs"]) / 1e3
    with open(out_path, "w") as fh:
        json.dump(rec, fh, indent=1)


if __name__ == "__main__":
    if sys.argv[1] == "stats":
        stats(sys.argv[2], sys.argv[3], sys.argv[4])
    elif sys.argv[1] == "traffic":
        traffic(sys.argv[2], sys.argv[3], sys.argv[4], sys.argv[5], sys.argv[6],
                sys.argv[7] if len(sys.argv) > 7 else None)
    else:
        raise SystemExit(__doc__)
