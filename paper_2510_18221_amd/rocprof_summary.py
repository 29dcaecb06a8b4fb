"""Summarise rocprofv3 CSV output of this library's kernels into short markdown.

    python -m paper_2510_18221_amd.rocprof_summary stats   <kernel_stats.csv>
    python -m paper_2510_18221_amd.rocprof_summary trace   <kernel_trace.csv> [--pattern k_forward]
    python -m paper_2510_18221_amd.rocprof_summary traffic <fetch counter_collection.csv> <write ...csv>
        [--copy-bytes N] [--kernel k_forward] [--algorithmic-bytes B]

`traffic` scales FETCH_SIZE / WRITE_SIZE (KiB per dispatch) by what the same
counters report for the largest plain device copy in the run (a copy of N bytes
reads N and writes N bytes), and prints the per-launch HBM traffic of the kernel.
"""
import argparse
import collections
import csv
import hashlib
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))


def forward_source_sha():
    h = hashlib.sha256()
    for f in ("eco_forward.hip", "eco_device.h"):
        h.update(open(os.path.join(HERE, "csrc", f), "rb").read())
    return h.hexdigest()[:16]


def stats(path):
    rows = list(csv.DictReader(open(path)))
    rows.sort(key=lambda r: -float(r["TotalDurationNs"]))
    print("| kernel | calls | avg us | min us | max us | % time |")
    print("|---|---:|---:|---:|---:|---:|")
    for r in rows:
        name = r["Name"]
        if len(name) > 80:
            name = name[:77] + "..."
        print(f"| `{name}` | {r['Calls']} | {float(r['AverageNs']) / 1e3:.1f} | {float(r['MinNs']) / 1e3:.1f} | "
              f"{float(r['MaxNs']) / 1e3:.1f} | {float(r['Percentage']):.2f} |")


def trace(path, pattern):
    """Per-dispatch durations of the kernels whose name contains `pattern` (kernel
    trace CSV): all launches, and the warm ones (every launch after the first of
    each kernel, whose first launch pays for code loading and cold caches)."""
    rows = [r for r in csv.DictReader(open(path)) if pattern in r["Kernel_Name"]]
    by = collections.defaultdict(list)
    for r in sorted(rows, key=lambda r: int(r["Start_Timestamp"])):
        by[r["Kernel_Name"]].append((int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3)
    print("| kernel | launches | mean us | warm launches | warm mean us | warm median us | min us |")
    print("|---|---:|---:|---:|---:|---:|---:|")
    for k, d in sorted(by.items(), key=lambda kv: -sum(kv[1])):
        warm = sorted(d[1:]) if len(d) > 1 else d
        name = k if len(k) < 70 else k[:67] + "..."
        print(f"| `{name}` | {len(d)} | {sum(d) / len(d):.1f} | {len(warm)} | {sum(warm) / len(warm):.1f} | "
              f"{warm[len(warm) // 2]:.1f} | {min(d):.1f} |")


def per_kernel(path, counter):
    agg = collections.defaultdict(list)
    for r in csv.DictReader(open(path)):
        if r["Counter_Name"] == counter:
            agg[r["Kernel_Name"]].append(float(r["Counter_Value"]))
    return agg


def traffic(fetch_csv, write_csv, copy_bytes, kernel, algorithmic):
    f = per_kernel(fetch_csv, "FETCH_SIZE")
    w = per_kernel(write_csv, "WRITE_SIZE")
    copy_f = max(max(v) for k, v in f.items() if "copyBuffer" in k)
    copy_w = max(max(v) for k, v in w.items() if "copyBuffer" in k)
    kib = copy_bytes / 1024.0
    sf, sw = kib / copy_f, kib / copy_w
    print(f"copy probe: {copy_bytes} B copied; FETCH_SIZE {copy_f:.1f} KiB -> scale {sf:.4f}; "
          f"WRITE_SIZE {copy_w:.1f} KiB -> scale {sw:.4f}")
    print()
    print("| kernel | dispatches | FETCH KiB (raw avg) | WRITE KiB (raw avg) | scaled read B | scaled write B |")
    print("|---|---:|---:|---:|---:|---:|")
    target = None
    for k in sorted(f, key=lambda k: -sum(f[k]) / len(f[k])):
        fa = sum(f[k]) / len(f[k])
        wa = sum(w.get(k, [0.0])) / max(len(w.get(k, [0.0])), 1)
        rb, wb = fa * sf * 1024, wa * sw * 1024
        name = k if len(k) < 70 else k[:67] + "..."
        print(f"| `{name}` | {len(f[k])} | {fa:.1f} | {wa:.1f} | {rb:.4g} | {wb:.4g} |")
        if kernel in k:
            target = (rb, wb)
    if target:
        rb, wb = target
        print()
        print(f"traffic_bytes_per_launch: {rb + wb:.6g}")
        if algorithmic:
            print(f"algorithmic_bytes_per_launch: {algorithmic:.6g}")
            print(f"traffic_over_algorithmic: {(rb + wb) / algorithmic:.4f}")
        print(f"source_sha256: {forward_source_sha()}")


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("mode", choices=["stats", "traffic", "trace"])
    ap.add_argument("--pattern", default="k_forward", help="trace: kernels whose name contains this")
    ap.add_argument("files", nargs="+")
    ap.add_argument("--copy-bytes", type=float, default=float(4 << 30))
    ap.add_argument("--kernel", default="k_forward")
    ap.add_argument("--algorithmic-bytes", type=float, default=0.0)
    a = ap.parse_args(argv)
    if a.mode == "stats":
        stats(a.files[0])
    elif a.mode == "trace":
        trace(a.files[0], a.pattern)
    else:
        traffic(a.files[0], a.files[1], a.copy_bytes, a.kernel, a.algorithmic_bytes)


if __name__ == "__main__":
    sys.exit(main())
