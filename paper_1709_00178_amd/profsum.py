"""Summaries of rocprofv3 CSV output for the committed profiles.

    python -m paper_1709_00178_amd.profsum stats  <run_kernel_stats.csv>  --cmd "..." \\
        [--marker NAME --kernel NAME] [--by-grid TEXT] > out.md
    python -m paper_1709_00178_amd.profsum traffic --fetch <dir> --write <dir> --kernel NAME \\
        --copy-bytes N --record KEY [--algorithmic BYTES] [--fetch-kib LO:HI] \\
        [--write-kib LO:HI] [--copy-fetch <dir> --copy-write <dir>] --cmd "..." > out.md

`traffic` turns per-dispatch FETCH_SIZE and WRITE_SIZE (KiB) of a kernel
into HBM bytes per launch, each scaled by what the same counter reads for the
library's copy kernel moving a known number of bytes (half read, half
written), and updates profiles/traffic.json with the kernel-source hash the
benchmark checks before reporting the figure.
"""
from __future__ import annotations

import argparse
import csv
import glob
import hashlib
import json
import os
import statistics

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
KERNEL_SOURCES = ["paper_1709_00178_amd/csrc/rings.hpp",
                  "paper_1709_00178_amd/csrc/ring_kernels.hpp",
                  "paper_1709_00178_amd/csrc/plain_impl.hpp",
                  "paper_1709_00178_amd/csrc/batch_abi.hpp",
                  "paper_1709_00178_amd/csrc/batch.hip"]


def kernel_hash() -> str:
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def trace_medians(stats_path: str) -> dict:
    """Median dispatch duration (us) per kernel name from the kernel trace
    written beside the stats file, when there is one."""
    trace = stats_path.replace("kernel_stats.csv", "kernel_trace.csv")
    if trace == stats_path or not os.path.exists(trace):
        return {}
    d: dict = {}
    for r in csv.DictReader(open(trace)):
        d.setdefault(r["Kernel_Name"], []).append(
            (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3)
    return {k: statistics.median(v) for k, v in d.items()}


def stats_table(path: str) -> str:
    rows = list(csv.DictReader(open(path)))
    med = trace_medians(path)
    out = ["| kernel | calls | avg us | median us | min us | max us | total % |",
           "|---|---:|---:|---:|---:|---:|---:|"]
    for r in rows:
        m = med.get(r["Name"])
        out.append(f"| `{r['Name']}` | {r['Calls']} | {float(r['AverageNs']) / 1e3:.1f} | "
                   f"{'%.1f' % m if m is not None else '-'} | "
                   f"{float(r['MinNs']) / 1e3:.1f} | {float(r['MaxNs']) / 1e3:.1f} | "
                   f"{float(r['Percentage']):.1f} |")
    return "\n".join(out)


def grid_table(stats_path: str, needle: str) -> str:
    """Dispatch durations per (kernel, grid size) for the kernels whose name
    holds `needle`, from the kernel trace beside the stats file: one row per
    launch shape, so calls of one kernel on different block sizes stay apart."""
    tpath = stats_path.replace("kernel_stats.csv", "kernel_trace.csv")
    d: dict = {}
    for r in csv.DictReader(open(tpath)):
        if needle in r["Kernel_Name"]:
            key = (r["Kernel_Name"], int(r["Grid_Size_X"]), int(r["Workgroup_Size_X"]))
            d.setdefault(key, []).append((int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3)
    out = ["| kernel | grid (threads) | workgroup | calls | mean us | median us | min us | max us |",
           "|---|---:|---:|---:|---:|---:|---:|---:|"]
    for (name, grid, wg), v in sorted(d.items()):
        out.append(f"| `{name}` | {grid} | {wg} | {len(v)} | {statistics.fmean(v):.1f} | "
                   f"{statistics.median(v):.1f} | {min(v):.1f} | {max(v):.1f} |")
    return "\n".join(out)


def marked_launches(stats_path: str, marker: str, kernel: str):
    """Durations (us) of the dispatches of `kernel` that ran wholly inside
    the marker range `marker` (rocprofv3 --marker-trace beside the stats)."""
    mpath = stats_path.replace("kernel_stats.csv", "marker_api_trace.csv")
    tpath = stats_path.replace("kernel_stats.csv", "kernel_trace.csv")
    ranges = [(int(r["Start_Timestamp"]), int(r["End_Timestamp"]))
              for r in csv.DictReader(open(mpath)) if r["Function"] == marker]
    if len(ranges) != 1:
        raise SystemExit(f"marker '{marker}' found {len(ranges)} times")
    t0, t1 = ranges[0]
    out = []
    for r in csv.DictReader(open(tpath)):
        a, b = int(r["Start_Timestamp"]), int(r["End_Timestamp"])
        if kernel in r["Kernel_Name"] and t0 <= a and b <= t1:
            out.append((b - a) / 1e3)
    return out


def kib_range(text: str):
    """'LO:HI' in KiB (either side may be empty) -> (lo, hi)."""
    lo, _, hi = text.partition(":")
    return float(lo or 0.0), float(hi or "inf")


def counter_means(directory: str, counter: str, kib=(0.0, float("inf"))) -> dict:
    """Mean value of `counter` per kernel name over its dispatches, keeping
    only dispatches whose value lies in the KiB range `kib` (the launches of
    one workload when the same kernel codes other shapes in the run)."""
    files = glob.glob(os.path.join(directory, "**", "*counter_collection.csv"), recursive=True)
    vals: dict = {}
    for fn in files:
        for r in csv.DictReader(open(fn)):
            if r["Counter_Name"] == counter and kib[0] <= float(r["Counter_Value"]) <= kib[1]:
                vals.setdefault(r["Kernel_Name"], []).append(float(r["Counter_Value"]))
    return {k: (statistics.fmean(v), len(v)) for k, v in vals.items()}


def find(d: dict, needle: str):
    hits = [k for k in d if needle in k]
    if len(hits) != 1:
        raise SystemExit(f"kernel '{needle}' matched {hits}")
    return d[hits[0]], hits[0]


def main():
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="what", required=True)
    a = sub.add_parser("stats")
    a.add_argument("csv")
    a.add_argument("--cmd", required=True)
    a.add_argument("--marker", default="")
    a.add_argument("--kernel", default="")
    a.add_argument("--by-grid", default="", help="also tabulate, per grid size, the kernels "
                   "whose name holds this text")
    b = sub.add_parser("traffic")
    b.add_argument("--fetch", required=True)
    b.add_argument("--write", required=True)
    b.add_argument("--kernel", required=True)
    b.add_argument("--copy-kernel", default="copy_kernel")
    b.add_argument("--copy-bytes", type=int, required=True)
    b.add_argument("--copy-fetch", default="", help="FETCH_SIZE run holding the copy kernel "
                   "(default: the --fetch run)")
    b.add_argument("--copy-write", default="", help="WRITE_SIZE run holding the copy kernel "
                   "(default: the --write run)")
    b.add_argument("--fetch-kib", default=":", help="LO:HI, keep dispatches whose FETCH_SIZE "
                   "(KiB) lies in the range")
    b.add_argument("--write-kib", default=":", help="LO:HI, the same for WRITE_SIZE")
    b.add_argument("--record", required=True)
    b.add_argument("--algorithmic", type=int, default=0)
    b.add_argument("--cmd", required=True)
    args = ap.parse_args()
    if args.what == "stats":
        print(f"Command: `{args.cmd}`\n")
        print(stats_table(args.csv))
        if args.by_grid:
            print("\nPer launch shape:\n")
            print(grid_table(args.csv, args.by_grid))
        if args.marker:
            d = marked_launches(args.csv, args.marker, args.kernel)
            print(f"\nInside the marker range `{args.marker}` (the bench's timed steps): "
                  f"{len(d)} launches of `{args.kernel}`, mean {statistics.fmean(d):.1f} us, "
                  f"median {statistics.median(d):.1f} us, min {min(d):.1f} us, "
                  f"max {max(d):.1f} us.")
        return
    fetch = counter_means(args.fetch, "FETCH_SIZE", kib_range(args.fetch_kib))
    write = counter_means(args.write, "WRITE_SIZE", kib_range(args.write_kib))
    (kf, nf), name = find(fetch, args.kernel)
    (kw, nw), _ = find(write, args.kernel)
    (cf, _), _ = find(counter_means(args.copy_fetch or args.fetch, "FETCH_SIZE"), args.copy_kernel)
    (cw, _), _ = find(counter_means(args.copy_write or args.write, "WRITE_SIZE"), args.copy_kernel)
    half_kib = args.copy_bytes / 2 / 1024
    f_scale, w_scale = half_kib / cf, half_kib / cw
    traffic = int(round((kf * f_scale + kw * w_scale) * 1024))
    path = os.path.join(ROOT, "profiles", "traffic.json")
    rec = json.load(open(path)) if os.path.exists(path) else {}
    rec[args.record] = {"kernel": name, "kernel_hash": kernel_hash(), "bytes_per_launch": traffic,
                        "fetch_kib": round(kf, 1), "write_kib": round(kw, 1),
                        "fetch_scale": round(f_scale, 4), "write_scale": round(w_scale, 4),
                        "dispatches": [nf, nw], "command": args.cmd}
    with open(path, "w") as f:
        json.dump(rec, f, indent=1, sort_keys=True)
        f.write("\n")
    print(f"Command: `{args.cmd}` (one `--pmc FETCH_SIZE` run, one `--pmc WRITE_SIZE` run)\n")
    print(f"Kernel: `{name}`\n")
    if args.fetch_kib != ":" or args.write_kib != ":":
        print(f"Dispatches kept: FETCH_SIZE in [{args.fetch_kib}] KiB and WRITE_SIZE in "
              f"[{args.write_kib}] KiB (this workload's launches; the same kernel codes other "
              f"shapes in the run).\n")
    if args.copy_fetch or args.copy_write:
        print(f"Copy-kernel calibration from the runs `{args.copy_fetch or args.fetch}` and "
              f"`{args.copy_write or args.write}` (same counters, same session).\n")
    print("| quantity | value |\n|---|---:|")
    print(f"| FETCH_SIZE per dispatch (KiB, mean of {nf}) | {kf:.1f} |")
    print(f"| WRITE_SIZE per dispatch (KiB, mean of {nw}) | {kw:.1f} |")
    print(f"| copy kernel FETCH_SIZE (KiB) for {half_kib:.0f} KiB read | {cf:.1f} |")
    print(f"| copy kernel WRITE_SIZE (KiB) for {half_kib:.0f} KiB written | {cw:.1f} |")
    print(f"| FETCH scale (true / counted) | {f_scale:.4f} |")
    print(f"| WRITE scale (true / counted) | {w_scale:.4f} |")
    print(f"| HBM bytes per launch (scaled) | {traffic} |")
    if args.algorithmic:
        print(f"| algorithmic bytes per launch | {args.algorithmic} |")
        print(f"| traffic / algorithmic | {traffic / args.algorithmic:.4f} |")


if __name__ == "__main__":
    main()
