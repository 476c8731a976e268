"""Condense rocprofv3 CSV output into the short text summaries kept with the
measurements.

  python -m paper_2606_19641_amd.profsum trace DIR [--match NAME ...]
      kernel durations per kernel and launch shape from DIR/*kernel_trace.csv
      (and the --stats table from DIR/*kernel_stats.csv when present)
  python -m paper_2606_19641_amd.profsum counters DIR [--match NAME ...]
      per-dispatch averages of every counter in DIR/*counter_collection.csv

Columns of the trace table, as rocprofv3 reports them: `wgs` workgroups of the
dispatch (grid size / workgroup size), `wg` threads per workgroup, `vgpr` the
architected VGPRs per thread as allocated (rocprofv3's VGPR_Count, rounded up
to the allocation granule), `agpr` the accumulation VGPRs, `lds` the
kernel's static LDS in bytes (rocprofv3's LDS_Block_Size: dynamic LDS given at
launch is not included), `scratch` private memory per thread in bytes;
durations in ns from the dispatch's start and end timestamps.
"""
from __future__ import annotations

import argparse
import collections
import csv
import glob
import os
import sys


def _one(pattern: str) -> str:
    found = sorted(glob.glob(pattern))
    if not found:
        raise SystemExit(f"no file matches {pattern}")
    return found[0]


def short_name(name: str, width: int = 60) -> str:
    name = name.replace("(anonymous namespace)::", "")
    cut = name.find("(")
    if cut > 0:
        name = name[:cut]
    name = name.replace("void ", "")
    return name[:width]


def trace(d: str, match=None) -> str:
    rows = list(csv.DictReader(open(_one(os.path.join(d, "*kernel_trace.csv")))))
    agg = collections.OrderedDict()
    for r in rows:
        if match and not any(m in r["Kernel_Name"] for m in match):
            continue
        wg = int(r["Workgroup_Size_X"]) * int(r.get("Workgroup_Size_Y", 1) or 1) * int(r.get("Workgroup_Size_Z", 1) or 1)
        grid = int(r["Grid_Size_X"]) * int(r.get("Grid_Size_Y", 1) or 1) * int(r.get("Grid_Size_Z", 1) or 1)
        key = (short_name(r["Kernel_Name"]), grid // max(wg, 1), wg, r.get("VGPR_Count", ""),
               r.get("Accum_VGPR_Count", ""), r.get("LDS_Block_Size", ""), r.get("Scratch_Size", ""))
        agg.setdefault(key, []).append(int(r["End_Timestamp"]) - int(r["Start_Timestamp"]))
    out = ["  %-52s %7s %5s %5s %5s %7s %7s %7s %10s %10s %10s" %
           ("kernel", "wgs", "wg", "vgpr", "agpr", "lds", "scratch", "calls", "avg_ns", "min_ns", "max_ns")]
    for key, v in sorted(agg.items(), key=lambda kv: -sum(kv[1])):
        name, wgs, wg, vg, ag, lds, scr = key
        out.append("  %-52s %7d %5d %5s %5s %7s %7s %7d %10.0f %10d %10d" %
                   (name, wgs, wg, vg, ag, lds, scr, len(v), sum(v) / len(v), min(v), max(v)))
    stats = sorted(glob.glob(os.path.join(d, "*kernel_stats.csv")))
    if stats:
        out.append("")
        out.append("rocprofv3 --stats (kernel_stats.csv, launch shapes together):")
        for r in csv.DictReader(open(stats[0])):
            if match and not any(m in r["Name"] for m in match):
                continue
            out.append("  %-52s calls %7s avg_ns %12.0f total%% %6.2f" %
                       (short_name(r["Name"]), r["Calls"], float(r["AverageNs"]), float(r["Percentage"])))
    return "\n".join(out)


def counters(d: str, match=None) -> str:
    rows = list(csv.DictReader(open(_one(os.path.join(d, "*counter_collection.csv")))))
    per = collections.defaultdict(lambda: collections.defaultdict(float))
    disp = collections.defaultdict(set)
    for r in rows:
        if match and not any(m in r["Kernel_Name"] for m in match):
            continue
        k = short_name(r["Kernel_Name"])
        per[k][r["Counter_Name"]] += float(r["Counter_Value"])
        disp[k].add(r["Dispatch_Id"])
    out = []
    for k, cs in per.items():
        n = max(len(disp[k]), 1)
        out.append(f"  {k}: {n} dispatches")
        for c, v in sorted(cs.items()):
            out.append(f"    {c:28s} {v / n:16.1f} per dispatch")
    return "\n".join(out)


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("kind", choices=("trace", "counters"))
    ap.add_argument("dir")
    ap.add_argument("--match", nargs="*")
    a = ap.parse_args(argv)
    print(trace(a.dir, a.match) if a.kind == "trace" else counters(a.dir, a.match))


if __name__ == "__main__":
    sys.exit(main())
