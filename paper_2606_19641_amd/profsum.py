"""Condense rocprofv3 CSV output into the short text summaries kept with the
measurements.

  python -m paper_2606_19641_amd.profsum trace DIR [--match NAME ...]
      kernel durations per kernel and launch shape from DIR/*kernel_trace.csv
      (and the --stats table from DIR/*kernel_stats.csv when present)
  python -m paper_2606_19641_amd.profsum counters DIR [--match NAME ...]
      per-dispatch averages of every counter in DIR/*counter_collection.csv
  python -m paper_2606_19641_amd.profsum hbm --fetch DIR --write DIR --sq DIR --kernel NAME
        --workload NAME --launch JSON --bytes N
      HBM bytes per launch of one kernel from a FETCH_SIZE pass and a
      WRITE_SIZE pass, each scaled by what the same counter reads for the
      plain copy (torch.neg over 256 MiB of float32: 256 MiB read, 256 MiB
      written) that the same run made, beside the kernel's SQ counters; ends
      with the machine-read fields the benchmark matches (kernel source hash,
      workload, launch setting)

Columns of the trace table, as rocprofv3 reports them: `wgs` workgroups of the
dispatch (grid size / workgroup size), `wg` threads per workgroup, `vgpr`
rocprofv3's VGPR_Count, which on gfx950 reads half the architected VGPRs a
lane is allocated (the compiler's count rounded up to the granule of 8, then
halved: 128 -> 64, 73 -> 40, 17 -> 12; the compiler's own figure comes from
hipcc -Rpass-analysis=kernel-resource-usage), `agpr` the accumulation VGPRs,
`lds` rocprofv3's LDS_Block_Size, the kernel's static LDS rounded up to the
512-byte allocation granule (dynamic LDS given at launch is not included),
`scratch` private memory per lane in bytes (register spills); durations in ns
from the dispatch's start and end timestamps.
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


def trace_by_name(d: str, match=None) -> str:
    """Durations per kernel name, every launch shape together."""
    rows = list(csv.DictReader(open(_one(os.path.join(d, "*kernel_trace.csv")))))
    agg = collections.defaultdict(list)
    for r in rows:
        if match and not any(m in r["Kernel_Name"] for m in match):
            continue
        agg[short_name(r["Kernel_Name"])].append(int(r["End_Timestamp"]) - int(r["Start_Timestamp"]))
    out = ["  %-52s %7s %10s %10s %10s %10s" % ("kernel", "calls", "avg_ns", "p50_ns", "max_ns", "total_ms")]
    for name, v in sorted(agg.items(), key=lambda kv: -sum(kv[1])):
        v = sorted(v)
        out.append("  %-52s %7d %10.0f %10d %10d %10.2f" %
                   (name, len(v), sum(v) / len(v), v[len(v) // 2], v[-1], sum(v) / 1e6))
    return "\n".join(out)


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


COPY_BYTES = 256 << 20
COPY_KERNEL = "neg"


def _per_dispatch(d: str, kernel: str) -> dict:
    """Mean of each counter over the dispatches of the kernels whose name holds `kernel`."""
    rows = list(csv.DictReader(open(_one(os.path.join(d, "*counter_collection.csv")))))
    tot, disp = collections.defaultdict(float), set()
    for r in rows:
        if kernel in r["Kernel_Name"]:
            tot[r["Counter_Name"]] += float(r["Counter_Value"])
            disp.add(r["Dispatch_Id"])
    if not disp:
        raise SystemExit(f"no dispatch of {kernel} in {d}")
    return {k: v / len(disp) for k, v in tot.items()}, len(disp)


def hbm(fetch_dir, write_dir, sq_dir, kernel, workload, launch, alg_bytes) -> str:
    from .tune import kernel_source_sha
    f, nf = _per_dispatch(fetch_dir, kernel)
    w, nw = _per_dispatch(write_dir, kernel)
    q, nq = _per_dispatch(sq_dir, kernel) if sq_dir else ({}, 0)
    cf, _ = _per_dispatch(fetch_dir, COPY_KERNEL)
    cw, _ = _per_dispatch(write_dir, COPY_KERNEL)
    sf = COPY_BYTES / (cf["FETCH_SIZE"] * 1024)
    sw = COPY_BYTES / (cw["WRITE_SIZE"] * 1024)
    fb = f["FETCH_SIZE"] * 1024 * sf
    wb = w["WRITE_SIZE"] * 1024 * sw
    out = [f"calibration: torch.neg over 256 MiB of float32 (256 MiB read, 256 MiB written)",
           f"  FETCH_SIZE {cf['FETCH_SIZE']:.1f} KiB per dispatch -> scale {sf:.4f}; "
           f"WRITE_SIZE {cw['WRITE_SIZE']:.1f} KiB per dispatch -> scale {sw:.4f}",
           f"{kernel}: averages over {nf} / {nw} / {nq} dispatches (fetch / write / SQ pass)",
           f"  FETCH_SIZE {f['FETCH_SIZE']:.1f} KiB -> {fb / 1e6:.3f} MB after scaling",
           f"  WRITE_SIZE {w['WRITE_SIZE']:.1f} KiB -> {wb / 1e6:.3f} MB after scaling",
           f"  HBM traffic {(fb + wb) / 1e6:.3f} MB per launch; algorithmic bytes {alg_bytes / 1e6:.3f} MB "
           f"-> traffic / algorithmic {(fb + wb) / alg_bytes:.4f}"]
    for k in sorted(q):
        out.append(f"  {k} {q[k]:.4f}")
    out += ["",
            "machine-read fields (the benchmark reports traffic only while the kernel source, workload "
            "and launch setting match):",
            f"kernel_source_sha256: {kernel_source_sha()}",
            f"workload: {workload}",
            f"launch: {launch}",
            f"kernel: {kernel}",
            f"algorithmic_bytes_per_launch: {alg_bytes}",
            f"fetch_bytes_per_launch: {fb:.0f}",
            f"write_bytes_per_launch: {wb:.0f}",
            f"traffic_bytes_per_launch: {fb + wb:.0f}"]
    if q:
        out += [f"valu_busy_pct: {q.get('VALUBusy', float('nan')):.3f}",
                f"lds_bank_conflict_pct: {q.get('LDSBankConflict', float('nan')):.3f}",
                f"valu_insts_per_launch: {q.get('SQ_INSTS_VALU', float('nan')):.0f}"]
    return "\n".join(out)


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("kind", choices=("trace", "counters", "hbm"))
    ap.add_argument("dir", nargs="?")
    ap.add_argument("--match", nargs="*")
    ap.add_argument("--by-name", action="store_true", help="trace: every launch shape of a kernel together")
    ap.add_argument("--fetch")
    ap.add_argument("--write")
    ap.add_argument("--sq")
    ap.add_argument("--kernel")
    ap.add_argument("--workload")
    ap.add_argument("--launch")
    ap.add_argument("--bytes", type=int)
    a = ap.parse_args(argv)
    if a.kind == "hbm":
        print(hbm(a.fetch, a.write, a.sq, a.kernel, a.workload, a.launch, a.bytes))
    elif a.kind == "trace":
        print(trace_by_name(a.dir, a.match) if a.by_name else trace(a.dir, a.match))
    else:
        print(counters(a.dir, a.match))


if __name__ == "__main__":
    sys.exit(main())
