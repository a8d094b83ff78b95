"""Summaries of rocprofv3 output for the k-bisimulation kernels.

    python -m paper_2111_12493_amd.profiling stats  <kernel_stats.csv>
    python -m paper_2111_12493_amd.profiling trace  <kernel_trace.csv> <k_done>
    python -m paper_2111_12493_amd.profiling counters <counter_collection.csv> [calib_bytes [k_done]]
    python -m paper_2111_12493_amd.profiling report <workload> <k_done> <algorithmic_bytes>
        <kernel_trace.csv> <fetch_counters.csv> <write_counters.csv> <calib_bytes> <out.json>

`trace` splits the dispatch sequence into summarization runs (one k_init
dispatch starts each run) and averages each kernel over the launches that
did work: refinement launches 1..k_done+1 of every run (the later ones of
the last queued chunk find the stop flag and return at once).

`counters` averages every counter per dispatch for each kernel (with k_done,
over the working refinement launches only).  When the profiled run also
executed one calibration kernel that
reads and writes `calib_bytes` bytes (the largest dispatch not of this
library), FETCH_SIZE and WRITE_SIZE (KiB per dispatch) are scaled by that
kernel's reading to HBM bytes per dispatch.
"""

from __future__ import annotations

import collections
import csv
import hashlib
import json
import os
import sys

CSRC = os.path.join(os.path.dirname(os.path.abspath(__file__)), "csrc")
# sources whose change invalidates counters taken on the refinement kernel
KERNEL_SOURCES = ("bsim_iter.hip", "bsim_device.h", "bsim_internal.h")


def kernel_fingerprint() -> str:
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(CSRC, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]

OWN = ("k_iterate", "k_hub", "k_init", "k_stage_vertices", "k_stage_edges", "k_pack_tiles",
       "k_hub_degrees", "k_hub_starts", "k_salt", "k_compact_flags", "k_fin_min", "k_fin_rep",
       "k_fin_ids", "k_edge_keys", "k_sort_hist", "k_sort_scatter", "k_unique_flags", "k_unpack",
       "k_scan_reduce", "k_scan_spine", "k_scan_down")


def short(name: str) -> str:
    """Kernel name without namespaces, template arguments and parameters."""
    name = name.replace("(anonymous namespace)::", "").replace("void ", "")
    return name.split("(")[0].split("<")[0].split("::")[-1][-48:]


def stats(path: str) -> str:
    rows = list(csv.DictReader(open(path)))
    lines = ["%-40s %8s %12s %10s %7s" % ("kernel", "calls", "total_ms", "avg_us", "pct")]
    for r in rows[:14]:
        lines.append("%-40s %8s %12.2f %10.2f %7.2f" % (short(r["Name"]), r["Calls"],
                                                        int(r["TotalDurationNs"]) / 1e6,
                                                        float(r["AverageNs"]) / 1e3,
                                                        float(r["Percentage"])))
    return "\n".join(lines)


def working_launch_durations(path: str, k_done: int):
    """Per kernel, durations (ns) of the working refinement-loop launches."""
    rows = sorted(csv.DictReader(open(path)), key=lambda r: int(r["Start_Timestamp"]))
    seen = collections.Counter()
    out = collections.defaultdict(list)
    for r in rows:
        k = short(r["Kernel_Name"])
        if k == "k_init":
            seen.clear()
            continue
        seen[k] += 1
        if k in ("k_iterate", "k_hub") and seen[k] <= k_done + 1:
            out[k].append(int(r["End_Timestamp"]) - int(r["Start_Timestamp"]))
    return out


def trace(path: str, k_done: int) -> str:
    d = working_launch_durations(path, k_done)
    lines = ["%-12s %10s %12s   (working launches only)" % ("kernel", "launches", "avg_us")]
    for k, v in sorted(d.items()):
        lines.append("%-12s %10d %12.2f" % (k, len(v), sum(v) / len(v) / 1e3))
    return "\n".join(lines)


def counters(path: str, calib_bytes: int = 0, k_done: int = 0):
    """Per kernel, the average of every counter per dispatch.  With k_done,
    refinement-loop kernels average over their working launches only."""
    per = collections.defaultdict(lambda: collections.defaultdict(float))
    meta = {}
    for r in csv.DictReader(open(path)):
        key = r["Dispatch_Id"]
        per[key][r["Counter_Name"]] += float(r["Counter_Value"])
        meta[key] = (int(r["Start_Timestamp"]), r["Kernel_Name"])
    scale = {}
    if calib_bytes:
        foreign = [per[key] for key in per if short(meta[key][1]) not in OWN]
        for c in ("FETCH_SIZE", "WRITE_SIZE"):
            vals = [cs[c] for cs in foreign if cs.get(c)]
            if vals:
                scale[c] = calib_bytes / max(vals)  # HBM bytes per counted unit
    by_kernel = collections.defaultdict(list)
    seen = collections.Counter()
    for key in sorted(per, key=lambda k: meta[k][0]):
        k = short(meta[key][1])
        if k == "k_init":
            seen.clear()
        seen[k] += 1
        if k_done and k in ("k_iterate", "k_hub") and seen[k] > k_done + 1:
            continue
        by_kernel[k].append(per[key])
    out = {}
    for k, disp in by_kernel.items():
        avg = {c: sum(d.get(c, 0.0) for d in disp) / len(disp) for c in disp[0]}
        entry = {"dispatches": len(disp), "avg": avg}
        for c, f in scale.items():
            if c in avg:
                entry[c.lower() + "_bytes_per_dispatch"] = avg[c] * f
        out[k] = entry
    return out, scale


def report(workload: str, k_done: int, algo_bytes: int, trace_csv: str, fetch_csv: str,
           write_csv: str, calib_bytes: int, out_json: str) -> dict:
    """Traffic of the refinement kernel per working launch, for bench.py."""
    dur = working_launch_durations(trace_csv, k_done)
    f, fs = counters(fetch_csv, calib_bytes, k_done)
    w, ws = counters(write_csv, calib_bytes, k_done)
    res = {"workload": workload, "kernel": "k_iterate", "kernel_sources_sha256_16": kernel_fingerprint(),
           "working_launches": len(dur["k_iterate"]),
           "avg_us": sum(dur["k_iterate"]) / len(dur["k_iterate"]) / 1e3,
           "hub_avg_us": sum(dur["k_hub"]) / max(len(dur["k_hub"]), 1) / 1e3,
           "fetch_bytes_per_launch": f["k_iterate"]["fetch_size_bytes_per_dispatch"],
           "write_bytes_per_launch": w["k_iterate"]["write_size_bytes_per_dispatch"],
           "fetch_scale_bytes_per_unit": fs["FETCH_SIZE"], "write_scale_bytes_per_unit": ws["WRITE_SIZE"],
           "raw_fetch_size_per_launch": f["k_iterate"]["avg"]["FETCH_SIZE"],
           "raw_write_size_per_launch": w["k_iterate"]["avg"]["WRITE_SIZE"],
           "algorithmic_bytes_per_launch": algo_bytes}
    res["bytes_per_launch"] = res["fetch_bytes_per_launch"] + res["write_bytes_per_launch"]
    with open(out_json, "w") as fh:
        json.dump(res, fh, indent=1)
    return res


def main(argv):
    if argv[1] == "stats":
        print(stats(argv[2]))
    elif argv[1] == "report":
        print(json.dumps(report(argv[2], int(argv[3]), int(argv[4]), argv[5], argv[6], argv[7],
                                int(argv[8]), argv[9]), indent=1))
    elif argv[1] == "trace":
        print(trace(argv[2], int(argv[3])))
    else:
        res, scale = counters(argv[2], int(argv[3]) if len(argv) > 3 else 0,
                              int(argv[4]) if len(argv) > 4 else 0)
        print(json.dumps({"scale_bytes_per_unit": scale, "kernels": res}, indent=1))


if __name__ == "__main__":
    main(sys.argv)
