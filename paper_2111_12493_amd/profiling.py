"""Summaries of rocprofv3 output for the k-bisimulation kernels.

    python -m paper_2111_12493_amd.profiling stats  <kernel_stats.csv>
    python -m paper_2111_12493_amd.profiling counters <counter_collection.csv> [copy_bytes]

`counters` averages every counter per dispatch for each kernel (dispatches
that returned at once, i.e. launches queued past the stop point, are left
out by taking the dispatches whose first counter is in the upper half), and
when the run included one device-to-device copy of `copy_bytes` bytes it
scales FETCH_SIZE / WRITE_SIZE (KiB per dispatch) by that copy's reading to
HBM bytes per dispatch.
"""

from __future__ import annotations

import collections
import csv
import json
import sys


def short(name: str) -> str:
    for key in ("k_iterate", "k_hub", "k_init", "copyBuffer"):
        if key in name:
            return key
    return name.split("(")[0][-40:]


def stats(path: str) -> str:
    rows = list(csv.DictReader(open(path)))
    lines = ["%-12s %8s %14s %12s %7s" % ("kernel", "calls", "total_ms", "avg_us", "pct")]
    for r in rows[:12]:
        lines.append("%-12s %8s %14.2f %12.2f %7s" % (short(r["Name"]), r["Calls"],
                                                        int(r["TotalDurationNs"]) / 1e6,
                                                        float(r["AverageNs"]) / 1e3,
                                                        r["Percentage"][:6]))
    return "\n".join(lines)


def counters(path: str, copy_bytes: int = 0):
    per = collections.defaultdict(lambda: collections.defaultdict(float))
    names = {}
    for r in csv.DictReader(open(path)):
        key = r.get("Dispatch_Id") or r.get("Correlation_Id")
        per[key][r["Counter_Name"]] += float(r["Counter_Value"])
        names[key] = r["Kernel_Name"]
    by_kernel = collections.defaultdict(list)
    for key, cs in per.items():
        by_kernel[short(names[key])].append(cs)
    out = {}
    scale = {}
    if copy_bytes and "copyBuffer" in by_kernel:
        big = max(by_kernel["copyBuffer"], key=lambda c: c.get("FETCH_SIZE", c.get("WRITE_SIZE", 0)))
        for c in ("FETCH_SIZE", "WRITE_SIZE"):
            if big.get(c):
                scale[c] = copy_bytes / big[c]  # bytes per counted KiB
    for k, disp in by_kernel.items():
        first = sorted(disp[0].keys())[0]
        vals = sorted(d[first] for d in disp)
        cut = vals[len(vals) // 2] * 0.5 if len(vals) > 2 else -1
        use = [d for d in disp if d[first] >= cut] or disp
        avg = {c: sum(d.get(c, 0.0) for d in use) / len(use) for c in disp[0]}
        entry = {"dispatches": len(disp), "averaged_over": len(use), "avg": avg}
        for c, f in scale.items():
            if c in avg:
                entry[c.lower() + "_bytes_per_dispatch"] = avg[c] * f
        out[k] = entry
    return out, scale


def main(argv):
    if argv[1] == "stats":
        print(stats(argv[2]))
    else:
        res, scale = counters(argv[2], int(argv[3]) if len(argv) > 3 else 0)
        print(json.dumps({"scale_bytes_per_counted_kib": scale, "kernels": res}, indent=1))


if __name__ == "__main__":
    main(sys.argv)
