"""Summaries of rocprofv3 output for the k-bisimulation kernels.

    python -m paper_2111_12493_amd.profiling stats  <kernel_stats.csv>
    python -m paper_2111_12493_amd.profiling trace  <kernel_trace.csv> <k_done>
    python -m paper_2111_12493_amd.profiling counters <counter_collection.csv> [calib_bytes [k_done]]
    python -m paper_2111_12493_amd.profiling summary <dir> <workload> <k_done> <algorithmic_bytes> <calib_bytes> <out_dir>
    python -m paper_2111_12493_amd.profiling report <workload> <k_done> <algorithmic_bytes>
        <kernel_trace.csv> <fetch_counters.csv> <write_counters.csv> <calib_bytes> <out.json>
    python -m paper_2111_12493_amd.profiling updates <incremental|plain> <batches>
    python -m paper_2111_12493_amd.profiling summary-updates <dir> <batches> <out_dir>

`updates` runs the update workload (the resident rmat24 state, k = 4, the
bench's seeded batches of 10^3-10^6 operations) in one form, for a profiler
to wrap; `summary-updates` turns the two kernel-stat tables
(<dir>/incremental, <dir>/plain) into profiles/updates_rmat24.md.

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


COMMANDS = """    rocprofv3 --kernel-trace --stats -d {d}/stats -o run --output-format csv -- \\
        python -u bench.py --no-cpu-baseline --no-incremental --no-batched --no-serving --no-directions --steps 2 --warmup 1
    rocprofv3 --pmc FETCH_SIZE -d {d}/fetch -o run --output-format csv -- \\
        python -u bench.py --no-cpu-baseline --no-incremental --no-batched --no-serving --no-directions --steps 1 --warmup 0 --calibrate-copy 1024
    rocprofv3 --pmc WRITE_SIZE -d {d}/write -o run --output-format csv -- \\
        python -u bench.py --no-cpu-baseline --no-incremental --no-batched --no-serving --no-directions --steps 1 --warmup 0 --calibrate-copy 1024
    rocprofv3 --pmc SQ_WAVES SQ_BUSY_CYCLES SQ_WAVE_CYCLES SQ_WAIT_ANY SQ_WAIT_INST_LDS SQ_INSTS_VALU \\
        SQ_INSTS_LDS SQ_LDS_BANK_CONFLICT -d {d}/sq1 -o run --output-format csv -- \\
        python -u bench.py --no-cpu-baseline --no-incremental --no-batched --no-serving --no-directions --steps 1 --warmup 0
    rocprofv3 --pmc SQ_INSTS_VMEM_RD SQ_INSTS_VMEM_WR SQ_ACTIVE_INST_VALU SQ_ACTIVE_INST_LDS \\
        SQ_ACTIVE_INST_VMEM SQ_INST_CYCLES_VMEM_RD GRBM_GUI_ACTIVE TCC_HIT -d {d}/sq2 -o run \\
        --output-format csv -- python -u bench.py --no-cpu-baseline --no-incremental --no-batched --no-serving --no-directions --steps 1 --warmup 0
"""


def summary(d: str, workload: str, k_done: int, algo_bytes: int, calib_bytes: int, out_dir: str) -> str:
    """Write <out_dir>/k_iterate_<workload>.md and _counters.json from the
    five rocprofv3 runs under directory d (see COMMANDS)."""
    j = os.path.join
    rep = report(workload, k_done, algo_bytes, j(d, "stats", "run_kernel_trace.csv"),
                 j(d, "fetch", "run_counter_collection.csv"), j(d, "write", "run_counter_collection.csv"),
                 calib_bytes, j(out_dir, "k_iterate_%s_counters.json" % workload))
    sq = []
    derived = {}
    for pas in ("sq1", "sq2"):
        res, _ = counters(j(d, pas, "run_counter_collection.csv"), 0, k_done)
        for k in ("k_iterate", "k_hub"):
            if k in res:
                avg = res[k]["avg"]
                derived.setdefault(k, {}).update(avg)
                sq.append("%s %s" % (k, " ".join("%s=%.4g" % kv for kv in sorted(avg.items()))))
    lines = ["# k_iterate / k_hub on %s (%d iterations)" % (workload, k_done), "",
             "Kernel source fingerprint (%s): %s" % (", ".join(KERNEL_SOURCES), rep["kernel_sources_sha256_16"]), "",
             "## Commands (repository root, one MI355X)", "", COMMANDS.format(d=d), "Summaries:", "",
             "    python -m paper_2111_12493_amd.profiling summary %s %s %d %d %d profiles"
             % (d, workload, k_done, algo_bytes, calib_bytes), "",
             "## Kernel stats (every dispatch of the profiled runs)", "", "```",
             stats(j(d, "stats", "run_kernel_stats.csv")), "```", "",
             "Launches past the stop test of a run return at once; over the working launches "
             "(1..k_done+1 of every run):", "", "```", trace(j(d, "stats", "run_kernel_trace.csv"), k_done), "```", "",
             "## HBM traffic per working k_iterate launch", "",
             "Calibration kernel (torch bitwise_not over %d bytes: reads and writes that many): one FETCH_SIZE "
             "unit = %.1f bytes, one WRITE_SIZE unit = %.1f bytes." % (calib_bytes, rep["fetch_scale_bytes_per_unit"],
                                                                       rep["write_scale_bytes_per_unit"]), "",
             "| | raw units | bytes |", "|---|---:|---:|",
             "| FETCH_SIZE | %.0f | %.1f MB |" % (rep["raw_fetch_size_per_launch"], rep["fetch_bytes_per_launch"] / 1e6),
             "| WRITE_SIZE | %.0f | %.1f MB |" % (rep["raw_write_size_per_launch"], rep["write_bytes_per_launch"] / 1e6),
             "| total | | %.1f MB |" % (rep["bytes_per_launch"] / 1e6),
             "| algorithmic | | %.1f MB |" % (algo_bytes / 1e6), "",
             "Measured / algorithmic = %.2f." % (rep["bytes_per_launch"] / algo_bytes), "",
             "## Issue counters per working launch", "", "```"] + sq + ["```", ""]
    k = derived.get("k_iterate", {})
    if k.get("GRBM_GUI_ACTIVE") and k.get("SQ_ACTIVE_INST_VALU"):
        busy = k["SQ_ACTIVE_INST_VALU"] * 4 / 1024 / (k["GRBM_GUI_ACTIVE"] / 8)
        wait = k.get("SQ_WAIT_ANY", 0) / max(k.get("SQ_WAVE_CYCLES", 1), 1)
        lines.append("k_iterate: VALU busy = SQ_ACTIVE_INST_VALU x 4 / 1024 SIMDs / (GRBM_GUI_ACTIVE / 8 XCDs) "
                     "= %.0f %%; SQ_WAIT_ANY / SQ_WAVE_CYCLES = %.0f %%." % (100 * busy, 100 * wait))
    path = j(out_dir, "k_iterate_%s.md" % workload)
    with open(path, "w") as fh:
        fh.write("\n".join(lines) + "\n")
    return path


UPDATE_COMMAND = """    rocprofv3 --kernel-trace --stats -d {d}/{form} -o run --output-format csv -- \\
        python -u -m paper_2111_12493_amd.profiling updates {form} {batches}"""


def run_updates(form: str, batches: int) -> None:
    """The update workload of the bench's incremental leg, one form only."""
    import time

    import numpy as np
    import torch

    from . import binding, devgen
    from . import graphgen as gg

    dg = devgen.make_device_config("rmat24")
    g = dg.to_host()
    ctx = binding.Context(0)
    if form == "plain":
        ctx.set_option("frontier_limit_pct", 0)
    st = binding.State(ctx, dg, 4, stop_at_fixpoint=False, summary_edges=False)
    st.result.free()
    rng = np.random.default_rng(17)
    dead = np.zeros(g.n + 4_000_000, dtype=bool)
    n = g.n
    for i in range(batches):
        size = int(round(10 ** rng.uniform(3, 6)))
        d = gg.sample_update_ops(g.row_off, g.tgt, g.lab, n, dead, rng, size, max(g.n_labels, 1),
                                 max(g.n_types, 1), rmat_scale=24)
        n = d["n_after"]
        batch = binding.UpdateBatch.from_op_arrays(d)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = st.apply(batch)
        wall = (time.perf_counter() - t0) * 1e3
        print("%s batch %d (%d ops): %.2f ms | merge %.2f, levels %.2f, classes+final %.2f"
              % (form, i, size, wall, r.ms_stage, r.ms_iterate, r.ms_finalize), file=sys.stderr, flush=True)
        r.free()
    st.free()
    ctx.close()


def summary_updates(d: str, batches: int, out_dir: str) -> str:
    lines = ["# Update batches on the resident rmat24 state (k = 4)", "",
             "2^24 vertices, 2^27 edges (R-MAT, drawn on the GPU), the bench's seeded batches of "
             "log-uniform 10^3-10^6 operations; one process per form.  The tables cover the whole "
             "process: graph generation (torch kernels, not listed), the state's creation (one "
             "refinement of levels 1-4 and its class passes) and %d update batches." % batches, "",
             "## Commands (repository root, one MI355X)", ""]
    for form in ("incremental", "plain"):
        lines.append(UPDATE_COMMAND.format(d=d, form=form, batches=batches))
    lines.append("")
    for form in ("incremental", "plain"):
        path = os.path.join(d, form, "run_kernel_stats.csv")
        rows = [r for r in csv.DictReader(open(path)) if short(r["Name"]).startswith("k_")]
        total = sum(int(r["TotalDurationNs"]) for r in rows)
        lines += ["## %s form: library kernels" % form, "",
                  "```", "%-28s %7s %11s %10s %13s" % ("kernel", "calls", "total_ms", "avg_us", "ms/update"),
                  "%-28s %7s %11.2f" % ("(all library kernels)", "", total / 1e6)]
        for r in rows[:16]:
            t = int(r["TotalDurationNs"])
            lines.append("%-28s %7s %11.2f %10.1f %13.2f" % (short(r["Name"]), r["Calls"], t / 1e6,
                                                            float(r["AverageNs"]) / 1e3, t / 1e6 / (batches + 1)))
        lines += ["```", ""]
    lines.append("ms/update divides by the batches plus the creation, which does the same kinds of work once.")
    os.makedirs(out_dir, exist_ok=True)
    out = os.path.join(out_dir, "updates_rmat24.md")
    with open(out, "w") as fh:
        fh.write("\n".join(lines) + "\n")
    return out


BATCHED_COMMAND = """    rocprofv3 --kernel-trace --stats -d {d} -o run --output-format csv -- \\
        python -u -m paper_2111_12493_amd.profiling batched {runs}"""


def run_batched(runs: int) -> None:
    """The batched workload of the bench's batched leg: 4,096 R-MAT graphs
    drawn on the GPU, summarized by `runs` batched calls (the first one a
    warm-up, like the bench's)."""
    import time

    import torch

    from . import binding, devgen

    graphs = devgen.batched_device(4096, 1e6, seed=23)
    ctx = binding.Context(0)
    print("batched: %d graphs, %d edges" % (len(graphs), sum(g.m for g in graphs)), flush=True)
    for i in range(runs):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        rs = binding.batch_summarize(ctx, graphs, summary_edges=True)
        torch.cuda.synchronize()
        print("run %d: %.1f ms, max k_done %d" % (i, (time.perf_counter() - t0) * 1e3, max(r.k_done for r in rs)),
              flush=True)
        for r in rs:
            r.free()
    ctx.close()


def summary_batched(d: str, runs: int, out_dir: str) -> str:
    path = os.path.join(d, "run_kernel_stats.csv")
    rows = [r for r in csv.DictReader(open(path)) if short(r["Name"]).startswith("k_")]
    total = sum(int(r["TotalDurationNs"]) for r in rows)
    lines = ["# Batched summarization of 4,096 R-MAT graphs", "",
             "4,096 graphs with edge counts log-uniform in 10^2-10^6 (4.28e8 edges in all), degree U(4, 16), "
             "32 types and 32 labels (Zipf 1.0), drawn on the GPU; %d batched calls (each graph to its own "
             "fixpoint), the first a warm-up." % runs, "",
             "## Command (repository root, one MI355X)", "",
             BATCHED_COMMAND.format(d=d, runs=runs), "",
             "## Library kernels (all calls)", "", "```",
             "%-28s %7s %11s %10s %11s" % ("kernel", "calls", "total_ms", "avg_us", "ms/call"),
             "%-28s %7s %11.2f %10s %11.2f" % ("(all library kernels)", "", total / 1e6, "", total / 1e6 / runs)]
    for r in rows[:16]:
        t = int(r["TotalDurationNs"])
        lines.append("%-28s %7s %11.2f %10.1f %11.2f" % (short(r["Name"]), r["Calls"], t / 1e6,
                                                        float(r["AverageNs"]) / 1e3, t / 1e6 / runs))
    lines += ["```", ""]
    os.makedirs(out_dir, exist_ok=True)
    out = os.path.join(out_dir, "batched_4096_rmat.md")
    with open(out, "w") as fh:
        fh.write("\n".join(lines) + "\n")
    return out


def main(argv):
    if argv[1] == "batched":
        run_batched(int(argv[2]))
        return
    if argv[1] == "summary-batched":
        print(summary_batched(argv[2], int(argv[3]), argv[4]))
        return
    if argv[1] == "updates":
        run_updates(argv[2], int(argv[3]))
        return
    if argv[1] == "summary-updates":
        print(summary_updates(argv[2], int(argv[3]), argv[4]))
        return
    if argv[1] == "summary":
        print(summary(argv[2], argv[3], int(argv[4]), int(argv[5]), int(argv[6]), argv[7]))
        return
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
