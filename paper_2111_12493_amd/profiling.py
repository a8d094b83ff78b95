"""Summaries of rocprofv3 output for the k-bisimulation kernels.

    python -m paper_2111_12493_amd.profiling stats  <kernel_stats.csv>
    python -m paper_2111_12493_amd.profiling trace  <kernel_trace.csv> <k_done>
    python -m paper_2111_12493_amd.profiling counters <counter_collection.csv> [calib_bytes [k_done]]
    python -m paper_2111_12493_amd.profiling summary <dir> <workload> <k_done> <algorithmic_bytes> <calib_bytes> <out_dir> [hash_launches]
    python -m paper_2111_12493_amd.profiling probes <workload> <out_dir>
    python -m paper_2111_12493_amd.profiling updates <incremental|plain> <batches>
    python -m paper_2111_12493_amd.profiling summary-updates <dir> <batches> <out_dir>

`summary` reads the kernel-trace run and the four counter passes that
commands() lists and writes profiles/k_iterate_<workload>.md and its
_counters.json (the traffic bench.py reports); `probes` times a STREAM-style
copy and the gather pattern of the refinement (bsim_probe_copy,
bsim_probe_gather) and writes profiles/probes_<workload>.md.

`updates` runs the update workload (the resident rmat24 state, k = 4, the
bench's seeded batches of 10^3-10^6 operations) in one form, for a profiler
to wrap; `summary-updates` turns the two kernel-stat tables
(<dir>/incremental, <dir>/plain) into profiles/updates_rmat24.md.

`trace` splits the dispatch sequence into summarization runs (one k_init
dispatch starts each run) and averages each kernel over the launches that
did work: refinement launches 1..k_done+1 of every run (the later ones of
the last queued chunk find the stop flag and return at once), or 1..k_done
when the run's launch k_done+1 ran as a split launch (its hash half finds
the stop, so only launches 1..k_done hashed a level): `hash_launches` says
which.

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


# Every profiled command runs one warm-up summarization first (it sizes the
# context's kept work buffer, so the measured runs place their temporaries
# as the timed bench steps do); the summaries skip that run.
SKIP_RUNS = 1


def working_launch_durations(path: str, k_done: int, n_work: int = 0, skip_runs: int = SKIP_RUNS):
    """Per kernel, durations (ns) of the working refinement-loop launches
    (the first n_work of every run after the first skip_runs; default
    n_work = k_done + 1)."""
    n_work = n_work or k_done + 1
    rows = sorted(csv.DictReader(open(path)), key=lambda r: int(r["Start_Timestamp"]))
    seen = collections.Counter()
    out = collections.defaultdict(list)
    run = 0
    for r in rows:
        k = short(r["Kernel_Name"])
        if k == "k_init":
            seen.clear()
            run += 1
            continue
        seen[k] += 1
        if run <= skip_runs:
            continue
        if k in ("k_iterate", "k_hub", "k_hub_finish") and seen[k] <= n_work:
            out[k].append(int(r["End_Timestamp"]) - int(r["Start_Timestamp"]))
    return out


def trace(path: str, k_done: int, n_work: int = 0) -> str:
    d = working_launch_durations(path, k_done, n_work)
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


ITER_KERNELS = ("k_iterate", "k_hub", "k_hub_finish")

# Counter passes (rocprofv3 collects no more than 4 TCC counters at once).
#   fetch: bytes read past L2 = 128 TCC_BUBBLE + 64 (TCC_EA0_RDREQ - TCC_BUBBLE
#          - TCC_EA0_RDREQ_32B) + 32 TCC_EA0_RDREQ_32B (rocprofv3's FETCH_SIZE
#          for gfx950), and TCC_EA0_RDREQ_DRAM (requests that went to DRAM)
#   l2:    TCC_HIT / TCC_MISS (the L2 hit rate of the gathers) and the write
#          requests of WRITE_SIZE: 32 (TCC_EA0_WRREQ - TCC_EA0_WRREQ_64B) + 64 TCC_EA0_WRREQ_64B
PASSES = {
    "fetch": "TCC_EA0_RDREQ_sum TCC_EA0_RDREQ_32B_sum TCC_BUBBLE_sum TCC_EA0_RDREQ_DRAM_sum",
    "l2": "TCC_HIT_sum TCC_MISS_sum TCC_EA0_WRREQ_sum TCC_EA0_WRREQ_64B_sum",
    "sq1": "SQ_WAVES SQ_BUSY_CYCLES SQ_WAVE_CYCLES SQ_WAIT_ANY SQ_WAIT_INST_LDS SQ_INSTS_VALU SQ_INSTS_LDS "
           "SQ_LDS_BANK_CONFLICT",
    "sq2": "SQ_INSTS_VMEM_RD SQ_INSTS_VMEM_WR SQ_ACTIVE_INST_VALU SQ_ACTIVE_INST_LDS SQ_ACTIVE_INST_VMEM "
           "SQ_INST_CYCLES_VMEM_RD GRBM_GUI_ACTIVE",
}
BENCH_ARGS = "--no-cpu-baseline --no-chaining --no-incremental --no-batched --no-serving --no-directions"


def commands(d: str, workload: str) -> str:
    b = "python -u bench.py --workload %s %s" % (workload, BENCH_ARGS)
    lines = ["    rocprofv3 --kernel-trace --stats -d %s/stats -o run --output-format csv -- \\" % d,
             "        %s --steps 2 --warmup 1" % b]
    for name, ctrs in PASSES.items():
        calib = " --calibrate-copy 1024" if name in ("fetch", "l2") else ""
        lines += ["    timeout -s KILL 300 rocprofv3 --pmc %s -d %s/%s -o run --output-format csv -- \\" % (ctrs, d, name),
                  "        %s --steps 1 --warmup 1%s" % (b, calib)]
    return "\n".join(lines)


def fetch_bytes(avg: dict) -> float:
    bub, rd, r32 = avg.get("TCC_BUBBLE_sum", 0.0), avg.get("TCC_EA0_RDREQ_sum", 0.0), avg.get("TCC_EA0_RDREQ_32B_sum", 0.0)
    return 128 * bub + 64 * (rd - bub - r32) + 32 * r32


def write_bytes(avg: dict) -> float:
    wr, w64 = avg.get("TCC_EA0_WRREQ_sum", 0.0), avg.get("TCC_EA0_WRREQ_64B_sum", 0.0)
    return 32 * (wr - w64) + 64 * w64


def pass_counters(path: str, k_done: int, n_work: int = 0, skip_runs: int = SKIP_RUNS):
    """Per kernel (working launches of the refinement loop only, runs after
    the first skip_runs), the average of every counter per dispatch, and the
    counters of the foreign dispatches (the calibration copy)."""
    per = collections.defaultdict(lambda: collections.defaultdict(float))
    meta = {}
    for r in csv.DictReader(open(path)):
        key = r["Dispatch_Id"]
        per[key][r["Counter_Name"]] += float(r["Counter_Value"])
        meta[key] = (int(r["Start_Timestamp"]), r["Kernel_Name"])
    by_kernel = collections.defaultdict(list)
    seen = collections.Counter()
    foreign = []
    run = 0
    for key in sorted(per, key=lambda k: meta[k][0]):
        k = short(meta[key][1])
        if k not in OWN and k not in ITER_KERNELS and not k.startswith("k_"):
            foreign.append(per[key])
            continue
        if k == "k_init":
            seen.clear()
            run += 1
        seen[k] += 1
        if run <= skip_runs:
            continue
        if k in ITER_KERNELS and seen[k] > (n_work or k_done + 1):
            continue
        by_kernel[k].append(per[key])
    avg = {k: {c: sum(d.get(c, 0.0) for d in v) / len(v) for c in v[0]} for k, v in by_kernel.items()}
    return avg, foreign


def summary(d: str, workload: str, k_done: int, algo_bytes: int, calib_bytes: int, out_dir: str,
            n_work: int = 0) -> str:
    """Write <out_dir>/k_iterate_<workload>.md and _counters.json from the
    rocprofv3 runs under directory d (see commands()).  n_work: the
    refinement launches per run that hashed a level (default k_done + 1)."""
    j = os.path.join
    n_work = n_work or k_done + 1
    dur = working_launch_durations(j(d, "stats", "run_kernel_trace.csv"), k_done, n_work)
    iter_us = sum(sum(dur[k]) / len(dur[k]) for k in ITER_KERNELS if dur.get(k)) / 1e3
    fa, ff = pass_counters(j(d, "fetch", "run_counter_collection.csv"), k_done, n_work)
    la, lf = pass_counters(j(d, "l2", "run_counter_collection.csv"), k_done, n_work)
    copy_read = max(fetch_bytes(c) for c in ff) if ff else 0.0
    copy_write = max(write_bytes(c) for c in lf) if lf else 0.0
    rs = calib_bytes / copy_read if copy_read else 1.0   # true bytes per counted byte
    ws = calib_bytes / copy_write if copy_write else 1.0
    fetch = sum(fetch_bytes(fa.get(k, {})) for k in ITER_KERNELS)
    write = sum(write_bytes(la.get(k, {})) for k in ITER_KERNELS)
    ki_f, ki_l = fa.get("k_iterate", {}), la.get("k_iterate", {})
    hit, miss = ki_l.get("TCC_HIT_sum", 0.0), ki_l.get("TCC_MISS_sum", 0.0)
    rep = {"workload": workload, "kernels": list(ITER_KERNELS), "kernel_sources_sha256_16": kernel_fingerprint(),
           "working_launches": len(dur.get("k_iterate", [])), "iteration_avg_us": iter_us,
           "avg_us": {k: sum(dur[k]) / len(dur[k]) / 1e3 for k in ITER_KERNELS if dur.get(k)},
           "counted_fetch_bytes_per_iteration": fetch, "counted_write_bytes_per_iteration": write,
           "copy_read_scale": rs, "copy_write_scale": ws,
           "fetch_bytes_per_launch": fetch * rs, "write_bytes_per_launch": write * ws,
           "k_iterate_l2_hit_rate": hit / (hit + miss) if hit + miss else None,
           "k_iterate_dram_read_share": (ki_f.get("TCC_EA0_RDREQ_DRAM_sum", 0.0) / ki_f["TCC_EA0_RDREQ_sum"]
                                         if ki_f.get("TCC_EA0_RDREQ_sum") else None),
           "algorithmic_bytes_per_launch": algo_bytes}
    rep["bytes_per_launch"] = rep["fetch_bytes_per_launch"] + rep["write_bytes_per_launch"]
    with open(j(out_dir, "k_iterate_%s_counters.json" % workload), "w") as fh:
        json.dump(rep, fh, indent=1)
    sq = []
    derived = {}
    for pas in ("sq1", "sq2"):
        res, _ = pass_counters(j(d, pas, "run_counter_collection.csv"), k_done, n_work)
        for k in ITER_KERNELS:
            if k in res:
                derived.setdefault(k, {}).update(res[k])
                sq.append("%s %s" % (k, " ".join("%s=%.4g" % kv for kv in sorted(res[k].items()))))
    tcc = []
    for k in ITER_KERNELS:
        for name, src in (("fetch", fa), ("l2", la)):
            if k in src:
                tcc.append("%s %s" % (k, " ".join("%s=%.4g" % kv for kv in sorted(src[k].items()))))
    lines = ["# One refinement iteration (k_iterate, k_hub, k_hub_finish) on %s (%d iterations per run)"
             % (workload, k_done), "",
             "Kernel source fingerprint (%s): %s" % (", ".join(KERNEL_SOURCES), rep["kernel_sources_sha256_16"]), "",
             "## Commands (repository root, one MI355X)", "", commands(d, workload), "", "Summaries:", "",
             "    python -m paper_2111_12493_amd.profiling summary %s %s %d %d %d profiles %d"
             % (d, workload, k_done, algo_bytes, calib_bytes, n_work), "",
             "## Kernel stats (every dispatch of the profiled runs)", "", "```",
             stats(j(d, "stats", "run_kernel_stats.csv")), "```", "",
             "Launches past the stop test of a run return at once; over the launches that hashed a "
             "level (1..%d of every run but the first, the warm-up run that sizes the context's work "
             "buffer; the counter tables below skip it too):" % n_work, "", "```",
             trace(j(d, "stats", "run_kernel_trace.csv"), k_done, n_work), "```", "",
             "One iteration = %.1f us; algorithmic bytes %.1f MB -> %.0f GB/s = %.1f %% of 8 TB/s."
             % (iter_us, algo_bytes / 1e6, algo_bytes / iter_us / 1e3, algo_bytes / iter_us / 1e3 / 80), "",
             "## Bytes past L2 per working iteration", "",
             "Read bytes = 128 TCC_BUBBLE + 64 (TCC_EA0_RDREQ - TCC_BUBBLE - TCC_EA0_RDREQ_32B) + 32 TCC_EA0_RDREQ_32B "
             "(rocprofv3's FETCH_SIZE for gfx950), write bytes = 32 (TCC_EA0_WRREQ - TCC_EA0_WRREQ_64B) + "
             "64 TCC_EA0_WRREQ_64B.  The calibration copy (torch bitwise_not over %d bytes, reads and writes that "
             "many) counted %.0f read and %.0f written bytes: true/counted = %.3f (read), %.3f (write)."
             % (calib_bytes, copy_read, copy_write, rs, ws), "",
             "| | counted | scaled by the copy |", "|---|---:|---:|",
             "| read | %.1f MB | %.1f MB |" % (fetch / 1e6, rep["fetch_bytes_per_launch"] / 1e6),
             "| written | %.1f MB | %.1f MB |" % (write / 1e6, rep["write_bytes_per_launch"] / 1e6),
             "| total | %.1f MB | %.1f MB |" % ((fetch + write) / 1e6, rep["bytes_per_launch"] / 1e6),
             "| algorithmic | | %.1f MB |" % (algo_bytes / 1e6), "",
             "Scaled traffic / algorithmic = %.2f." % (rep["bytes_per_launch"] / algo_bytes), ""]
    if rep["k_iterate_l2_hit_rate"] is not None:
        lines.append("k_iterate: L2 hit rate TCC_HIT / (TCC_HIT + TCC_MISS) = %.1f %%." % (100 * rep["k_iterate_l2_hit_rate"]))
    if rep["k_iterate_dram_read_share"] is not None:
        lines.append("k_iterate: TCC_EA0_RDREQ_DRAM / TCC_EA0_RDREQ = %.1f %% of the read requests past L2 went to "
                     "DRAM; the rest were served by the memory-side cache." % (100 * rep["k_iterate_dram_read_share"]))
    lines += ["", "## Counters per working launch", "", "```"] + tcc + sq + ["```", ""]
    k = derived.get("k_iterate", {})
    if k.get("GRBM_GUI_ACTIVE") and k.get("SQ_ACTIVE_INST_VALU"):
        busy = k["SQ_ACTIVE_INST_VALU"] * 4 / 1024 / (k["GRBM_GUI_ACTIVE"] / 8)
        wait = k.get("SQ_WAIT_ANY", 0) / max(k.get("SQ_WAVE_CYCLES", 1), 1)
        lines.append("k_iterate: VALU busy = SQ_ACTIVE_INST_VALU x 4 / 1024 SIMDs / (GRBM_GUI_ACTIVE / 8 XCDs) "
                     "= %.0f %%; SQ_WAIT_ANY / SQ_WAVE_CYCLES = %.0f %%." % (100 * busy, 100 * wait))
    if k.get("SQ_INSTS_LDS"):
        lines.append("k_iterate: SQ_LDS_BANK_CONFLICT / SQ_INSTS_LDS = %.2f cycles per LDS instruction."
                     % (k.get("SQ_LDS_BANK_CONFLICT", 0) / k["SQ_INSTS_LDS"]))
    path = j(out_dir, "k_iterate_%s.md" % workload)
    with open(path, "w") as fh:
        fh.write("\n".join(lines) + "\n")
    return path


def run_probes(workload: str, out_dir: str) -> str:
    """The memory-pattern ceilings of the refinement on a workload: a
    STREAM-style copy, and the gather probe (stream the targets, gather one
    8-byte value per edge) over the graph's targets as generated, with the
    vertices renumbered by descending in-degree, and with random ids."""
    import torch

    from . import binding
    from . import graphgen as gg

    torch.cuda.set_device(0)
    ctx = binding.Context(0)
    lines = ["# Memory-pattern ceilings on %s" % workload, "",
             "Command (repository root, one MI355X):", "",
             "    python -u -m paper_2111_12493_amd.profiling probes %s %s" % (workload, out_dir), ""]
    gib = 4 << 30
    ms = binding.probe_copy(ctx, gib, reps=10)
    copy_gbs = 2 * gib / ms / 1e6
    lines += ["STREAM-style copy of %d GiB (read + write): %.3f ms -> %.0f GB/s (%.1f %% of 8 TB/s)."
              % (gib >> 30, ms, copy_gbs, copy_gbs / 80), ""]
    g = gg.make_config(workload)
    dg = binding.DeviceGraph(g)
    n, m = g.n, g.m
    del g
    h = torch.zeros(max(n, 1), dtype=torch.int64, device="cuda")
    tgt0 = dg.tgt.clone()
    lines += ["Gather probe over the %d targets of %s (n = %d), gathering from an %d-entry 8-byte array; "
              "algorithmic bytes = 12 per edge (4 B target + 8 B gathered value):" % (m, workload, n, n), "",
              "| vertex ids | ms per pass | GB/s | % of 8 TB/s |", "|---|---:|---:|---:|"]
    indeg = torch.bincount(tgt0.to(torch.int64), minlength=n)
    rank = torch.empty(n, dtype=torch.int64, device="cuda")
    rank[torch.argsort(indeg, descending=True, stable=True)] = torch.arange(n, device="cuda")
    gen = torch.Generator(device="cuda")
    gen.manual_seed(1)
    variants = (("as generated", tgt0),
                ("renumbered by in-degree", rank[tgt0.to(torch.int64)].to(torch.int32)),
                ("random permutation", torch.randperm(n, generator=gen, device="cuda")[tgt0.to(torch.int64)]
                 .to(torch.int32)),
                ("sequential (e mod n)", (torch.arange(m, device="cuda") % n).to(torch.int32)))
    res = {}
    for name, t in variants:
        dg.tgt = t.contiguous()
        ms = binding.probe_gather(ctx, dg, h, reps=10)
        gbs = 12 * m / ms / 1e6
        res[name] = ms
        lines.append("| %s | %.3f | %.0f | %.1f |" % (name, ms, gbs, gbs / 80))
    dg.tgt = tgt0
    lines.append("")
    ctx.close()
    os.makedirs(out_dir, exist_ok=True)
    path = os.path.join(out_dir, "probes_%s.md" % workload)
    with open(path, "w") as fh:
        fh.write("\n".join(lines) + "\n")
    print("\n".join(lines))
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
    # k_types runs once per batched run: the calls plus the autotuner's
    # candidate runs on the first call of the size class
    n_run = sum(int(r["Calls"]) for r in rows if short(r["Name"]) == "k_types") or runs
    lines = ["# Batched summarization of 4,096 R-MAT graphs", "",
             "4,096 graphs with edge counts log-uniform in 10^2-10^6 (4.28e8 edges in all), degree U(4, 16), "
             "32 types and 32 labels (Zipf 1.0), drawn on the GPU; %d batched calls (each graph to its own "
             "fixpoint) on a fresh context.  The first call of the size class autotunes: it runs the first "
             "candidate once untimed (that run sizes the context's work buffer), every candidate schedule on "
             "the batch, and then the fastest, so the profile holds %d batched runs; ms/run divides by them."
             % (runs, n_run), "",
             "## Command (repository root, one MI355X)", "",
             BATCHED_COMMAND.format(d=d, runs=runs), "",
             "## Library kernels (all runs)", "", "```",
             "%-28s %7s %11s %10s %11s" % ("kernel", "calls", "total_ms", "avg_us", "ms/run"),
             "%-28s %7s %11.2f %10s %11.2f" % ("(all library kernels)", "", total / 1e6, "", total / 1e6 / n_run)]
    for r in rows[:16]:
        t = int(r["TotalDurationNs"])
        lines.append("%-28s %7s %11.2f %10.1f %11.2f" % (short(r["Name"]), r["Calls"], t / 1e6,
                                                        float(r["AverageNs"]) / 1e3, t / 1e6 / n_run))
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
        print(summary(argv[2], argv[3], int(argv[4]), int(argv[5]), int(argv[6]), argv[7],
                      int(argv[8]) if len(argv) > 8 else 0))
        return
    if argv[1] == "probes":
        run_probes(argv[2], argv[3])
        return
    if argv[1] == "stats":
        print(stats(argv[2]))
    elif argv[1] == "trace":
        print(trace(argv[2], int(argv[3])))
    else:
        res, scale = counters(argv[2], int(argv[3]) if len(argv) > 3 else 0,
                              int(argv[4]) if len(argv) > 4 else 0)
        print(json.dumps({"scale_bytes_per_unit": scale, "kernels": res}, indent=1))


if __name__ == "__main__":
    main(sys.argv)
