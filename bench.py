#!/usr/bin/env python3
"""Benchmark of the MI355X k-bisimulation path.

One step = one full batch summarization (staging, type hashes, refinement
iterations to the fixpoint or the cap, relabel, block sizes, summary edges)
of one device-resident synthetic graph through the C ABI.  Default workload
(rmat27): an R-MAT graph (a, b, c = 0.57, 0.19, 0.19) with 2^27 vertices and
2^30 edges, 1,024 type labels (Zipf 1.2, 0-4 per vertex) and 256 edge labels
(Zipf 1.2) stored as uint16, run to the fixpoint capped at k = 64; the graph
comes from the counter-based generator, so the oracle digests of the same
graph pin it.

Prints ONE JSON line (rank 0, N = 1) with the whole-job throughput in
edge-iterations/s (sum over executed iterations of |E|, over the wall time
of the timed steps), the refinement iteration's HBM roofline figures and a
bounded CPU-oracle baseline.  Extra keys: the long k-chaining workload
(rmat22_chains, 2^25 edges plus 64 chains of 2,000 edges, >= 2,001
iterations), the incremental, serving, batched and direction legs.
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, published


def iteration_bytes(n: int, m: int, label_bytes: int) -> int:
    """Algorithmic HBM bytes of one refinement iteration: per edge the target
    id, the label and the gathered neighbour hash; per vertex its offset, its
    type hash, its new hash and one count-table slot (16 B)."""
    return m * (4 + label_bytes + 8) + n * (4 + 8 + 8 + 16)


def read_traffic(workload: str):
    """HBM bytes per working refinement launch (FETCH_SIZE + WRITE_SIZE,
    scaled by a copy kernel's reading) from the committed rocprofv3 counter
    summary profiles/k_iterate_<workload>_counters.json; None if there is
    none or the kernel sources changed after the counters were taken."""
    from paper_2111_12493_amd.profiling import kernel_fingerprint

    path = os.path.join(ROOT, "profiles", "k_iterate_%s_counters.json" % workload)
    if not os.path.exists(path):
        return None
    with open(path) as f:
        d = json.load(f)
    if d.get("kernel_sources_sha256_16") != kernel_fingerprint():
        return None
    return d.get("bytes_per_launch")


def traffic_detail(workload: str):
    """The counted bytes behind read_traffic and the copy-kernel scales that
    turn them into bytes (None where read_traffic is None)."""
    if read_traffic(workload) is None:
        return None
    with open(os.path.join(ROOT, "profiles", "k_iterate_%s_counters.json" % workload)) as f:
        d = json.load(f)
    return {"counted_read_bytes": d.get("counted_fetch_bytes_per_iteration"),
            "counted_write_bytes": d.get("counted_write_bytes_per_iteration"),
            "copy_read_scale": d.get("copy_read_scale"), "copy_write_scale": d.get("copy_write_scale"),
            "l2_hit_rate": d.get("k_iterate_l2_hit_rate"),
            "source": "profiles/k_iterate_%s_counters.json (rocprofv3 TCC counter passes)" % workload}


def host_cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(g, stride: int):
    """The oracle (one thread) on a bounded sample of the headline graph:
    type hashes of all vertices (untimed), then the refinement step h^1 of
    every stride-th vertex (its gathers reach the full h^0 array) and the
    class refinement of those vertices, timed.  Edge-iterations/s = the
    sample's edges over that time."""
    import numpy as np

    from oracle import oracle as orc

    # one core for the oracle; the mask is restored afterwards, since every
    # thread started later (the library's host threads, the server's
    # workers) inherits it
    mask = os.sched_getaffinity(0)
    try:
        os.sched_setaffinity(0, {sorted(mask)[0]})
    except Exception:
        pass
    try:
        t = orc.type_hashes(g)
        count = (g.n + stride - 1) // stride
        deg = np.diff(g.row_off.astype(np.int64))
        edges = int(deg[::stride].sum())
        t0 = time.perf_counter()
        h1 = orc.step_strided(g, t, t, 0, stride, count)
        orc.refine_classes(np.zeros(count, dtype=np.uint32), h1)
        dt = time.perf_counter() - t0
    finally:
        try:
            os.sched_setaffinity(0, mask)
        except Exception:
            pass
    return {"value": edges / dt, "unit": "edge-iterations/s", "cores": 1, "kind": "oracle",
            "host_cpu": host_cpu_model(),
            "sample": "one refinement step (h^1 from h^0, gathers over the whole graph) and the class "
                      "refinement of every %d-th vertex of the headline graph: %d vertices, %d edges, "
                      "single thread, %.1f s" % (stride, count, edges, dt)}


def percentile(v, q):
    v = sorted(v)
    return v[min(len(v) - 1, int(round(q * (len(v) - 1))))]


def serving_leg(args, binding, gg, torch, g, dbase):
    """Serving under Poisson arrivals: update batches for a resident state
    (rmat24, k = 4) and fresh summarize requests (R-MAT, degree 8, device
    resident, to the fixpoint) arrive at equal rates; the arrival rate sweeps
    25/50/75/90 % of the measured capacity of the plain form.  Chosen form:
    the server with 4 workers (continuous batching by footprint, overlapping
    requests) and incremental updates.  Plain form: one worker, first come
    first served, every update recomputed in full (frontier limit 0).  Both
    forms see the same arrival sequence at each rate; latency is submit to
    completion, from the server's own clock."""
    import numpy as np

    from paper_2111_12493_amd import devgen

    rng = np.random.default_rng(29)
    pool = []
    for i in range(args.serve_pool):
        m = int(round(10 ** rng.uniform(4, np.log10(args.serve_max_edges))))
        n = max(2, m // 8)
        pool.append(devgen.rmat_device(int(np.ceil(np.log2(n))), m, n_types=128, n_labels=64, n=n,
                                       seed=int(rng.integers(1, 1 << 30))))
    n_upd = max(args.serve_requests, args.serve_calib)  # each run applies a prefix to a fresh state
    dead = np.zeros(g.n + 4_000_000, dtype=bool)
    n_v = g.n
    scale = int(np.ceil(np.log2(max(g.n, 2))))
    batches = []
    t0 = time.perf_counter()
    for i in range(n_upd):
        d = gg.sample_update_ops(g.row_off, g.tgt, g.lab, n_v, dead, rng,
                                 int(round(10 ** rng.uniform(3, np.log10(args.serve_max_ops)))),
                                 max(g.n_labels, 1), max(g.n_types, 1), rmat_scale=scale)
        n_v = d["n_after"]
        batches.append(binding.UpdateBatch.from_op_arrays(d))
    print("# serving: %d fresh graphs in the pool, %d update batches sampled in %.1f s"
          % (len(pool), len(batches), time.perf_counter() - t0), file=sys.stderr, flush=True)

    def server(plain):
        srv = binding.Server(workers=1 if plain else args.serve_workers)
        if plain:
            srv.set_option("frontier_limit_pct", 0)
        res, state = srv.poll(srv.submit_summarize(dbase, k_max=4, stop_at_fixpoint=False, summary_edges=False,
                                                   keep_state=True))
        res.free()
        return srv, state

    # capacity of the plain form: mean service time over a calibration mix,
    # one request at a time (the first update batches, on a state of its own)
    srv, state = server(plain=True)
    svc = {"summarize": [], "update": []}
    try:
        for i in range(args.serve_calib):
            for kind in ("summarize", "update"):
                t = time.perf_counter()
                tk = srv.submit_summarize(pool[i % len(pool)], summary_edges=False) if kind == "summarize" \
                    else srv.submit_update(state, batches[i])
                r, _ = srv.poll(tk)
                r.free()
                svc[kind].append(time.perf_counter() - t)
        srv.release_state(state)
    finally:
        srv.free()
    mean_svc = (np.mean(svc["summarize"]) + np.mean(svc["update"])) / 2
    capacity = 1.0 / mean_svc
    print("# serving: plain service %.1f ms (summaries) / %.1f ms (updates) -> capacity %.1f requests/s"
          % (1e3 * np.mean(svc["summarize"]), 1e3 * np.mean(svc["update"]), capacity), file=sys.stderr, flush=True)

    points = []
    for frac in args.serve_loads:
        lam = frac * capacity
        arng = np.random.default_rng(int(1000 * frac))
        gaps = arng.exponential(1.0 / lam, size=args.serve_requests)
        kinds = arng.random(args.serve_requests) < 0.5  # True: update
        point = {"load": frac, "rate_per_s": lam, "requests": args.serve_requests}
        blocks = {}
        for form in ("chosen", "plain"):
            srv, state = server(plain=form == "plain")
            try:
                tickets = []
                ui = si = 0
                torch.cuda.synchronize()
                start = time.perf_counter()
                due = start
                for gap, upd in zip(gaps, kinds):
                    due += gap
                    wait = due - time.perf_counter()
                    if wait > 0:
                        time.sleep(wait)
                    if upd:
                        tickets.append(("u", srv.submit_update(state, batches[ui])))
                        ui += 1
                    else:
                        tickets.append(("s", srv.submit_summarize(pool[si % len(pool)], summary_edges=False)))
                        si += 1
                nb = []
                for kind, tk in tickets:
                    r, _ = srv.poll(tk)
                    nb.append(r.n_blocks)
                    r.free()
                st = srv.stats()
                srv.release_state(state)
            finally:
                srv.free()
            blocks[form] = nb
            point[form] = {"p50_ms": st["p50_ms"][0], "p99_ms": st["p99_ms"][0],
                           "summarize_p50_ms": st["p50_ms"][1], "summarize_p99_ms": st["p99_ms"][1],
                           "update_p50_ms": st["p50_ms"][2], "update_p99_ms": st["p99_ms"][2],
                           "requests_per_s": len(tickets) / (st["busy_ms"] / 1e3) if st["busy_ms"] else None}
            print("# serving load %.2f (%.1f req/s) %s: p50 %.1f ms p99 %.1f ms (updates %.1f / %.1f, summaries "
                  "%.1f / %.1f), %.1f req/s" % (frac, lam, form, point[form]["p50_ms"], point[form]["p99_ms"],
                                                point[form]["update_p50_ms"], point[form]["update_p99_ms"],
                                                point[form]["summarize_p50_ms"], point[form]["summarize_p99_ms"],
                                                point[form]["requests_per_s"] or 0), file=sys.stderr, flush=True)
        if blocks["chosen"] != blocks["plain"]:
            raise RuntimeError("serving results differ between the two forms at load %.2f" % frac)
        point["p99_ratio_plain_over_chosen"] = point["plain"]["p99_ms"] / point["chosen"]["p99_ms"]
        points.append(point)
    return {"workload": "%s resident (k=4): Poisson arrivals of update batches (log-uniform 10^3-%.0e ops, "
                        "ADD/MOD/DEL 60/25/15) and fresh R-MAT summaries (log-uniform 10^4-%.0e edges, degree 8, "
                        "to the fixpoint; %d distinct graphs) at equal rates"
                        % (args.inc_workload, args.serve_max_ops, args.serve_max_edges, len(pool)),
            "capacity_requests_per_s": capacity, "plain_service_ms": {k: 1e3 * float(np.mean(v)) for k, v in svc.items()},
            "chosen_form": "%d workers, continuous batching by footprint, incremental updates" % args.serve_workers,
            "plain_form": "one worker, first come first served, every update recomputed in full",
            "points": points}


def incremental_leg(args, binding, gg, torch, g, dg, workload=None, rmat_endpoints=True, k=4):
    """Update-batch latency on a resident graph (levels 0..k): the
    incremental form (frontier re-hash, full levels once a frontier exceeds
    the limit, class index updated for the re-keyed vertices) beside the
    plain form (every level recomputed and its classes rebuilt for all
    vertices) on the same batches, each on its own copy of the state."""
    import numpy as np

    workload = workload or args.inc_workload
    print("# incremental: %s, k=%d, %d vertices, %d edges" % (workload, k, g.n, g.m), file=sys.stderr, flush=True)
    ctx_i, ctx_p = binding.Context(0), binding.Context(0)
    if args.inc_frontier_pct is not None:
        ctx_i.set_option("frontier_limit_pct", args.inc_frontier_pct)
    if args.inc_frontier_edge_pct is not None:
        ctx_i.set_option("frontier_edge_pct", args.inc_frontier_edge_pct)
    ctx_p.set_option("frontier_limit_pct", 0)
    t0 = time.perf_counter()
    st_i = binding.State(ctx_i, dg, k, stop_at_fixpoint=False, summary_edges=False)
    torch.cuda.synchronize()
    create_s = time.perf_counter() - t0
    st_p = binding.State(ctx_p, dg, k, stop_at_fixpoint=False, summary_edges=False)
    st_i.result.free()
    st_p.result.free()
    rng = np.random.default_rng(17)  # the same batches for every k
    dead = np.zeros(g.n + 4_000_000, dtype=bool)
    if g.alive is not None:
        dead[:g.n] = g.alive == 0
    n = g.n
    scale = int(np.ceil(np.log2(max(g.n, 2))))
    lat_i, lat_p, sizes, ops_total = [], [], [], 0
    # one untimed batch on both states first: the first launch of each
    # kernel in the process pays for loading it
    d = gg.sample_update_ops(g.row_off, g.tgt, g.lab, n, dead, np.random.default_rng(16), 1000,
                             max(g.n_labels, 1), max(g.n_types, 1), rmat_scale=scale if rmat_endpoints else None)
    n = d["n_after"]
    warm = binding.UpdateBatch.from_op_arrays(d)
    for st in (st_i, st_p):
        st.apply(warm).free()
    for i in range(args.inc_batches):
        size = int(round(10 ** rng.uniform(3, np.log10(args.inc_max_ops))))
        d = gg.sample_update_ops(g.row_off, g.tgt, g.lab, n, dead, rng, size, max(g.n_labels, 1),
                                 max(g.n_types, 1), rmat_scale=scale if rmat_endpoints else None)
        n = d["n_after"]
        batch = binding.UpdateBatch.from_op_arrays(d)
        nb, ph = {}, {}
        # the forms take turns going first: the second run of a batch finds
        # its operation arrays in the host caches
        forms = ((st_i, lat_i), (st_p, lat_p)) if i % 2 == 0 else ((st_p, lat_p), (st_i, lat_i))
        for st, lat in forms:
            torch.cuda.synchronize()
            t = time.perf_counter()
            r = st.apply(batch)
            lat.append((time.perf_counter() - t) * 1e3)
            nb[id(st)] = r.n_blocks
            ph[id(st)] = (r.ms_resolve, r.ms_stage, r.ms_iterate, r.ms_finalize)
            r.free()
        if nb[id(st_i)] != nb[id(st_p)]:
            raise RuntimeError("incremental and full recomputation disagree on batch %d" % i)
        ops_total += size
        sizes.append(size)
        print("# update batch %d (k=%d): %d ops, incremental %.2f ms, full recomputation %.2f ms "
              "(host op resolution, then device merge/levels/finalize: %.1f, %.1f/%.1f/%.1f and %.1f, %.1f/%.1f/%.1f ms)"
              % ((i, k, size, lat_i[-1], lat_p[-1]) + ph[id(st_i)] + ph[id(st_p)]), file=sys.stderr, flush=True)

    # change detection: the ordered batch between the first snapshot and
    # the state's graph after all batches, from the two device CSRs
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    n_diff = binding.diff_snapshots(ctx_i, dg, st_i.device_graph(), as_tuples=False)
    torch.cuda.synchronize()
    diff_ms = (time.perf_counter() - t0) * 1e3
    print("# snapshot diff: %d ops in %.1f ms" % (n_diff, diff_ms), file=sys.stderr, flush=True)
    st_i.free()
    st_p.free()
    ctx_i.close()
    ctx_p.close()
    p50, p99 = percentile(lat_i, 0.5), percentile(lat_i, 0.99)
    q50, q99 = percentile(lat_p, 0.5), percentile(lat_p, 0.99)
    # the same measurements, split at 10^4 operations per batch
    small = [i for i, z in enumerate(sizes) if z < 10000]
    by_size = {"batches_below_1e4_ops": len(small)}
    if small:
        by_size["p50_ms"] = percentile([lat_i[i] for i in small], 0.5)
        by_size["plain_p50_ms"] = percentile([lat_p[i] for i in small], 0.5)
    return {"workload": "%s resident, k=%d, update batches of log-uniform 10^3-%.0e ops (ADD/MOD/DEL 60/25/15, "
                        "%s endpoints for new edges)" % (workload, k, args.inc_max_ops,
                                                         "R-MAT" if rmat_endpoints else "uniform"),
            "k": k,
            "batches": len(lat_i), "ops": ops_total, "p50_ms": p50, "p99_ms": p99,
            "plain_p50_ms": q50, "plain_p99_ms": q99, "speedup_p50": q50 / p50, "speedup_p99": q99 / p99,
            "small_batches": by_size, "state_create_s": create_s, "summary_edges": False,
            "per_batch_ops_incremental_plain_ms": [[z, round(a, 3), round(b, 3)]
                                                   for z, a, b in zip(sizes, lat_i, lat_p)],
            "order": "the two forms alternate which runs a batch first",
            "snapshot_diff": {"ops": n_diff, "ms": diff_ms,
                              "what": "bsim_diff_snapshots between the first snapshot and the graph after "
                                      "all batches"},
            "plain_form": "same update batch, every level recomputed for all vertices"}


def directions_leg(binding, torch, ctx, dg, g):
    """The direction and label parameterizations (Sec. 2.4) on the headline
    graph, each to its fixpoint after one untimed run: backward (incoming
    edges), both directions, and forward over the even labels.  The rate
    counts the edges each signature reads (2|E| for both directions)."""
    import numpy as np

    even = list(range(0, max(int(g.n_labels), 1), 2))
    kept = int(np.isin(g.lab, np.asarray(even, dtype=g.lab.dtype)).sum())
    out = {}
    for name, kw, edges in (("backward", dict(direction="in"), g.m), ("both", dict(direction="both"), 2 * g.m),
                            ("even_labels", dict(labels=even), kept)):
        binding.summarize(ctx, dg, k_max=binding.K_UNBOUNDED, **kw).free()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = binding.summarize(ctx, dg, k_max=binding.K_UNBOUNDED, **kw)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        out[name] = {"k_done": r.k_done, "blocks": r.n_blocks, "edges_read": edges, "s": wall,
                     "edge_iterations_per_s": r.k_done * edges / wall,
                     "ms_stage": r.ms_stage, "ms_iterate": r.ms_iterate}
        r.free()
        print("# %s: k_done=%d blocks=%d %.3f s" % (name, out[name]["k_done"], out[name]["blocks"], wall),
              file=sys.stderr, flush=True)
    return out


def batched_leg(args, binding, gg, torch):
    """One batched run over many R-MAT graphs against one call per graph.
    The batched call's schedule (small graphs in the persistent launch or
    not, hub-table size) is the autotuner's, picked during the warm-up call
    and cached for the size class."""
    from paper_2111_12493_amd import devgen

    graphs = devgen.batched_device(args.batch_graphs, args.batch_max_edges, seed=23)
    dgs = graphs
    ctx = binding.Context(0)
    edges = sum(g.m for g in graphs)
    print("# batched: %d graphs, %d edges" % (len(graphs), edges), file=sys.stderr, flush=True)
    t = time.perf_counter()
    rs = binding.batch_summarize(ctx, dgs, summary_edges=True)  # warm-up; the autotuner's first call
    torch.cuda.synchronize()
    tune_s = time.perf_counter() - t
    for r in rs:
        r.free()
    picked = {"small_graph_edges": ctx.get_option("batch_small_edges"),
              "hub_table_slots": ctx.get_option("batch_hub_table_slots")}
    torch.cuda.synchronize()
    t = time.perf_counter()
    rs = binding.batch_summarize(ctx, dgs, summary_edges=True)
    torch.cuda.synchronize()
    tb = time.perf_counter() - t
    work = sum(r.k_done * g.m for r, g in zip(rs, graphs))
    # algorithmic bytes of the refinement levels each graph ran, over the
    # call's refinement phase (device events)
    algo = sum(r.k_done * iteration_bytes(g.n, g.m, 4) for r, g in zip(rs, graphs))
    ms_iter = rs[0].ms_iterate
    kmax = max(r.k_done for r in rs)
    phases = {"stage_ms": rs[0].ms_stage, "iterate_ms": ms_iter, "finalize_ms": rs[0].ms_finalize}
    for r in rs:
        r.free()
    torch.cuda.synchronize()
    t = time.perf_counter()
    for dg in dgs:
        binding.summarize(ctx, dg).free()
    torch.cuda.synchronize()
    tp = time.perf_counter() - t
    ctx.close()
    achieved = algo / (ms_iter * 1e-3) / 1e9 if ms_iter else 0.0
    # the same batch plus small graphs with deep fixpoints (chains of 200
    # edges): in the union they keep every launch going; the persistent
    # small-graph launch finishes them in LDS.  Tuned schedule against the
    # union-only one.
    chains = [binding.DeviceGraph(gg.chain(200)) for _ in range(args.batch_chains)]
    deep = {}
    for name, opt in (("tuned", None), ("union_only", 0)):
        c = binding.Context(0)
        if opt is not None:
            c.set_option("batch_small_edges", opt)
        for r in binding.batch_summarize(c, dgs + chains, summary_edges=True):  # warm-up (tuning)
            r.free()
        torch.cuda.synchronize()
        t = time.perf_counter()
        rs = binding.batch_summarize(c, dgs + chains, summary_edges=True)
        torch.cuda.synchronize()
        deep[name] = {"s": time.perf_counter() - t, "max_k_done": max(r.k_done for r in rs),
                      "small_graph_edges": c.get_option("batch_small_edges")}
        for r in rs:
            r.free()
        c.close()
    deep["speedup"] = deep["union_only"]["s"] / deep["tuned"]["s"]
    print("# batched + %d chains: tuned %.3f s, union only %.3f s" % (args.batch_chains, deep["tuned"]["s"],
                                                                      deep["union_only"]["s"]),
          file=sys.stderr, flush=True)
    return {"workload": "%d R-MAT graphs, edges log-uniform 10^2-%.0e, degree U(4,16), 32 types / 32 labels "
                        "(Zipf 1.0), each to its own fixpoint" % (len(graphs), args.batch_max_edges),
            "graphs": len(graphs), "edges": edges, "max_k_done": kmax, "edge_iterations": work,
            "batched_s": tb, "per_graph_s": tp, "value_batched": work / tb, "value_per_graph": work / tp,
            "speedup": tp / tb, "schedule": picked, "autotune_first_call_s": tune_s, "phases": phases,
            "with_deep_small_graphs": dict(deep, what="the same graphs plus %d chains of 200 edges"
                                                        % args.batch_chains),
            "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": achieved / HBM_PEAK_GBS, "algorithmic_bytes": algo,
                         "what": "refinement levels of every graph (its own k_done) over the batched call's "
                                 "refinement phase"}}


WORKLOADS = {
    # name: iteration cap of the workload's runs (None = to the fixpoint)
    "rmat27": 64,
    "rmat22_chains": None,
    "uniform_10k_50k": 10,
}


def timed_summaries(binding, torch, ctx, dg, k_max, steps, warmup, tag):
    """`warmup` untimed and `steps` timed summarizations (to the fixpoint,
    capped at k_max); per-step records and the timed wall time."""

    def step():
        r = binding.summarize(ctx, dg, k_max=k_max, stop_at_fixpoint=True)
        rec = dict(k_done=r.k_done, launches=r.n_iter_launches, ms_kernels=r.ms_iter_kernels,
                   ms_hub=r.ms_hub_kernels, timed=r.n_timed_launches,
                   ms_iterate=r.ms_iterate, ms_stage=r.ms_stage, ms_finalize=r.ms_finalize,
                   ms_total=r.ms_total, n_blocks=r.n_blocks, n_se=r.n_summary_edges)
        r.free()
        return rec

    for i in range(warmup):
        rec = step()
        print("# %s warmup %d: k_done=%d blocks=%d %.1f ms" % (tag, i, rec["k_done"], rec["n_blocks"],
                                                               rec["ms_total"]), file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    recs = []
    t0 = time.perf_counter()
    for i in range(steps):
        recs.append(step())
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    for i, r in enumerate(recs):
        print("# %s step %d: k_done=%d launches=%d stage %.2f ms, iterate %.2f ms (kernels %.2f + hubs %.2f over "
              "%d timed launches), finalize %.2f ms" % (tag, i, r["k_done"], r["launches"], r["ms_stage"],
                                                         r["ms_iterate"], r["ms_kernels"], r["ms_hub"], r["timed"],
                                                         r["ms_finalize"]), file=sys.stderr, flush=True)
    return recs, wall


def roofline(recs, g, workload):
    """HBM roofline of the refinement iteration (the refinement launch plus
    the hub-bucket and hub-finish launches of the same iteration), from the
    HIP events the library records on its own stream around the working
    launches (1..k_done+1 of a run; the rest of the last queued chunk return
    at once and are not timed)."""
    label_bytes = 2 if g.lab.dtype.itemsize == 2 else 4
    b_iter = iteration_bytes(g.n, g.m, label_bytes)
    kern_ms = sum(r["ms_kernels"] for r in recs)
    hub_ms = sum(r["ms_hub"] for r in recs)
    timed = sum(r["timed"] for r in recs)
    iter_us = (kern_ms + hub_ms) * 1e3 / max(timed, 1)
    achieved = b_iter / (iter_us * 1e-6) / 1e9 if timed else 0.0
    return {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "traffic": read_traffic(workload),
            "traffic_detail": traffic_detail(workload),
            "kernel": "k_iterate + k_hub + k_hub_finish (one refinement iteration)",
            "algorithmic_bytes_per_launch": b_iter, "avg_launch_us": iter_us,
            "k_iterate_avg_us": kern_ms * 1e3 / max(timed, 1), "hub_kernels_avg_us": hub_ms * 1e3 / max(timed, 1),
            "timed_launches": timed,
            "launches_issued": sum(r["launches"] for r in recs)}


def chaining_leg(args, binding, torch):
    """The long k-chaining workload (rmat22_chains: R-MAT scale 22, 2^25 edges,
    plus 64 chains of 2,000 edges; >= 2,001 iterations to the fixpoint)."""
    from paper_2111_12493_amd import graphgen as gg

    g = gg.make_config("rmat22_chains")
    dg = binding.DeviceGraph(g)
    ctx = binding.Context(0)
    ctx.set_option("time_launches", 16)  # events on every launch would add gaps
    recs, wall = timed_summaries(binding, torch, ctx, dg, binding.K_UNBOUNDED, args.chain_steps, 1, "rmat22_chains")
    out = {"workload": "rmat22_chains", "vertices": g.n, "edges": g.m, "k_done": recs[-1]["k_done"],
           "blocks": recs[-1]["n_blocks"], "steps": len(recs), "ms_per_step": wall * 1e3 / len(recs),
           "edge_iterations_per_s": sum(r["k_done"] for r in recs) * g.m / wall,
           "roofline": roofline(recs, g, "rmat22_chains")}
    if not args.no_directions:
        out["directions"] = directions_leg(binding, torch, ctx, dg, g)
    ctx.close()
    return out


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="rmat27", choices=sorted(WORKLOADS))
    ap.add_argument("--cpu-stride", type=int, default=16,
                    help="CPU baseline: the oracle's step on every N-th vertex of the headline graph")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--time-every", type=int, default=1,
                    help="bracket every N-th refinement launch of the headline runs with HIP events")
    ap.add_argument("--no-chaining", action="store_true")
    ap.add_argument("--chain-steps", type=int, default=3)
    ap.add_argument("--no-incremental", action="store_true")
    ap.add_argument("--inc-workload", default="rmat24")
    ap.add_argument("--inc-batches", type=int, default=16)
    ap.add_argument("--inc-uniform", default="uniform24",
                    help="second incremental workload (a uniform graph); empty to skip")
    ap.add_argument("--inc-max-ops", type=float, default=1e6)
    ap.add_argument("--inc-frontier-pct", type=int, default=None,
                    help="frontier limit of the incremental form (the library's default if not given)")
    ap.add_argument("--inc-frontier-edge-pct", type=int, default=None,
                    help="frontier edge limit of the incremental form (the library's default if not given)")
    ap.add_argument("--inc-k", type=int, nargs="+", default=[4, 2, 1],
                    help="levels of the resident states (the first is the main line's)")
    ap.add_argument("--no-serving", action="store_true")
    ap.add_argument("--serve-requests", type=int, default=100, help="requests per arrival rate")
    ap.add_argument("--serve-loads", type=float, nargs="+", default=[0.25, 0.5, 0.75, 0.9])
    ap.add_argument("--serve-calib", type=int, default=8, help="calibration requests of each kind")
    ap.add_argument("--serve-pool", type=int, default=24, help="distinct fresh graphs")
    ap.add_argument("--serve-workers", type=int, default=4)
    ap.add_argument("--serve-max-ops", type=float, default=1e5)
    ap.add_argument("--serve-max-edges", type=float, default=1e7)
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--no-directions", action="store_true")
    ap.add_argument("--batch-graphs", type=int, default=4096)
    ap.add_argument("--batch-max-edges", type=float, default=1e6)
    ap.add_argument("--batch-chains", type=int, default=64)
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="first run one elementwise copy kernel over this many MiB, so that a "
                         "rocprofv3 counter run can scale FETCH_SIZE/WRITE_SIZE")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU: the library has no multi-GPU path; run with --gpus 1",
              file=sys.stderr)
        return 2

    import torch

    from paper_2111_12493_amd import binding
    from paper_2111_12493_amd import graphgen as gg

    torch.cuda.set_device(0)
    t_gen = time.perf_counter()
    g = gg.make_config(args.workload)
    gen_s = time.perf_counter() - t_gen
    print("# workload %s: %d vertices, %d edges (generated on the host in %.1f s)"
          % (args.workload, g.n, g.m, gen_s), file=sys.stderr, flush=True)
    if args.calibrate_copy:
        nbytes = args.calibrate_copy << 20
        src = torch.empty(nbytes, dtype=torch.uint8, device="cuda").fill_(1)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        torch.bitwise_not(src, out=dst)  # one elementwise kernel: reads and writes nbytes
        torch.cuda.synchronize()
        print("# calibration kernel: %d bytes read, %d bytes written" % (nbytes, nbytes),
              file=sys.stderr, flush=True)
        del src, dst
    dg = binding.DeviceGraph(g)
    ctx = binding.Context(0)
    ctx.set_option("time_launches", args.time_every)
    torch.cuda.synchronize()
    k_cap = WORKLOADS[args.workload]
    recs, wall = timed_summaries(binding, torch, ctx, dg, binding.K_UNBOUNDED if k_cap is None else k_cap,
                                 args.steps, args.warmup, args.workload)
    edge_iters = sum(r["k_done"] for r in recs) * g.m
    iter_ms = sum(r["ms_iterate"] for r in recs)
    out = {
        "metric": "edge-iterations/s for k-bisimulation (% HBM roofline); p50/p99 update latency",
        "value": edge_iters / wall,
        "unit": "edge-iterations/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": wall * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u64",
        "data": "synthetic",
        "config": {"workload": args.workload, "vertices": g.n, "edges": g.m,
                   "k_cap": k_cap, "k_done": recs[-1]["k_done"], "fixpoint": None,
                   "blocks": recs[-1]["n_blocks"], "summary_edges": recs[-1]["n_se"],
                   "label_bytes": int(g.lab.dtype.itemsize), "parallelism": "single GPU"},
        "roofline": roofline(recs, g, args.workload),
        # the same steps split by phase (device events of each call)
        "phases_ms_per_step": {"stage": sum(r["ms_stage"] for r in recs) / len(recs),
                               "iterate": iter_ms / len(recs),
                               "finalize": sum(r["ms_finalize"] for r in recs) / len(recs)},
        "iteration_loop_edge_iterations_per_s": edge_iters / (iter_ms * 1e-3) if iter_ms else None,
        "host_generation_s": gen_s,
    }
    r = binding.summarize(ctx, dg, k_max=binding.K_UNBOUNDED if k_cap is None else k_cap, stop_at_fixpoint=True,
                          summary_edges=False)
    out["config"]["fixpoint"] = int(r.fixpoint)
    r.free()
    ctx.close()
    del dg
    torch.cuda.empty_cache()
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(g, args.cpu_stride)
        print("# cpu baseline: %.3g edge-iterations/s" % out["cpu_baseline"]["value"], file=sys.stderr, flush=True)
    del g
    if not args.no_chaining:
        out["long_chaining"] = chaining_leg(args, binding, torch)
    torch.cuda.empty_cache()
    if not (args.no_incremental and args.no_serving):
        from paper_2111_12493_amd import devgen

        # the resident graph is drawn on the GPU; the update sampler reads a host copy
        if args.inc_workload in devgen.DEVICE_CONFIGS:
            dg24 = devgen.make_device_config(args.inc_workload)
            g24 = dg24.to_host()
        else:
            g24 = gg.make_config(args.inc_workload)
            dg24 = binding.DeviceGraph(g24)
        if not args.no_incremental:
            for i, k in enumerate(args.inc_k):
                key = "incremental" if i == 0 else "incremental_k%d" % k
                out[key] = incremental_leg(args, binding, gg, torch, g24, dg24, k=k)
        if not args.no_serving:
            out["serving"] = serving_leg(args, binding, gg, torch, g24, dg24)
        del g24, dg24
    if not args.no_incremental and args.inc_uniform:
        from paper_2111_12493_amd import devgen

        # the same batches on a graph without hubs, where a change stays local
        dgu = devgen.make_device_config(args.inc_uniform)
        gu = dgu.to_host()
        for i, k in enumerate(args.inc_k):
            key = "incremental_uniform" if i == 0 else "incremental_uniform_k%d" % k
            out[key] = incremental_leg(args, binding, gg, torch, gu, dgu, workload=args.inc_uniform,
                                       rmat_endpoints=False, k=k)
        del gu, dgu
    if not args.no_batched:
        out["batched"] = batched_leg(args, binding, gg, torch)
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
