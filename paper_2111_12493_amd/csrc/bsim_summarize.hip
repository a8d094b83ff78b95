// bsim_summarize.hip -- host driver of one batch summarization.
//
// Device round trips per call: one after staging (tile and hub counts), one
// per queued chunk of refinement launches (the sticky done flag, read while
// the next chunk is already queued), two in finalize (block and edge
// counts).  Refinement launches are queued in chunks that double up to
// ctx->chunk_max, so a run of thousands of iterations (long k-chaining)
// costs only the kernels themselves plus a few early-exit launches.
#include <algorithm>
#include <functional>
#include <cstdlib>
#include <cstring>

#include "bsim_api_internal.h"

namespace bsim {

void validate_params(const bsim_graph& graph, const bsim_params& p, bool directions) {
    if (graph.label_bytes != 2 && graph.label_bytes != 4)
        throw DeviceError{BSIM_E_INVALID, "label_bytes must be 2 or 4"};
    if (graph.mem_kind != BSIM_MEM_HOST && graph.mem_kind != BSIM_MEM_DEVICE)
        throw DeviceError{BSIM_E_INVALID, "unknown mem_kind"};
    if (graph.n_edges >= (1ull << 32))
        throw DeviceError{BSIM_E_UNSUPPORTED, "this library supports fewer than 2^32 edges"};
    if (graph.n_vertices >= 0xFFFFFFFFu)
        throw DeviceError{BSIM_E_UNSUPPORTED, "too many vertices"};
    if (!graph.row_off || !graph.type_off)
        throw DeviceError{BSIM_E_INVALID, "row_off and type_off are required"};
    if (graph.n_edges && (!graph.targets || !graph.labels))
        throw DeviceError{BSIM_E_INVALID, "targets and labels are required"};
    if (!(p.flags & BSIM_STOP_AT_FIXPOINT) && p.k_max > (1u << 24))
        throw DeviceError{BSIM_E_INVALID, "without a fixpoint test k_max must be finite (< 2^24)"};
    if (p.flags & ~(BSIM_STOP_AT_FIXPOINT | BSIM_KEEP_LEVELS | BSIM_UNTYPED | BSIM_RESULT_ON_HOST |
                    BSIM_NO_SUMMARY_EDGES | BSIM_BACKWARD | BSIM_BOTH_DIRECTIONS | BSIM_PREV_LEVEL_EDGES))
        throw DeviceError{BSIM_E_INVALID, "unknown flag bits"};
    if ((p.flags & BSIM_BACKWARD) && (p.flags & BSIM_BOTH_DIRECTIONS))
        throw DeviceError{BSIM_E_INVALID, "BSIM_BACKWARD and BSIM_BOTH_DIRECTIONS exclude each other"};
    if ((p.flags & BSIM_PREV_LEVEL_EDGES) && (p.flags & (BSIM_BACKWARD | BSIM_BOTH_DIRECTIONS)))
        throw DeviceError{BSIM_E_INVALID, "BSIM_PREV_LEVEL_EDGES is defined for the forward direction only"};
    if (!directions && (p.flags & (BSIM_BACKWARD | BSIM_BOTH_DIRECTIONS)))
        throw DeviceError{BSIM_E_UNSUPPORTED, "edge directions other than outgoing are supported by "
                                              "bsim_summarize without a state only"};
}

void upload_graph(const bsim_graph& in, Staged& g, Arena& arena, hipStream_t s) {
    g.n = in.n_vertices;
    g.m = in.n_edges;
    g.label_bytes = in.label_bytes;
    if (in.mem_kind == BSIM_MEM_DEVICE) {
        g.row_off = in.row_off;
        g.tgt = in.targets;
        g.lab = in.labels;
        g.type_off = in.type_off;
        g.type_ids = in.type_ids;
        g.alive = in.alive;
        return;
    }
    const size_t n = in.n_vertices, m = in.n_edges;
    uint32_t* ro = arena.alloc<uint32_t>(n + 1);
    hip_check(hipMemcpyAsync(ro, in.row_off, (n + 1) * 4, hipMemcpyHostToDevice, s), "upload row_off");
    uint32_t* to = arena.alloc<uint32_t>(n + 1);
    hip_check(hipMemcpyAsync(to, in.type_off, (n + 1) * 4, hipMemcpyHostToDevice, s), "upload type_off");
    // type_off[n] tells how many type ids follow; read it from the host copy
    const size_t nt = in.type_off[n];
    uint32_t* ti = arena.alloc<uint32_t>(nt + 1);
    if (nt) hip_check(hipMemcpyAsync(ti, in.type_ids, nt * 4, hipMemcpyHostToDevice, s), "upload types");
    uint32_t* tg = arena.alloc<uint32_t>(m + 1);
    void* lb = arena.alloc<uint8_t>(m * in.label_bytes + 4);
    if (m) {
        hip_check(hipMemcpyAsync(tg, in.targets, m * 4, hipMemcpyHostToDevice, s), "upload targets");
        hip_check(hipMemcpyAsync(lb, in.labels, m * in.label_bytes, hipMemcpyHostToDevice, s), "upload labels");
    }
    uint8_t* al = nullptr;
    if (in.alive) {
        al = arena.alloc<uint8_t>(n + 1);
        hip_check(hipMemcpyAsync(al, in.alive, n, hipMemcpyHostToDevice, s), "upload alive");
    }
    g.row_off = ro;
    g.type_off = to;
    g.type_ids = ti;
    g.tgt = tg;
    g.lab = lb;
    g.alive = al;
}

LoopResult run_refinement(bsim_ctx* ctx, const Staged& g, const bsim_params& p, RunBuffers& rb,
                          LevelSink* sink, Arena& arena, uint32_t* rep_prev, bool use_timers) {
    hipStream_t s = ctx->stream;
    const bool stop = (p.flags & BSIM_STOP_AT_FIXPOINT) != 0;
    const bool untyped = (p.flags & BSIM_UNTYPED) != 0;
    if (sink && !sink->levels.empty()) rb.h[0] = sink->levels[0];
    launch_init(g, rb, untyped, s);
    if (rb.bc.gid && rb.small.n_small) {
        // the small graphs of a batch go to their stop levels now, each in one
        // workgroup; their per-level counts need history rows up to there
        // (with the fixpoint test a graph of n vertices stops by level max(n, 1))
        const uint64_t depth =
            stop ? std::min<uint64_t>(p.k_max, static_cast<uint64_t>(rb.small.max_n) + 1) : p.k_max;
        const uint64_t need = depth + 2;
        if (need > rb.bc.hist_cap) {
            const size_t G = rb.bc.n_graphs;
            uint32_t* nh = arena.alloc<uint32_t>(need * G);
            hip_check(hipMemsetAsync(nh, 0, need * G * 4, s), "history clear");
            hip_check(hipMemcpyAsync(nh, rb.bc.hist, static_cast<size_t>(rb.bc.hist_cap) * G * 4,
                                     hipMemcpyDeviceToDevice, s), "history copy");
            rb.bc.hist = nh;
            rb.bc.hist_cap = static_cast<uint32_t>(need);
        }
        launch_small_graphs(g, rb, rb.small, p.k_max, stop, s);
    }

    LoopResult lr;
    // launch k tests level k-2, so launch k_max + 2 always sees the cap
    const uint64_t k_last = static_cast<uint64_t>(p.k_max) + 2;
    uint64_t k = 1;
    // Launches queued per stop-flag check.  The host waits for the previous
    // chunk's status while the current one runs, so a chunk only has to
    // outlast that round trip; every launch queued past the stop is wasted
    // (an early-exit launch still dispatches its whole grid).  So the chunk
    // is capped at about 4 ms of estimated work (a refinement launch streams
    // roughly 40,000 edges per microsecond): one launch at a time for a graph
    // of 2^30 edges, chunks doubling up to chunk_max for small graphs and
    // long k-chaining.  A batched run covers many small graphs that stop
    // within a few levels, and its launches are large: it starts shorter.
    const double est_us = (static_cast<double>(g.m) + g.n) / 40000.0 + 10.0;
    const uint32_t chunk_cap =
        static_cast<uint32_t>(std::max(1.0, std::min<double>(ctx->chunk_max, 4000.0 / est_us)));
    uint32_t chunk = std::min<uint32_t>(rb.bc.gid ? 2u : 4u, chunk_cap);
    int pending = -1;
    hipEvent_t* ev = ctx->loop_ev;  // created with the ctx
    bool done = false;
    bool prev_taken = false;
    std::vector<hipEvent_t> timers;  // (start, after refinement, after hubs) per timed launch
    std::vector<uint32_t> timed_k;   // the launches timed
    std::vector<uint8_t> timed_split;  // ... and whether each ran as a split launch
    struct TimerGuard {
        std::vector<hipEvent_t>& t;
        ~TimerGuard() {
            for (hipEvent_t e : t) (void)hipEventDestroy(e);
        }
    } timer_guard{timers};
    // Queue refinement launch kk: fused, or as its split half then its hash
    // half.  ends_run, if given, runs between the halves and says whether the
    // split half ended the run; the hash half then only records the stop.
    auto issue = [&](uint32_t kk, bool split_first, const std::function<bool()>& ends_run) {
        if (sink && !sink->levels.empty()) {
            // keep every level: iteration kk reads levels[kk-1], writes levels[kk]
            const uint32_t top = static_cast<uint32_t>(sink->levels.size()) - 1;
            rb.h[(kk - 1) & 1] = sink->levels[std::min(kk - 1, top)];
            rb.h[kk & 1] = sink->levels[std::min(kk, top)];
        }
        hipEvent_t et[3] = {nullptr, nullptr, nullptr};
        const bool timed = use_timers && ctx->time_launches && kk % ctx->time_launches == 0;
        if (timed) {
            timed_k.push_back(kk);
            timed_split.push_back(split_first ? 1 : 0);
            for (hipEvent_t& e : et) {
                hip_check(hipEventCreate(&e), "event");
                timers.push_back(e);
            }
            hip_check(hipEventRecord(et[0], s), "event");
        }
        const bool all = sink && !sink->levels.empty();
        if (rb.bc.gid) launch_graph_stop(rb, kk, p.k_max, stop, s);
        bool stop_only = false;
        if (split_first) {
            launch_iteration(g, rb, kk, p.k_max, stop, all, s, kPhaseSplit);
            stop_only = ends_run && ends_run();
            launch_iteration(g, rb, kk, p.k_max, stop, all, s, kPhaseHash, stop_only);
        } else {
            launch_iteration(g, rb, kk, p.k_max, stop, all, s);
        }
        if (rep_prev && kk == p.k_max && g.n) {
            // launch k splits level k-1 and nothing after it in the launch
            // changes the classes: rep now names the (k_max-1)-classes, or
            // the final ones of a run that stopped earlier at a fixpoint
            hip_check(hipMemcpyAsync(rep_prev, rb.rep, static_cast<size_t>(g.n) * 4, hipMemcpyDeviceToDevice, s),
                      "previous classes");
            prev_taken = true;
        }
        if (timed) hip_check(hipEventRecord(et[1], s), "event");
        if (kk <= p.k_max && !stop_only) launch_hubs(g, rb, kk, s);
        if (timed) hip_check(hipEventRecord(et[2], s), "event");
        lr.launches++;
        if (split_first) lr.split_launches++;
    };
    // One launch per stop check (launches of milliseconds, or chunk_max 1):
    // the host waits for every launch anyway, so it reads the founded count
    // of the level the launch split.  A level that founds few classes is
    // often the last to change; the next launch then runs its split half
    // first and hashes only if the run goes on, instead of hashing a level
    // that the fixpoint test discards (at most kMaxSplitLaunches per run).
    constexpr uint32_t kMaxSplitLaunches = 8;
    const bool one_by_one = !rb.bc.gid && stop && ctx->tail_split_ppm && (chunk_cap == 1 || ctx->chunk_max == 1);
    try {
        if (one_by_one) {
            bool split_first = false;
            for (uint64_t kq = 1; kq <= k_last && !done; kq++) {
                const uint32_t kk = static_cast<uint32_t>(kq);
                // the stop test of the hash half (level kk-1) from the split
                // half's founded count: a fixpoint or the level cap
                bool predicted = false;
                const std::function<bool()> ends_run = [&]() {
                    hip_check(hipMemcpyAsync(ctx->count_host, rb.lcnt + ((kk - 1) & (kStripeRing - 1)) * kStripes,
                                             kStripes * sizeof(uint32_t), hipMemcpyDeviceToHost, s), "count copy");
                    hip_check(hipStreamSynchronize(s), "split wait");
                    uint64_t c = 0;
                    for (int i = 0; i < kStripes; i++) c += ctx->count_host[i];
                    const uint32_t lv = kk - 1;
                    predicted = (lv >= 1 && c == 0) || lv >= p.k_max;
                    return predicted;
                };
                issue(kk, split_first, ends_run);
                hip_check(hipMemcpyAsync(&ctx->status_host[0], rb.status, sizeof(RunStatus), hipMemcpyDeviceToHost,
                                         s), "status copy");
                // launch kk completed the split of level kk-1 (k_init: level 0)
                hip_check(hipMemcpyAsync(ctx->count_host, rb.lcnt + ((kk - 1) & (kStripeRing - 1)) * kStripes,
                                         kStripes * sizeof(uint32_t), hipMemcpyDeviceToHost, s), "count copy");
                hip_check(hipStreamSynchronize(s), "status wait");
                done = ctx->status_host[0].done != 0;
                if (predicted && !done)
                    throw DeviceError{BSIM_E_DEVICE, "internal: a stop-only launch found the run going on"};
                uint64_t founded = 0;
                for (int i = 0; i < kStripes; i++) founded += ctx->count_host[i];
                split_first = lr.split_launches < kMaxSplitLaunches &&
                              founded * 1000000ull <= static_cast<uint64_t>(ctx->tail_split_ppm) * g.n;
            }
            if (!done) throw DeviceError{BSIM_E_DEVICE, "refinement did not reach its stop test"};
        }
        while (!done) {
            if (k <= k_last) {
                const uint32_t c = static_cast<uint32_t>(std::min<uint64_t>(chunk, k_last - k + 1));
                if (rb.bc.gid && k + c > rb.bc.hist_cap) {
                    // launch kk writes level kk-1 of the per-graph history: grow it
                    // while no launch is in flight
                    hip_check(hipStreamSynchronize(s), "history sync");
                    const uint64_t cap = std::max<uint64_t>(2ull * rb.bc.hist_cap, k + c + 1);
                    const size_t G = rb.bc.n_graphs;
                    uint32_t* nh = arena.alloc<uint32_t>(cap * G);
                    hip_check(hipMemsetAsync(nh, 0, cap * G * 4, s), "history clear");
                    hip_check(hipMemcpyAsync(nh, rb.bc.hist, static_cast<size_t>(rb.bc.hist_cap) * G * 4,
                                             hipMemcpyDeviceToDevice, s), "history copy");
                    rb.bc.hist = nh;
                    rb.bc.hist_cap = static_cast<uint32_t>(cap);
                }
                for (uint32_t i = 0; i < c; i++, k++) issue(static_cast<uint32_t>(k), false, nullptr);
                const int slot = pending < 0 ? 0 : (pending ^ 1);
                hip_check(hipMemcpyAsync(&ctx->status_host[slot], rb.status, sizeof(RunStatus),
                                         hipMemcpyDeviceToHost, s), "status copy");
                hip_check(hipEventRecord(ev[slot], s), "status event");
                if (pending >= 0) {
                    hip_check(hipEventSynchronize(ev[pending]), "status wait");
                    done = ctx->status_host[pending].done != 0;
                }
                pending = slot;
                chunk = std::min<uint32_t>(chunk * 2, chunk_cap);
            } else {
                hip_check(hipEventSynchronize(ev[pending]), "status wait");
                done = ctx->status_host[pending].done != 0;
                if (!done) throw DeviceError{BSIM_E_DEVICE, "refinement did not reach its stop test"};
            }
        }
    } catch (...) {
        (void)hipStreamSynchronize(s);
        throw;
    }
    hip_check(hipStreamSynchronize(s), "loop sync");
    RunStatus st;
    hip_check(hipMemcpy(&st, rb.status, sizeof(RunStatus), hipMemcpyDeviceToHost), "final status");
    // launch j (1-based) hashed iff j <= k_done + 1: launch k_done + 2 finds
    // the stop at level k_done and returns at once, as do all later ones; a
    // split launch k_done + 1 finds it in its hash half and hashes nothing
    for (size_t i = 0; i + 2 < timers.size(); i += 3) {
        if (timed_k[i / 3] > st.k_done + 1) break;
        if (timed_k[i / 3] == st.k_done + 1 && timed_split[i / 3]) break;
        float a = 0.f, b = 0.f;
        hip_check(hipEventElapsedTime(&a, timers[i], timers[i + 1]), "launch timer");
        hip_check(hipEventElapsedTime(&b, timers[i + 1], timers[i + 2]), "launch timer");
        lr.ms_kernels += a;
        lr.ms_hub_kernels += b;
        lr.n_timed++;
    }
    if (st.error & kErrHubSplit)
        throw DeviceError{BSIM_E_DEVICE, "a hub hash bucket could not be split to fit its table"};
    // k_max = 0, or a run whose stop was seen before launch k_max: the final
    // classes (level 0, or a fixpoint's)
    if (rep_prev && !prev_taken && g.n)
        hip_check(hipMemcpyAsync(rep_prev, rb.rep, static_cast<size_t>(g.n) * 4, hipMemcpyDeviceToDevice, s),
                  "previous classes");
    lr.k_done = st.k_done;
    lr.fixpoint = st.fixpoint;
    if (rb.bc.gid) {  // batched: counts and final buffers are per graph
        lr.h_final = nullptr;
        return lr;
    }
    lr.blocks_per_iter.resize(static_cast<size_t>(lr.k_done) + 1);
    hip_check(hipMemcpy(lr.blocks_per_iter.data(), rb.totals, (lr.k_done + 1) * 4, hipMemcpyDeviceToHost),
              "block counts");
    if (sink && !sink->levels.empty())
        lr.h_final = sink->levels[std::min<size_t>(lr.k_done, sink->levels.size() - 1)];
    else
        lr.h_final = rb.h[lr.k_done & 1];
    return lr;
}

bsim_result* make_result(bsim_ctx* ctx, const Staged& g, const LoopResult& lr, const uint64_t* h,
                         FinalOut& fo, Arena& keep, uint32_t flags, uint64_t* hashes_preset) {
    hipStream_t s = ctx->stream;
    bsim_result* r = new bsim_result();
    ResultPriv* p = new ResultPriv();
    memset(r, 0, sizeof(*r));
    r->priv = p;
    p->device = ctx->device;
    p->stream = s;
    p->blocks_per_iter = lr.blocks_per_iter;
    r->n_vertices = g.n;
    r->k_done = lr.k_done;
    r->fixpoint = lr.fixpoint;
    r->n_blocks = fo.n_blocks;
    r->n_summary_edges = fo.n_se;
    r->n_iter_launches = lr.launches;
    r->ms_iter_kernels = lr.ms_kernels;
    r->ms_hub_kernels = lr.ms_hub_kernels;
    r->n_timed_launches = lr.n_timed;
    r->n_split_launches = lr.split_launches;
    r->blocks_per_iter = p->blocks_per_iter.data();
    uint64_t* hashes = hashes_preset ? hashes_preset : keep.alloc<uint64_t>(g.n);
    if (g.n) hip_check(hipMemcpyAsync(hashes, h, static_cast<size_t>(g.n) * 8, hipMemcpyDeviceToDevice, s),
                       "hashes");
    void* dev[] = {hashes, fo.block_ids, fo.block_sizes, fo.se_src, fo.se_label, fo.se_dst};
    if (flags & BSIM_RESULT_ON_HOST) {
        const size_t sizes[] = {static_cast<size_t>(g.n) * 8, static_cast<size_t>(g.n) * 4,
                                static_cast<size_t>(fo.n_blocks) * 4, fo.n_se * 4, fo.n_se * 4, fo.n_se * 4};
        void* host[6];
        for (int i = 0; i < 6; i++) {
            host[i] = malloc(sizes[i] ? sizes[i] : 8);
            if (!host[i]) throw DeviceError{BSIM_E_NOMEM, "host result allocation failed"};
            p->host_ptrs.push_back(host[i]);
            if (sizes[i])
                hip_check(hipMemcpyAsync(host[i], dev[i], sizes[i], hipMemcpyDeviceToHost, s), "result copy");
        }
        hip_check(hipStreamSynchronize(s), "result sync");
        keep.release();
        r->mem_kind = BSIM_MEM_HOST;
        r->hashes = static_cast<uint64_t*>(host[0]);
        r->block_ids = static_cast<uint32_t*>(host[1]);
        r->block_sizes = static_cast<uint32_t*>(host[2]);
        r->se_src = static_cast<uint32_t*>(host[3]);
        r->se_label = static_cast<uint32_t*>(host[4]);
        r->se_dst = static_cast<uint32_t*>(host[5]);
    } else {
        for (void* q : dev) {
            p->device_ptrs.push_back(q);
            keep.detach(q);
        }
        r->mem_kind = BSIM_MEM_DEVICE;
        r->hashes = hashes;
        r->block_ids = fo.block_ids;
        r->block_sizes = fo.block_sizes;
        r->se_src = fo.se_src;
        r->se_label = fo.se_label;
        r->se_dst = fo.se_dst;
    }
    return r;
}

bsim_result* summarize_graph(bsim_ctx* ctx, const bsim_graph& graph, const bsim_params& p,
                             const std::vector<uint32_t>* labels) {
    validate_params(graph, p, true);
    hipStream_t s = ctx->stream;
    Arena arena(s), keep(s);
    ctx_back_arena(ctx, arena);
    hipEvent_t ev[4];
    for (auto& e : ev) hip_check(hipEventCreate(&e), "event");
    struct EvGuard {
        hipEvent_t* e;
        ~EvGuard() {
            for (int i = 0; i < 4; i++) (void)hipEventDestroy(e[i]);
        }
    } guard{ev};
    hip_check(hipEventRecord(ev[0], s), "event");
    Staged g;
    upload_graph(graph, g, arena, s);
    g.hub_table_slots = ctx->hub_table_slots;
    RunStatus* stage_status = arena.alloc<RunStatus>(1);
    stage_graph(g, stage_status, &ctx->status_host[3], arena, s);
    // direction / label parameterizations: refine the view h, take the
    // summary edges from the kept edges f
    const bool view = labels || (p.flags & (BSIM_BACKWARD | BSIM_BOTH_DIRECTIONS));
    DirectedView dv;
    if (view) {
        direction_view(g, p.flags, labels, dv, arena, s);
        stage_graph(dv.h, stage_status, &ctx->status_host[3], arena, s);
    }
    const Staged& gr = view ? dv.h : g;
    const Staged& gf = view ? dv.f : g;
    RunBuffers rb;
    alloc_run_buffers(gr, p.k_max, (p.flags & BSIM_STOP_AT_FIXPOINT) != 0, rb, arena, s);
    hip_check(hipEventRecord(ev[1], s), "event");
    const bool prev_edges = (p.flags & BSIM_PREV_LEVEL_EDGES) != 0;
    uint32_t* rep_prev = prev_edges ? arena.alloc<uint32_t>(gr.n + 1) : nullptr;
    LoopResult lr = run_refinement(ctx, gr, p, rb, nullptr, arena, rep_prev);
    hip_check(hipEventRecord(ev[2], s), "event");
    FinalOut fo;
    if (prev_edges)
        finalize_prev_level(gf, rb.rep, rep_prev, !(p.flags & BSIM_NO_SUMMARY_EDGES), fo, arena, keep, s);
    else
        finalize(gf, rb.rep, !(p.flags & BSIM_NO_SUMMARY_EDGES), fo, arena, keep, s);
    if (fo.n_blocks != lr.blocks_per_iter.back())
        throw DeviceError{BSIM_E_DEVICE, "internal: class count mismatch in finalize"};
    bsim_result* r = make_result(ctx, g, lr, lr.h_final, fo, keep, p.flags);
    hip_check(hipEventRecord(ev[3], s), "event");
    hip_check(hipEventSynchronize(ev[3]), "event");
    (void)hipEventElapsedTime(&r->ms_stage, ev[0], ev[1]);
    (void)hipEventElapsedTime(&r->ms_iterate, ev[1], ev[2]);
    (void)hipEventElapsedTime(&r->ms_finalize, ev[2], ev[3]);
    (void)hipEventElapsedTime(&r->ms_total, ev[0], ev[3]);
    ctx_note_demand(ctx, arena);
    return r;
}

}  // namespace bsim
