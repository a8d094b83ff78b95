// bsim_server.hip -- serving loop (a11): continuous batching of summarize
// and update requests.
//
// Worker threads each own a context and a HIP stream (default priority), so
// requests that run at the same time overlap their kernels on the device.
// When a request may start is the scheduler's decision (bsim_sched.h:
// admission by estimated device footprint against the budget left by
// running requests and server-owned states, submission order among those
// that fit, one update of a state at a time in submission order, refusal of
// requests that can never fit).  This file estimates the footprints, copies
// the requests, runs them, and keeps the contexts of the states the server
// owns: a server-owned state gets a context and stream of its own, so its
// updates never share a context with other work.  A state's device bytes
// are read only while none of its requests is queued or running.
#include <cstring>
#include <memory>
#include <string>
#include <thread>

#include "bsim_api_internal.h"
#include "bsim_sched.h"

using namespace bsim;

namespace {

struct HostGraphCopy {
    std::vector<uint32_t> row_off, tgt, type_off, type_ids;
    std::vector<uint8_t> lab, alive;
};

// What a worker needs to run a request.
struct Payload {
    uint32_t keep_state = 0;
    bsim_graph graph{};
    std::shared_ptr<HostGraphCopy> copy;
    bsim_params params{};
    bsim_state* state = nullptr;
    std::vector<bsim_update> ops;
    std::vector<std::vector<uint32_t>> op_types;
};

// A state the server owns: its context and stream, and its device bytes.
struct OwnedState {
    bsim_ctx* ctx = nullptr;
    hipStream_t stream = nullptr;
    uint64_t bytes = 0;
};

using Sched = Scheduler<Payload, OwnedState>;

uint64_t summarize_footprint(const bsim_graph& g, const bsim_params& p, bool keep) {
    const uint64_t n = g.n_vertices, m = g.n_edges, lb = g.label_bytes;
    const bool edges = !(p.flags & BSIM_NO_SUMMARY_EDGES);
    uint64_t b = m * (4 + lb + 8) + n * 160 + (1u << 20);
    if (g.mem_kind == BSIM_MEM_HOST) b += m * (4 + lb) + n * 16;
    if (edges) b += m * 36;
    // previous-level classes and their block ids
    if (p.flags & BSIM_PREV_LEVEL_EDGES) b += n * 24;
    // the direction view: kept edges with sources, and the view itself (2m
    // edges for both directions) staged a second time
    if (p.flags & (BSIM_BACKWARD | BSIM_BOTH_DIRECTIONS))
        b += m * (12 + lb) + ((p.flags & BSIM_BOTH_DIRECTIONS) ? 2 : 1) * m * (4 + 4 + 8) + n * 48;
    if (keep) {
        const uint64_t K = std::min<uint64_t>(p.k_max, 4096);
        b += m * (2 * (8 + lb) + 16 + 36) + n * (8 * (K + 1) + 140);
    }
    return b;
}

// Per-call scratch of an update: uploaded changes, prefix sums, finalize
// (estimated from the state's device bytes).
uint64_t update_footprint(uint64_t state_bytes_now, uint64_t n_ops) {
    return n_ops * 96 + state_bytes_now / 4 + (1u << 20);
}

}  // namespace

struct bsim_server {
    int device = 0;
    std::unique_ptr<Sched> sched;
    std::vector<std::thread> workers;
    std::vector<bsim_ctx*> ctxs;
    std::vector<hipStream_t> streams;
    std::mutex opt_mu;
    std::vector<std::pair<std::string, int64_t>> options;  // applied to every context of the server

    void worker(uint32_t w);
};

void bsim_server::worker(uint32_t w) {
    (void)hipSetDevice(device);
    Sched::Entry e;
    while (sched->next(e)) {
        Payload& r = e.payload;
        SchedDone d;
        OwnedState os;
        bsim_result* res = nullptr;
        bsim_state* st = nullptr;
        if (e.kind == BSIM_REQ_SUMMARIZE) {
            bsim_ctx* ctx = ctxs[w];
            if (r.keep_state) {
                // a server-owned state runs on a context and stream of its own
                if (hipStreamCreateWithFlags(&os.stream, hipStreamNonBlocking) != hipSuccess) {
                    d.status = BSIM_E_DEVICE;
                } else if ((d.status = bsim_ctx_create(device, os.stream, &os.ctx)) == BSIM_OK) {
                    ctx = os.ctx;
                    ctx->keep_work = 0;
                    std::vector<std::pair<std::string, int64_t>> opts;
                    {
                        std::lock_guard<std::mutex> lk(opt_mu);
                        opts = options;
                    }
                    for (const auto& o : opts) (void)bsim_ctx_set_option(ctx, o.first.c_str(), o.second);
                }
            }
            if (d.status == BSIM_OK)
                d.status = bsim_summarize(ctx, &r.graph, &r.params, r.keep_state ? &st : nullptr, &res);
            if (d.status == BSIM_OK && st) os.bytes = state_bytes(st);
            if (d.status != BSIM_OK || !st) {
                if (os.ctx) bsim_ctx_free(os.ctx);
                if (os.stream) (void)hipStreamDestroy(os.stream);
                os = OwnedState{};
            }
        }
        uint64_t new_bytes = 0;
        if (e.kind == BSIM_REQ_UPDATE) {
            d.status = bsim_apply_updates(r.state, r.ops.data(), r.ops.size(), &res);
            // this thread still holds the state (the scheduler runs one of its
            // requests at a time): its size is stable
            new_bytes = state_bytes(r.state);
        }
        d.result = res;
        d.state = st;
        sched->complete(e, d, os.ctx ? &os : nullptr, new_bytes);
        e = Sched::Entry{};
    }
}

extern "C" {

int bsim_server_create(int device, uint64_t budget, uint32_t n_workers, bsim_server** out) {
    if (!out || n_workers == 0 || n_workers > 64) return BSIM_E_INVALID;
    *out = nullptr;
    if (hipSetDevice(device) != hipSuccess) return BSIM_E_DEVICE;
    if (budget == 0) {
        size_t fr = 0, tot = 0;
        if (hipMemGetInfo(&fr, &tot) != hipSuccess) return BSIM_E_DEVICE;
        budget = static_cast<uint64_t>(fr) / 10 * 9;
    }
    bsim_server* s = new bsim_server();
    s->device = device;
    s->sched.reset(new Sched(budget));
    for (uint32_t w = 0; w < n_workers; w++) {
        hipStream_t st = nullptr;
        bsim_ctx* c = nullptr;
        int rc = hipStreamCreateWithFlags(&st, hipStreamNonBlocking) == hipSuccess ? BSIM_OK : BSIM_E_DEVICE;
        if (rc == BSIM_OK) rc = bsim_ctx_create(device, st, &c);
        if (rc != BSIM_OK) {
            if (st) (void)hipStreamDestroy(st);
            bsim_server_free(s);
            return rc;
        }
        // the scheduler's memory budget counts a request's temporaries
        // while it runs only: workers keep no buffer between requests
        c->keep_work = 0;
        s->streams.push_back(st);
        s->ctxs.push_back(c);
    }
    for (uint32_t w = 0; w < n_workers; w++) s->workers.emplace_back(&bsim_server::worker, s, w);
    *out = s;
    return BSIM_OK;
}

int bsim_server_submit(bsim_server* s, const bsim_request* req, uint64_t* ticket) {
    if (!s || !req || !ticket) return BSIM_E_INVALID;
    Sched::Entry e;
    e.kind = req->kind;
    e.t_submit = Sched::Clock::now();
    Payload& r = e.payload;
    try {
        if (req->kind == BSIM_REQ_SUMMARIZE) {
            if (!req->graph) return BSIM_E_INVALID;
            const bsim_graph& g = *req->graph;
            // a direction flag takes a view of the graph: no resident state
            validate_params(g, req->params, !req->keep_state);
            if (req->keep_state && (req->params.flags & BSIM_PREV_LEVEL_EDGES))
                throw DeviceError{BSIM_E_UNSUPPORTED, "BSIM_PREV_LEVEL_EDGES is supported without a state only"};
            r.keep_state = req->keep_state ? 1 : 0;
            r.params = req->params;
            r.graph = g;
            if (g.mem_kind == BSIM_MEM_HOST) {
                auto c = std::make_shared<HostGraphCopy>();
                const size_t n = g.n_vertices, m = g.n_edges;
                c->row_off.assign(g.row_off, g.row_off + n + 1);
                c->type_off.assign(g.type_off, g.type_off + n + 1);
                c->type_ids.assign(g.type_ids, g.type_ids + c->type_off[n]);
                if (m) {
                    c->tgt.assign(g.targets, g.targets + m);
                    const uint8_t* lb = static_cast<const uint8_t*>(g.labels);
                    c->lab.assign(lb, lb + m * g.label_bytes);
                }
                if (g.alive) c->alive.assign(g.alive, g.alive + n);
                r.graph.row_off = c->row_off.data();
                r.graph.type_off = c->type_off.data();
                r.graph.type_ids = c->type_ids.data();
                r.graph.targets = c->tgt.data();
                r.graph.labels = c->lab.data();
                r.graph.alive = g.alive ? c->alive.data() : nullptr;
                r.copy = c;
            }
            e.footprint = summarize_footprint(g, req->params, r.keep_state);
        } else if (req->kind == BSIM_REQ_UPDATE) {
            if (!req->state || (req->n_ops && !req->ops)) return BSIM_E_INVALID;
            r.state = req->state;
            e.state = req->state;
            r.ops.assign(req->ops, req->ops + req->n_ops);
            r.op_types.resize(r.ops.size());
            for (size_t i = 0; i < r.ops.size(); i++) {
                if (r.ops[i].n_types && r.ops[i].types) {
                    r.op_types[i].assign(r.ops[i].types, r.ops[i].types + r.ops[i].n_types);
                    r.ops[i].types = r.op_types[i].data();
                }
            }
        } else {
            return BSIM_E_INVALID;
        }
    } catch (const DeviceError& e) {
        return e.status;
    } catch (const std::bad_alloc&) {
        return BSIM_E_NOMEM;
    }
    const size_t n_ops = r.ops.size();
    return s->sched->submit(
        std::move(e), [](const void* st) { return state_bytes(static_cast<const bsim_state*>(st)); },
        [n_ops](uint64_t sb) { return update_footprint(sb, n_ops); }, ticket);
}

int bsim_server_poll(bsim_server* s, uint64_t ticket, int wait, bsim_result** out, bsim_state** state_out) {
    if (!s || !out) return BSIM_E_INVALID;
    *out = nullptr;
    if (state_out) *state_out = nullptr;
    SchedDone d;  // stays empty for an unknown, collected or unfinished ticket
    const int rc = s->sched->poll(ticket, wait != 0, &d);
    *out = static_cast<bsim_result*>(d.result);
    if (state_out) *state_out = static_cast<bsim_state*>(d.state);
    return rc;
}

int bsim_server_set_option(bsim_server* s, const char* name, int64_t value) {
    if (!s || !name) return BSIM_E_INVALID;
    if (!strcmp(name, "keep_work")) return BSIM_E_UNSUPPORTED;  // the memory budget needs it off
    // validated on a worker context first; contexts are not thread safe, so
    // only while the server is idle
    return s->sched->with_idle([&](std::map<const void*, OwnedState>& owned) {
        for (bsim_ctx* c : s->ctxs) {
            const int rc = bsim_ctx_set_option(c, name, value);
            if (rc != BSIM_OK) return rc;
        }
        for (auto& kv : owned) (void)bsim_ctx_set_option(kv.second.ctx, name, value);
        std::lock_guard<std::mutex> lk(s->opt_mu);
        s->options.emplace_back(name, value);
        return static_cast<int>(BSIM_OK);
    });
}

int bsim_server_stats_get(bsim_server* s, bsim_server_stats* out) {
    if (!s || !out) return BSIM_E_INVALID;
    memset(out, 0, sizeof(*out));
    const SchedStats st = s->sched->stats();
    out->submitted = st.submitted;
    out->completed = st.completed;
    out->failed = st.failed;
    out->bytes_in_use = st.bytes_in_use;
    out->bytes_budget = st.bytes_budget;
    for (int i = 0; i < 3; i++) {
        out->p50_ms[i] = st.p50_ms[i];
        out->p99_ms[i] = st.p99_ms[i];
    }
    out->busy_ms = st.busy_ms;
    return BSIM_OK;
}

int bsim_server_release_state(bsim_server* s, bsim_state* st) {
    if (!s || !st) return BSIM_E_INVALID;
    OwnedState os;
    if (!s->sched->release(st, &os)) return BSIM_E_INVALID;
    bsim_state_free(st);
    bsim_ctx_free(os.ctx);
    (void)hipStreamDestroy(os.stream);
    return BSIM_OK;
}

void bsim_server_free(bsim_server* s) {
    if (!s) return;
    // requests that have not started are cancelled (BSIM_E_BUSY); the
    // running ones finish
    s->sched->stop();
    for (auto& t : s->workers) t.join();
    (void)hipSetDevice(s->device);
    std::vector<SchedDone> left;
    std::map<const void*, OwnedState> owned;
    s->sched->drain(&left, &owned);
    for (const SchedDone& d : left)
        if (d.result) bsim_result_free(static_cast<bsim_result*>(d.result));
    for (auto& kv : owned) {
        bsim_state_free(static_cast<bsim_state*>(const_cast<void*>(kv.first)));
        bsim_ctx_free(kv.second.ctx);
        (void)hipStreamDestroy(kv.second.stream);
    }
    for (bsim_ctx* c : s->ctxs) bsim_ctx_free(c);
    for (hipStream_t st : s->streams) (void)hipStreamDestroy(st);
    delete s;
}

}  // extern "C"
