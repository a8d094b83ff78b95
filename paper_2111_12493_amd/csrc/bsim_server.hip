// bsim_server.hip -- serving loop (a11): continuous batching of summarize
// and update requests.
//
// Worker threads each own a context and a HIP stream (default priority), so
// requests that run at the same time overlap their kernels on the device.
// A request is admitted when its estimated device footprint fits the budget
// left by running requests and server-owned states; requests that do not fit
// yet wait and start as memory frees up, in submission order among those
// that fit.  A request that cannot fit beside the server-owned states even
// with nothing else running is refused (BSIM_E_BUSY) at submit, or failed
// with BSIM_E_BUSY once that becomes true while it waits.  Updates of one
// state are applied one at a time, in submission order.  A server-owned state
// gets a context and stream of its own, so its updates never share a context
// with other work.  The device bytes of every state the server has seen are
// read only by the thread that runs its requests, and kept under the lock
// for admission.
#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <set>
#include <thread>

#include "bsim_api_internal.h"

using namespace bsim;

namespace {

using Clock = std::chrono::steady_clock;

struct HostGraphCopy {
    std::vector<uint32_t> row_off, tgt, type_off, type_ids;
    std::vector<uint8_t> lab, alive;
};

struct Request {
    uint64_t ticket = 0;
    uint32_t kind = 0;
    uint32_t keep_state = 0;
    bsim_graph graph{};
    std::shared_ptr<HostGraphCopy> copy;
    bsim_params params{};
    bsim_state* state = nullptr;
    std::vector<bsim_update> ops;
    std::vector<std::vector<uint32_t>> op_types;
    uint64_t footprint = 0;
    Clock::time_point t_submit;
};

struct Done {
    int status = BSIM_OK;
    bsim_result* result = nullptr;
    bsim_state* state = nullptr;
};

struct OwnedState {
    bsim_ctx* ctx = nullptr;
    hipStream_t stream = nullptr;
    uint64_t bytes = 0;
};

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
    uint64_t budget = 0, in_use = 0;
    std::vector<std::thread> workers;
    std::vector<bsim_ctx*> ctxs;
    std::vector<hipStream_t> streams;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<Request> queue;
    std::set<const bsim_state*> busy;
    std::map<uint64_t, Done> done;
    std::vector<bool> collected;               // by ticket: result already handed out
    std::map<bsim_state*, OwnedState> owned;
    uint64_t owned_bytes = 0;                  // sum of owned[].bytes (part of in_use)
    std::map<const bsim_state*, uint64_t> sbytes;  // device bytes of each state seen
    uint32_t running = 0;
    uint64_t next_ticket = 1, submitted = 0, completed = 0, failed = 0;
    bool stopping = false;
    std::vector<double> lat[3];
    Clock::time_point first_submit, last_done;
    bool any_submit = false;
    std::vector<std::pair<std::string, int64_t>> options;  // applied to every context of the server

    void worker(uint32_t w);
    bool pick(Request& out);
    void finish_locked(const Request& r, const Done& d);
    void fail_unfit_locked();
};

// Record a finished (or failed, or refused) request.  Holds mu.
void bsim_server::finish_locked(const Request& r, const Done& d) {
    const auto now = Clock::now();
    const double ms = std::chrono::duration<double, std::milli>(now - r.t_submit).count();
    lat[0].push_back(ms);
    lat[r.kind == BSIM_REQ_SUMMARIZE ? 1 : 2].push_back(ms);
    last_done = now;
    completed++;
    if (d.status != BSIM_OK) failed++;
    done[r.ticket] = d;
}

// With nothing running, a queued request larger than what the owned states
// leave of the budget can never start: fail it with BSIM_E_BUSY (one of a
// state's updates failing this way does not reorder the others).  Holds mu.
void bsim_server::fail_unfit_locked() {
    if (running) return;
    bool any = false;
    for (auto it = queue.begin(); it != queue.end();) {
        if (owned_bytes + it->footprint > budget) {
            Done d;
            d.status = BSIM_E_BUSY;
            finish_locked(*it, d);
            it = queue.erase(it);
            any = true;
        } else {
            ++it;
        }
    }
    if (any) cv_done.notify_all();
}

bool bsim_server::pick(Request& out) {
    fail_unfit_locked();
    // first request in submission order that fits and keeps per-state order
    std::set<const bsim_state*> earlier;
    for (auto it = queue.begin(); it != queue.end(); ++it) {
        if (it->kind == BSIM_REQ_UPDATE) {
            const bool blocked = busy.count(it->state) || earlier.count(it->state);
            earlier.insert(it->state);
            if (blocked) continue;
        }
        if (in_use + it->footprint > budget) continue;
        out = std::move(*it);
        queue.erase(it);
        return true;
    }
    return false;
}

void bsim_server::worker(uint32_t w) {
    (void)hipSetDevice(device);
    for (;;) {
        Request r;
        {
            std::unique_lock<std::mutex> lk(mu);
            cv_work.wait(lk, [&] { return (stopping && queue.empty()) || pick(r); });
            if (!r.kind) return;  // stopping with an empty queue
            in_use += r.footprint;
            running++;
            if (r.kind == BSIM_REQ_UPDATE) busy.insert(r.state);
        }
        Done d;
        OwnedState os;
        if (r.kind == BSIM_REQ_SUMMARIZE) {
            bsim_ctx* ctx = ctxs[w];
            if (r.keep_state) {
                // a server-owned state runs on a context and stream of its own
                if (hipStreamCreateWithFlags(&os.stream, hipStreamNonBlocking) != hipSuccess) {
                    d.status = BSIM_E_DEVICE;
                } else if ((d.status = bsim_ctx_create(device, os.stream, &os.ctx)) == BSIM_OK) {
                    ctx = os.ctx;
                    std::vector<std::pair<std::string, int64_t>> opts;
                    {
                        std::lock_guard<std::mutex> lk(mu);
                        opts = options;
                    }
                    for (const auto& o : opts) (void)bsim_ctx_set_option(ctx, o.first.c_str(), o.second);
                }
            }
            if (d.status == BSIM_OK)
                d.status = bsim_summarize(ctx, &r.graph, &r.params, r.keep_state ? &d.state : nullptr, &d.result);
            if (d.status == BSIM_OK && d.state) os.bytes = state_bytes(d.state);
            if (d.status != BSIM_OK || !d.state) {
                if (os.ctx) bsim_ctx_free(os.ctx);
                if (os.stream) (void)hipStreamDestroy(os.stream);
                os = OwnedState{};
            }
        }
        uint64_t new_bytes = 0;
        if (r.kind == BSIM_REQ_UPDATE) {
            d.status = bsim_apply_updates(r.state, r.ops.data(), r.ops.size(), &d.result);
            // this thread still holds the state (busy): its size is stable
            new_bytes = state_bytes(r.state);
        }
        {
            std::lock_guard<std::mutex> lk(mu);
            in_use -= r.footprint;
            running--;
            if (os.ctx) {
                owned[d.state] = os;
                in_use += os.bytes;
                owned_bytes += os.bytes;
                sbytes[d.state] = os.bytes;
            }
            if (r.kind == BSIM_REQ_UPDATE) {
                busy.erase(r.state);
                sbytes[r.state] = new_bytes;
                auto it = owned.find(r.state);
                if (it != owned.end()) {  // an update may grow an owned state
                    in_use = in_use - it->second.bytes + new_bytes;
                    owned_bytes = owned_bytes - it->second.bytes + new_bytes;
                    it->second.bytes = new_bytes;
                }
            }
            finish_locked(r, d);
        }
        cv_done.notify_all();
        cv_work.notify_all();
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
    s->budget = budget;
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
        s->streams.push_back(st);
        s->ctxs.push_back(c);
    }
    for (uint32_t w = 0; w < n_workers; w++) s->workers.emplace_back(&bsim_server::worker, s, w);
    *out = s;
    return BSIM_OK;
}

int bsim_server_submit(bsim_server* s, const bsim_request* req, uint64_t* ticket) {
    if (!s || !req || !ticket) return BSIM_E_INVALID;
    Request r;
    r.kind = req->kind;
    r.t_submit = Clock::now();
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
            r.footprint = summarize_footprint(g, req->params, r.keep_state);
        } else if (req->kind == BSIM_REQ_UPDATE) {
            if (!req->state || (req->n_ops && !req->ops)) return BSIM_E_INVALID;
            r.state = req->state;
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
    {
        std::lock_guard<std::mutex> lk(s->mu);
        if (r.kind == BSIM_REQ_UPDATE) {
            // with a request of the state queued or running, a worker may be
            // resizing it: take its size as of the last request; otherwise
            // nothing here touches it and it can be read now
            bool in_flight = s->busy.count(r.state) != 0;
            for (const Request& q : s->queue) in_flight = in_flight || q.state == r.state;
            auto it = s->sbytes.find(r.state);
            uint64_t sb = 0;
            if (in_flight && it != s->sbytes.end()) {
                sb = it->second;
            } else {
                sb = state_bytes(r.state);
                s->sbytes[r.state] = sb;
            }
            r.footprint = update_footprint(sb, r.ops.size());
        }
        if (s->stopping) return BSIM_E_INVALID;
        if (r.footprint + s->owned_bytes > s->budget) return BSIM_E_BUSY;
        r.ticket = s->next_ticket++;
        s->collected.push_back(false);
        *ticket = r.ticket;
        if (!s->any_submit) {
            s->first_submit = r.t_submit;
            s->any_submit = true;
        }
        s->submitted++;
        s->queue.push_back(std::move(r));
    }
    s->cv_work.notify_all();
    return BSIM_OK;
}

int bsim_server_poll(bsim_server* s, uint64_t ticket, int wait, bsim_result** out, bsim_state** state_out) {
    if (!s || !out) return BSIM_E_INVALID;
    *out = nullptr;
    if (state_out) *state_out = nullptr;
    std::unique_lock<std::mutex> lk(s->mu);
    if (ticket == 0 || ticket >= s->next_ticket) return BSIM_E_INVALID;
    if (s->collected[ticket - 1]) return BSIM_E_INVALID;  // each ticket is collected once
    auto ready = [&] { return s->done.count(ticket) != 0; };
    if (!ready()) {
        if (!wait) return BSIM_E_BUSY;
        s->cv_done.wait(lk, ready);
    }
    Done d = s->done[ticket];
    s->done.erase(ticket);
    s->collected[ticket - 1] = true;
    *out = d.result;
    if (state_out) *state_out = d.state;
    return d.status;
}

int bsim_server_set_option(bsim_server* s, const char* name, int64_t value) {
    if (!s || !name) return BSIM_E_INVALID;
    // validated on a worker context first; contexts are not thread safe, so
    // only while the server is idle
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->running || !s->queue.empty()) return BSIM_E_BUSY;
    for (bsim_ctx* c : s->ctxs) {
        const int rc = bsim_ctx_set_option(c, name, value);
        if (rc != BSIM_OK) return rc;
    }
    for (auto& kv : s->owned) (void)bsim_ctx_set_option(kv.second.ctx, name, value);
    s->options.emplace_back(name, value);
    return BSIM_OK;
}

int bsim_server_stats_get(bsim_server* s, bsim_server_stats* out) {
    if (!s || !out) return BSIM_E_INVALID;
    memset(out, 0, sizeof(*out));
    std::lock_guard<std::mutex> lk(s->mu);
    out->submitted = s->submitted;
    out->completed = s->completed;
    out->failed = s->failed;
    out->bytes_in_use = s->in_use;
    out->bytes_budget = s->budget;
    for (int i = 0; i < 3; i++) {
        std::vector<double> v = s->lat[i];
        if (v.empty()) continue;
        std::sort(v.begin(), v.end());
        auto pct = [&](double q) { return v[std::min(v.size() - 1, static_cast<size_t>(q * (v.size() - 1) + 0.5))]; };
        out->p50_ms[i] = pct(0.50);
        out->p99_ms[i] = pct(0.99);
    }
    if (s->any_submit && s->completed)
        out->busy_ms = std::chrono::duration<double, std::milli>(s->last_done - s->first_submit).count();
    return BSIM_OK;
}

int bsim_server_release_state(bsim_server* s, bsim_state* st) {
    if (!s || !st) return BSIM_E_INVALID;
    OwnedState os;
    {
        std::unique_lock<std::mutex> lk(s->mu);
        auto it = s->owned.find(st);
        if (it == s->owned.end()) return BSIM_E_INVALID;
        // wait until no request of this state is queued or running
        s->cv_done.wait(lk, [&] {
            if (s->busy.count(st)) return false;
            for (const Request& q : s->queue)
                if (q.state == st) return false;
            return true;
        });
        os = it->second;
        s->owned.erase(it);
        s->sbytes.erase(st);
        s->in_use -= os.bytes;
        s->owned_bytes -= os.bytes;
    }
    bsim_state_free(st);
    bsim_ctx_free(os.ctx);
    (void)hipStreamDestroy(os.stream);
    s->cv_work.notify_all();
    return BSIM_OK;
}

void bsim_server_free(bsim_server* s) {
    if (!s) return;
    {
        // requests that have not started are cancelled (BSIM_E_BUSY); the
        // running ones finish
        std::lock_guard<std::mutex> lk(s->mu);
        s->stopping = true;
        for (const Request& r : s->queue) {
            Done d;
            d.status = BSIM_E_BUSY;
            s->finish_locked(r, d);
        }
        s->queue.clear();
    }
    s->cv_work.notify_all();
    s->cv_done.notify_all();
    for (auto& t : s->workers) t.join();
    (void)hipSetDevice(s->device);
    for (auto& kv : s->done) {
        if (kv.second.result) bsim_result_free(kv.second.result);
    }
    for (auto& kv : s->owned) {
        bsim_state_free(kv.first);
        bsim_ctx_free(kv.second.ctx);
        (void)hipStreamDestroy(kv.second.stream);
    }
    for (bsim_ctx* c : s->ctxs) bsim_ctx_free(c);
    for (hipStream_t st : s->streams) (void)hipStreamDestroy(st);
    delete s;
}

}  // extern "C"
