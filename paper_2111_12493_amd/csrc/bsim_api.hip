// bsim_api.hip -- the C ABI (include/bsim.h): contexts, batch summarization
// and results.  The call sequence of bsim_summarize follows Algorithm 4:
// initialization (type hashes), k hash-messaging phases, FindAndMerge; the
// phase loop stops at the fixpoint as described in bsim.h.
#include <cstdlib>
#include <cstring>
#include <new>

#include "bsim_api_internal.h"

using namespace bsim;

namespace bsim {

std::atomic<int64_t> g_fail_alloc_countdown{0};

// Allocating and returning the hundred-odd pool blocks of a large call costs
// milliseconds of host time per call (hipFreeAsync alone averages over
// 100 us on large blocks); one kept buffer costs nothing once grown.
void ctx_back_arena(bsim_ctx* ctx, Arena& arena, size_t at_least) {
    if (!ctx->keep_work) return;
    ctx->work_want = std::max(ctx->work_want, at_least);
    if (ctx->work_want > ctx->work_cap) {
        ctx_release_work(ctx);
        void* p = nullptr;
        if (device_alloc(&p, ctx->work_want, ctx->stream) == hipSuccess) {
            ctx->work = p;
            ctx->work_cap = ctx->work_want;
        } else {
            (void)hipGetLastError();
            ctx->work_want = 0;  // learn the demand again
        }
    }
    if (ctx->work) arena.back(ctx->work, ctx->work_cap);
}

void ctx_note_demand(bsim_ctx* ctx, const Arena& arena) {
    if (ctx->keep_work) ctx->work_want = std::max(ctx->work_want, arena.demand());
}

void ctx_release_work(bsim_ctx* ctx) {
    if (ctx->work) (void)hipFreeAsync(ctx->work, ctx->stream);
    ctx->work = nullptr;
    ctx->work_cap = 0;
}

}  // namespace bsim

extern "C" {

const char* bsim_status_string(int status) {
    switch (status) {
        case BSIM_OK: return "ok";
        case BSIM_E_INVALID: return "invalid input";
        case BSIM_E_RANGE: return "id or label out of range";
        case BSIM_E_NOMEM: return "out of memory";
        case BSIM_E_DEVICE: return "HIP runtime error";
        case BSIM_E_UNSUPPORTED: return "unsupported input";
        case BSIM_E_BUSY: return "busy";
        case BSIM_E_IO: return "file I/O error";
        default: return "unknown status";
    }
}

int bsim_ctx_create(int device, void* hip_stream, bsim_ctx** out) {
    if (!out) return BSIM_E_INVALID;
    *out = nullptr;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) return BSIM_E_DEVICE;
    if (hipSetDevice(device) != hipSuccess) return BSIM_E_DEVICE;
    bsim_ctx* c = new (std::nothrow) bsim_ctx();
    if (!c) return BSIM_E_NOMEM;
    c->device = device;
    c->stream = static_cast<hipStream_t>(hip_stream);
    c->hub_table_slots = query_hub_table_slots(device);
    if (hipHostMalloc(reinterpret_cast<void**>(&c->status_host), 4 * sizeof(RunStatus),
                      hipHostMallocDefault) != hipSuccess) {
        delete c;
        return BSIM_E_NOMEM;
    }
    if (hipHostMalloc(reinterpret_cast<void**>(&c->count_host), kStripes * sizeof(uint32_t),
                      hipHostMallocDefault) != hipSuccess) {
        bsim_ctx_free(c);
        return BSIM_E_NOMEM;
    }
    for (hipEvent_t& e : c->loop_ev) {
        if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) {
            bsim_ctx_free(c);
            return BSIM_E_DEVICE;
        }
    }
    // the allocation-free entry point's scratch on this device (once per device)
    const int rc = noalloc_scratch_init(device, &c->err);
    if (rc != BSIM_OK) {
        bsim_ctx_free(c);
        return rc;
    }
    // keep freed stream-ordered memory cached for later calls
    hipMemPool_t pool;
    if (hipDeviceGetDefaultMemPool(&pool, device) == hipSuccess) {
        uint64_t thr = UINT64_MAX;
        (void)hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &thr);
    }
    *out = c;
    return BSIM_OK;
}

void bsim_ctx_free(bsim_ctx* ctx) {
    if (!ctx) return;
    (void)hipSetDevice(ctx->device);
    ctx_release_work(ctx);
    (void)hipStreamSynchronize(ctx->stream);
    if (ctx->status_host) (void)hipHostFree(ctx->status_host);
    if (ctx->count_host) (void)hipHostFree(ctx->count_host);
    for (hipEvent_t e : ctx->loop_ev)
        if (e) (void)hipEventDestroy(e);
    delete ctx;
}

const char* bsim_last_error(const bsim_ctx* ctx) { return ctx ? ctx->err.c_str() : ""; }

const char* bsim_option_names(void) {
    return "chunk_max (refinement launches queued per stop-flag check, 1..4096); "
           "time_launches (N, 0..1048576: time every N-th refinement launch with HIP events, 0 = off); "
           "hub_table_slots (LDS slots of a hub-bucket block: power of two, 64..device limit); "
           "frontier_limit_pct (0..100: an update level whose frontier exceeds this share of the vertices is "
           "recomputed for all vertices; 0 = always, the plain full recomputation; default 10); "
           "frontier_edge_pct (1..100: the same for a frontier's share of the out-edges; default 15); "
           "tail_split_ppm (0..1000000: when refinement launches run one per stop check, a level that founds "
           "at most this many classes per million vertices has the next level's split run as a launch of its "
           "own, so a run that stops there computes no further hashes; 0 = off, default 100); "
           "autotune (0/1: batched calls pick their schedule per size class by timing the candidates on the "
           "first call of the class; 1 = default); "
           "batch_small_edges (N >= 0: a fixed batched schedule, graphs of at most N edges that fit one "
           "workgroup go to the small-graph launch, 0 = none; turns autotune off); "
           "batch_hub_table_slots (read only: the hub-table slots of the last batched call); "
           "keep_work (0/1: summarize and batched calls keep their temporaries in one device buffer of the "
           "largest size an earlier call needed, released with the ctx; 0 = every call allocates and returns "
           "them, and the buffer is released now; 1 = default); "
           "fail_alloc_after (N, 0..2^40: for tests of the failure paths, the N-th device allocation from now "
           "in this process fails as if the device were out of memory; 0 = off; reads the allocations left)";
}

int bsim_ctx_set_option(bsim_ctx* ctx, const char* name, int64_t value) {
    if (!ctx || !name) return BSIM_E_INVALID;
    if (!strcmp(name, "chunk_max")) {
        if (value < 1 || value > 4096) return BSIM_E_RANGE;
        ctx->chunk_max = static_cast<uint32_t>(value);
        return BSIM_OK;
    }
    if (!strcmp(name, "time_launches")) {
        if (value < 0 || value > (1 << 20)) return BSIM_E_RANGE;
        ctx->time_launches = static_cast<uint32_t>(value);
        return BSIM_OK;
    }
    if (!strcmp(name, "frontier_limit_pct")) {
        if (value < 0 || value > 100) return BSIM_E_RANGE;
        ctx->frontier_limit_pct = static_cast<uint32_t>(value);
        return BSIM_OK;
    }
    if (!strcmp(name, "frontier_edge_pct")) {
        if (value < 1 || value > 100) return BSIM_E_RANGE;
        ctx->frontier_edge_pct = static_cast<uint32_t>(value);
        return BSIM_OK;
    }
    if (!strcmp(name, "tail_split_ppm")) {
        if (value < 0 || value > 1000000) return BSIM_E_RANGE;
        ctx->tail_split_ppm = static_cast<uint32_t>(value);
        return BSIM_OK;
    }
    if (!strcmp(name, "fail_alloc_after")) {
        if (value < 0 || value > (1ll << 40)) return BSIM_E_RANGE;
        g_fail_alloc_countdown.store(value);
        return BSIM_OK;
    }
    if (!strcmp(name, "keep_work")) {
        if (value < 0 || value > 1) return BSIM_E_RANGE;
        ctx->keep_work = static_cast<uint32_t>(value);
        if (!value) {
            ctx_release_work(ctx);
            ctx->work_want = 0;
            if (hipStreamSynchronize(ctx->stream) != hipSuccess) return BSIM_E_DEVICE;
        }
        return BSIM_OK;
    }
    if (!strcmp(name, "autotune")) {
        if (value < 0 || value > 1) return BSIM_E_RANGE;
        ctx->autotune = static_cast<uint32_t>(value);
        if (!value) ctx->batch_tune.clear();
        return BSIM_OK;
    }
    if (!strcmp(name, "batch_small_edges")) {
        // a fixed schedule for the next batched calls (0: no small-graph launch)
        if (value < 0) return BSIM_E_RANGE;
        ctx->autotune = 0;
        ctx->batch_tune.clear();
        ctx->last_batch.small_edges = static_cast<uint64_t>(value);
        ctx->fixed_small_edges = static_cast<uint64_t>(value);
        return BSIM_OK;
    }
    if (!strcmp(name, "hub_table_slots")) {
        // power of two between 64 and what the device's LDS allows
        if (value < 64 || value > query_hub_table_slots(ctx->device, true) || (value & (value - 1)))
            return BSIM_E_RANGE;
        ctx->hub_table_slots = static_cast<uint32_t>(value);
        return BSIM_OK;
    }
    return BSIM_E_INVALID;
}

int bsim_ctx_get_option(const bsim_ctx* ctx, const char* name, int64_t* value) {
    if (!ctx || !name || !value) return BSIM_E_INVALID;
    if (!strcmp(name, "chunk_max")) {
        *value = ctx->chunk_max;
        return BSIM_OK;
    }
    if (!strcmp(name, "time_launches")) {
        *value = ctx->time_launches;
        return BSIM_OK;
    }
    if (!strcmp(name, "hub_table_slots")) {
        *value = ctx->hub_table_slots;
        return BSIM_OK;
    }
    if (!strcmp(name, "frontier_limit_pct")) {
        *value = ctx->frontier_limit_pct;
        return BSIM_OK;
    }
    if (!strcmp(name, "frontier_edge_pct")) {
        *value = ctx->frontier_edge_pct;
        return BSIM_OK;
    }
    if (!strcmp(name, "autotune")) {
        *value = ctx->autotune;
        return BSIM_OK;
    }
    if (!strcmp(name, "keep_work")) {
        *value = ctx->keep_work;
        return BSIM_OK;
    }
    if (!strcmp(name, "tail_split_ppm")) {
        *value = ctx->tail_split_ppm;
        return BSIM_OK;
    }
    if (!strcmp(name, "fail_alloc_after")) {
        *value = g_fail_alloc_countdown.load();
        return BSIM_OK;
    }
    if (!strcmp(name, "batch_small_edges")) {
        // the schedule of the last batched call (UINT64_MAX read as -1: every graph that fits)
        *value = static_cast<int64_t>(ctx->last_batch.small_edges);
        return BSIM_OK;
    }
    if (!strcmp(name, "batch_hub_table_slots")) {
        *value = ctx->last_batch.hub_table_slots;
        return BSIM_OK;
    }
    return BSIM_E_INVALID;
}

int bsim_summarize(bsim_ctx* ctx, const bsim_graph* graph, const bsim_params* params,
                   bsim_state** state_out, bsim_result** out) {
    if (out) *out = nullptr;
    if (state_out) *state_out = nullptr;
    if (!ctx || !graph || !params || !out) return BSIM_E_INVALID;
    try {
        hip_check(hipSetDevice(ctx->device), "set device");
        if (state_out) return summarize_with_state(ctx, *graph, *params, state_out, out);
        *out = summarize_graph(ctx, *graph, *params, nullptr);
        return BSIM_OK;
    } catch (const DeviceError& e) {
        ctx->err = e.msg;
        (void)hipStreamSynchronize(ctx->stream);
        return e.status;
    } catch (const std::bad_alloc&) {
        ctx->err = "host allocation failed";
        return BSIM_E_NOMEM;
    }
}

int bsim_summarize_labels(bsim_ctx* ctx, const bsim_graph* graph, const bsim_params* params,
                          const uint32_t* labels, uint32_t n_labels, bsim_result** out) {
    if (out) *out = nullptr;
    if (!ctx || !graph || !params || !out || (n_labels && !labels)) return BSIM_E_INVALID;
    try {
        hip_check(hipSetDevice(ctx->device), "set device");
        const std::vector<uint32_t> keep(labels, labels + n_labels);
        *out = summarize_graph(ctx, *graph, *params, &keep);
        return BSIM_OK;
    } catch (const DeviceError& e) {
        ctx->err = e.msg;
        (void)hipStreamSynchronize(ctx->stream);
        return e.status;
    } catch (const std::bad_alloc&) {
        ctx->err = "host allocation failed";
        return BSIM_E_NOMEM;
    }
}

namespace bsim {
SharedArrays::~SharedArrays() {
    if (!device_ptrs.empty()) {
        (void)hipSetDevice(device);
        for (void* q : device_ptrs) (void)hipFreeAsync(q, stream);
        (void)hipStreamSynchronize(stream);
    }
    for (void* q : host_ptrs) free(q);
}
}  // namespace bsim

void bsim_result_free(bsim_result* r) {
    if (!r) return;
    ResultPriv* p = static_cast<ResultPriv*>(r->priv);
    if (p) {
        if (p->device_ptrs.size()) {
            (void)hipSetDevice(p->device);
            for (void* q : p->device_ptrs) (void)hipFreeAsync(q, p->stream);
            (void)hipStreamSynchronize(p->stream);
        }
        for (void* q : p->host_ptrs) free(q);
        delete p;
    }
    delete r;
}

int bsim_result_copy(const bsim_result* r, const char* field, void* dst, uint32_t dst_mem_kind) {
    if (!r || !field || !dst) return BSIM_E_INVALID;
    const void* src = nullptr;
    size_t bytes = 0;
    if (!strcmp(field, "hashes")) {
        src = r->hashes;
        bytes = static_cast<size_t>(r->n_vertices) * 8;
    } else if (!strcmp(field, "block_ids")) {
        src = r->block_ids;
        bytes = static_cast<size_t>(r->n_vertices) * 4;
    } else if (!strcmp(field, "block_sizes")) {
        src = r->block_sizes;
        bytes = static_cast<size_t>(r->n_blocks) * 4;
    } else if (!strcmp(field, "se_src")) {
        src = r->se_src;
        bytes = static_cast<size_t>(r->n_summary_edges) * 4;
    } else if (!strcmp(field, "se_label")) {
        src = r->se_label;
        bytes = static_cast<size_t>(r->n_summary_edges) * 4;
    } else if (!strcmp(field, "se_dst")) {
        src = r->se_dst;
        bytes = static_cast<size_t>(r->n_summary_edges) * 4;
    } else {
        return BSIM_E_INVALID;
    }
    if (bytes == 0) return BSIM_OK;
    ResultPriv* p = static_cast<ResultPriv*>(r->priv);
    if (r->mem_kind == BSIM_MEM_HOST && dst_mem_kind == BSIM_MEM_HOST) {
        memcpy(dst, src, bytes);
        return BSIM_OK;
    }
    hipMemcpyKind kind = r->mem_kind == BSIM_MEM_HOST
                             ? hipMemcpyHostToDevice
                             : (dst_mem_kind == BSIM_MEM_HOST ? hipMemcpyDeviceToHost : hipMemcpyDeviceToDevice);
    if (hipSetDevice(p->device) != hipSuccess) return BSIM_E_DEVICE;
    if (hipMemcpyAsync(dst, src, bytes, kind, p->stream) != hipSuccess) return BSIM_E_DEVICE;
    if (hipStreamSynchronize(p->stream) != hipSuccess) return BSIM_E_DEVICE;
    return BSIM_OK;
}

void bsim_host_free(void* p) { free(p); }

}  // extern "C"
