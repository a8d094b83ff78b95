// bsim_noalloc.hip -- bsim_summarize_noalloc: the batch summarization of a
// device-resident graph into caller buffers, for callers that cannot
// allocate device memory (code under HIP graph capture, tight serving loops,
// harnesses that forbid it).
//
// Every temporary array of the call (the tile / hub schedule, type and
// level hashes, class representatives, split tables, hub scratch keys, the
// finalize sort) is carved out of one file-scope device array, `scratch`,
// by a bump arena that refuses to reach the allocator.  Each device holds
// its own copy of the array for the life of the process; its address on a
// device is looked up once, with that device current, when the first
// context on it is created (bsim_ctx_create).  The kernels are those of
// bsim_summarize and take that address like any other buffer.
//
// All calls on one device share its scratch: calls that overlap in time on
// one device (two host threads, or two streams) race and must not be made.
// Every region a call reads is written or cleared by the same call first, so
// nothing carries over from the previous call.
#include <mutex>

#include "bsim_api_internal.h"

namespace {

constexpr uint64_t kScratchBytes = 256ull << 20;
constexpr int kMaxDevices = 64;

static __device__ __align__(256) uint8_t scratch[kScratchBytes];

std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

}  // namespace

namespace bsim {

int noalloc_scratch_init(int device, std::string* err) {
    if (device < 0 || device >= kMaxDevices) {
        if (err) *err = "device index beyond the scratch table";
        return BSIM_E_UNSUPPORTED;
    }
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (g_scratch_ptr[device]) return BSIM_OK;
    // the array's name is a host-side stand-in: only this address is the
    // device's copy (the caller made `device` current)
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
        if (err) *err = std::string("scratch address lookup: ") + hipGetErrorString(e);
        return BSIM_E_DEVICE;
    }
    g_scratch_ptr[device] = p;
    return BSIM_OK;
}

namespace {

void* scratch_of(int device) {
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    return (device >= 0 && device < kMaxDevices) ? g_scratch_ptr[device] : nullptr;
}

// A bound on the scratch a graph needs, so that clearly oversized graphs are
// refused before any launch (the strict arena is the exact check): per vertex
// the type and two level hashes, the representative, two split tables and
// the tile lists; per edge the hub keys, the summary-edge keys, the sort's
// second buffer, flags, positions and the three output columns.
uint64_t scratch_bound(uint64_t n, uint64_t m) {
    return 72 * n + 2 * 8 * split_table_slots(n) + 56 * m + (16ull << 20);
}

void run(bsim_ctx* ctx, const bsim_graph& graph, const bsim_params& p, bsim_noalloc_out& out) {
    validate_params(graph, p);
    if (graph.mem_kind != BSIM_MEM_DEVICE)
        throw DeviceError{BSIM_E_INVALID, "bsim_summarize_noalloc takes device-resident graphs only"};
    if (p.flags & ~(BSIM_STOP_AT_FIXPOINT | BSIM_UNTYPED | BSIM_NO_SUMMARY_EDGES))
        throw DeviceError{BSIM_E_UNSUPPORTED, "bsim_summarize_noalloc takes only BSIM_STOP_AT_FIXPOINT, "
                                              "BSIM_UNTYPED and BSIM_NO_SUMMARY_EDGES"};
    const bool edges = !(p.flags & BSIM_NO_SUMMARY_EDGES);
    const uint64_t n = graph.n_vertices, m = graph.n_edges;
    if ((n && (!out.hashes || !out.block_ids || !out.block_sizes)) || !out.blocks_per_iter ||
        (edges && m && (!out.se_src || !out.se_label || !out.se_dst)))
        throw DeviceError{BSIM_E_INVALID, "an output array is missing"};
    // k_done <= k_max, and at most n + 1 with the fixpoint test
    const uint64_t k_bound =
        (p.flags & BSIM_STOP_AT_FIXPOINT) ? std::min<uint64_t>(p.k_max, n + 1) : static_cast<uint64_t>(p.k_max);
    if (out.blocks_per_iter_cap < k_bound + 1)
        throw DeviceError{BSIM_E_INVALID, "blocks_per_iter_cap must be at least min(k_max, n + 1) + 1"};
    if (scratch_bound(n, m) > kScratchBytes)
        throw DeviceError{BSIM_E_UNSUPPORTED, "the graph needs more than the " + std::to_string(kScratchBytes) +
                                                  " bytes of scratch of bsim_summarize_noalloc"};
    void* base = scratch_of(ctx->device);
    if (!base) throw DeviceError{BSIM_E_DEVICE, "no scratch address for this device"};
    hipStream_t s = ctx->stream;
    Arena arena(s);
    arena.back(base, kScratchBytes);
    arena.set_strict(true);
    Staged g;
    upload_graph(graph, g, arena, s);  // device pointers, nothing copied
    g.hub_table_slots = ctx->hub_table_slots;
    RunStatus* stage_status = arena.alloc<RunStatus>(1);
    stage_graph(g, stage_status, &ctx->status_host[3], arena, s);
    RunBuffers rb;
    alloc_run_buffers(g, p.k_max, (p.flags & BSIM_STOP_AT_FIXPOINT) != 0, rb, arena, s);
    LoopResult lr = run_refinement(ctx, g, p, rb, nullptr, arena, nullptr, false);
    FinalOut fo;
    finalize(g, rb.rep, edges, fo, arena, arena, s);
    if (fo.n_blocks != lr.blocks_per_iter.back())
        throw DeviceError{BSIM_E_DEVICE, "internal: class count mismatch in finalize"};
    // results into the caller's arrays
    if (n) {
        hip_check(hipMemcpyAsync(out.hashes, lr.h_final, n * 8, hipMemcpyDeviceToDevice, s), "hashes");
        hip_check(hipMemcpyAsync(out.block_ids, fo.block_ids, n * 4, hipMemcpyDeviceToDevice, s), "block ids");
    }
    if (fo.n_blocks)
        hip_check(hipMemcpyAsync(out.block_sizes, fo.block_sizes, fo.n_blocks * 4ull, hipMemcpyDeviceToDevice, s),
                  "block sizes");
    if (edges && fo.n_se) {
        hip_check(hipMemcpyAsync(out.se_src, fo.se_src, fo.n_se * 4, hipMemcpyDeviceToDevice, s), "se_src");
        hip_check(hipMemcpyAsync(out.se_label, fo.se_label, fo.n_se * 4, hipMemcpyDeviceToDevice, s), "se_label");
        hip_check(hipMemcpyAsync(out.se_dst, fo.se_dst, fo.n_se * 4, hipMemcpyDeviceToDevice, s), "se_dst");
    }
    hip_check(hipStreamSynchronize(s), "noalloc sync");
    for (size_t i = 0; i < lr.blocks_per_iter.size(); i++) out.blocks_per_iter[i] = lr.blocks_per_iter[i];
    out.k_done = lr.k_done;
    out.fixpoint = lr.fixpoint;
    out.n_blocks = fo.n_blocks;
    out.n_summary_edges = edges ? fo.n_se : 0;
    out.scratch_used = arena.demand();
}

}  // namespace
}  // namespace bsim

using namespace bsim;

extern "C" {

uint64_t bsim_noalloc_scratch_bytes(void) { return kScratchBytes; }

int bsim_summarize_noalloc(bsim_ctx* ctx, const bsim_graph* graph, const bsim_params* params,
                           bsim_noalloc_out* out) {
    if (!ctx || !graph || !params || !out) return BSIM_E_INVALID;
    try {
        hip_check(hipSetDevice(ctx->device), "set device");
        bsim_noalloc_out o = *out;
        run(ctx, *graph, *params, o);
        *out = o;
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

}  // extern "C"
