// bsim_batch.hip -- batched summarization (a10): many independent graphs in
// one refinement run.
//
// The graphs are laid out as one disjoint union (vertex, edge and type ids
// shifted by per-graph offsets) and refined by the same tile / hub launches
// as a single graph, so one launch serves every graph and small graphs ride
// along with large ones instead of paying a launch sequence each.  A hash
// depends only on the vertex's own graph (no edge crosses graphs), so every
// vertex gets the hash it would get alone.  What is per graph:
//   - level-0 classes are keyed by a virtual class per graph, so no class
//     spans two graphs and class counts are counted per graph;
//   - a stop launch before every refinement launch applies the fixpoint /
//     k_max rule to each graph; a stopped graph's vertices keep their level
//     classes and hash buffer from then on;
//   - finalize numbers the union's classes by first occurrence; a graph's
//     vertices are contiguous, so its blocks are a contiguous id range and
//     its summary edges a contiguous slice of the sorted union edges.
// Each per-graph result is a view into the union's arrays, rebased to the
// graph's own vertex and block ids: identical to summarizing it alone.
#include <algorithm>
#include <chrono>
#include <cstring>

#include "bsim_api_internal.h"
#include "bsim_device.h"

namespace bsim {
namespace {

struct GraphPtrs {
    const uint32_t* row_off;
    const uint32_t* tgt;
    const void* lab;
    const uint32_t* type_off;
    const uint32_t* type_ids;
    const uint8_t* alive;
    uint32_t n;
    uint32_t pad;
};

// Largest g with off[g] <= x (off has G entries, off[0] = 0): the owner of
// item x when graphs own the ranges [off[g], off[g+1]).
__device__ __forceinline__ uint32_t owner(const uint64_t* off, uint32_t G, uint64_t x) {
    uint32_t lo = 0, hi = G;
    while (hi - lo > 1) {
        const uint32_t mid = (lo + hi) >> 1;
        if (off[mid] <= x) lo = mid; else hi = mid;
    }
    return lo;
}

// owner() for the items of one block: the owners of the block's first and
// last items bound the search (owners grow with the item), so each thread
// searches only the few graphs the block spans.  Every thread of the block
// must call it (it holds a barrier); count is the number of items.
__device__ __forceinline__ uint32_t block_owner(const uint64_t* off, uint32_t G, uint64_t count, uint64_t x,
                                                uint32_t* s_range) {
    const uint64_t first = static_cast<uint64_t>(blockIdx.x) * kBlock;
    const uint64_t last = min(first + kBlock, count) - 1;
    if (threadIdx.x == 0) {
        s_range[0] = owner(off, G, first);
        s_range[1] = owner(off, G, last);
    }
    __syncthreads();
    uint32_t lo = s_range[0], hi = s_range[1] + 1;
    const uint64_t y = min(x, last);
    while (hi - lo > 1) {
        const uint32_t mid = (lo + hi) >> 1;
        if (off[mid] <= y) lo = mid; else hi = mid;
    }
    return lo;
}

__global__ void k_type_counts(const GraphPtrs* gp, uint32_t G, uint32_t* cnt) {
    const uint32_t g = blockIdx.x * kBlock + threadIdx.x;
    if (g < G) cnt[g] = gp[g].type_off[gp[g].n];
}

__global__ void k_union_vertices(const GraphPtrs* __restrict__ gp, const uint64_t* __restrict__ voff,
                                 const uint64_t* __restrict__ eoff, const uint64_t* __restrict__ toff, uint32_t G,
                                 uint32_t n, uint32_t* __restrict__ row_off, uint32_t* __restrict__ type_off,
                                 uint8_t* __restrict__ alive, uint32_t* __restrict__ gid, RunStatus* status) {
    __shared__ uint32_t s_range[2];
    const uint32_t v = blockIdx.x * kBlock + threadIdx.x;
    const uint32_t g = block_owner(voff, G, n, v, s_range);
    if (v >= n) return;
    const GraphPtrs p = gp[g];
    const uint32_t l = v - static_cast<uint32_t>(voff[g]);
    row_off[v] = p.row_off[l] + static_cast<uint32_t>(eoff[g]);
    type_off[v] = p.type_off[l] + static_cast<uint32_t>(toff[g]);
    alive[v] = p.alive ? (p.alive[l] ? 1 : 0) : 1;
    gid[v] = g;
    // every graph's offsets must start at 0 and end at its own edge count
    if ((l == 0 && (p.row_off[0] != 0 || p.type_off[0] != 0)) ||
        (l + 1 == p.n && p.row_off[p.n] != eoff[g + 1] - eoff[g]))
        atomicOr(&status->error, kErrInvalid);
}

template <typename LabT>
__global__ void k_union_edges(const GraphPtrs* __restrict__ gp, const uint64_t* __restrict__ eoff,
                              const uint64_t* __restrict__ voff, uint32_t G, uint32_t m,
                              uint32_t* __restrict__ tgt, LabT* __restrict__ lab, RunStatus* status) {
    __shared__ uint32_t s_range[2];
    const uint32_t e = blockIdx.x * kBlock + threadIdx.x;
    const uint32_t g = block_owner(eoff, G, m, e, s_range);
    if (e >= m) return;
    const GraphPtrs p = gp[g];
    const uint32_t l = e - static_cast<uint32_t>(eoff[g]);
    const uint32_t w = p.tgt[l];
    if (w >= p.n) atomicOr(&status->error, kErrRange);
    tgt[e] = w + static_cast<uint32_t>(voff[g]);
    lab[e] = static_cast<const LabT*>(p.lab)[l];
}

__global__ void k_union_types(const GraphPtrs* __restrict__ gp, const uint64_t* __restrict__ toff, uint32_t G,
                              uint32_t nt, uint32_t* __restrict__ ids) {
    __shared__ uint32_t s_range[2];
    const uint32_t i = blockIdx.x * kBlock + threadIdx.x;
    const uint32_t g = block_owner(toff, G, nt, i, s_range);
    if (i >= nt) return;
    ids[i] = gp[g].type_ids[i - static_cast<uint32_t>(toff[g])];
}

// Per-graph views: block ids and summary edges rebased, hashes taken from
// the buffer of each graph's final parity.
__global__ void k_rebase_vertices(const uint32_t* __restrict__ gid, const uint32_t* __restrict__ done_level,
                                  const uint64_t* __restrict__ bbase, const uint64_t* __restrict__ h0,
                                  const uint64_t* __restrict__ h1, uint32_t n, uint32_t* __restrict__ bid,
                                  uint64_t* __restrict__ hashes) {
    const uint32_t v = blockIdx.x * kBlock + threadIdx.x;
    if (v >= n) return;
    const uint32_t g = gid[v];
    const uint32_t b = bid[v];
    if (b != 0xFFFFFFFFu) bid[v] = b - static_cast<uint32_t>(bbase[g]);
    hashes[v] = (done_level[g] & 1) ? h1[v] : h0[v];
}

// First summary edge of every graph: lower bound of its first block id.
__global__ void k_edge_starts(const uint32_t* __restrict__ se_src, uint32_t nse, const uint64_t* __restrict__ bbase,
                              uint32_t G, uint64_t* __restrict__ seoff) {
    const uint32_t g = blockIdx.x * kBlock + threadIdx.x;
    if (g > G) return;
    const uint64_t key = bbase[g];
    uint32_t lo = 0, hi = nse;
    while (lo < hi) {
        const uint32_t mid = (lo + hi) >> 1;
        if (se_src[mid] < key) lo = mid + 1; else hi = mid;
    }
    seoff[g] = lo;
}

__global__ void k_rebase_edges(const uint64_t* __restrict__ seoff, const uint64_t* __restrict__ bbase, uint32_t G,
                               uint32_t nse, uint32_t* __restrict__ se_src, uint32_t* __restrict__ se_dst) {
    __shared__ uint32_t s_range[2];
    const uint32_t i = blockIdx.x * kBlock + threadIdx.x;
    const uint32_t g = block_owner(seoff, G, nse, i, s_range);
    if (i >= nse) return;
    const uint32_t b = static_cast<uint32_t>(bbase[g]);
    se_src[i] -= b;
    se_dst[i] -= b;
}

inline uint32_t grid_for(uint64_t n) { return std::max<uint32_t>(ceil_div(n, kBlock), 1); }

template <typename T>
T* upload_vec(Arena& arena, const std::vector<T>& v, hipStream_t s) {
    T* d = arena.alloc<T>(v.size() + 1);
    if (!v.empty()) hip_check(hipMemcpyAsync(d, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, s), "upload");
    return d;
}

// Build the union on the device from the graphs' own arrays (host or device).
void build_union(const bsim_graph* graphs, uint32_t G, Staged& u, uint32_t*& gid, RunStatus* status,
                 RunStatus* status_host, Arena& arena, hipStream_t s) {
    const uint32_t lb = graphs[0].label_bytes;
    const bool on_host = graphs[0].mem_kind == BSIM_MEM_HOST;
    std::vector<GraphPtrs> gp(G);
    std::vector<uint64_t> voff(G + 1, 0), eoff(G + 1, 0), toff(G + 1, 0);
    for (uint32_t g = 0; g < G; g++) {
        voff[g + 1] = voff[g] + graphs[g].n_vertices;
        eoff[g + 1] = eoff[g] + graphs[g].n_edges;
    }
    if (voff[G] + G + 2 >= 0xFFFFFFF0ull) throw DeviceError{BSIM_E_UNSUPPORTED, "batch has too many vertices"};
    if (eoff[G] >= (1ull << 32)) throw DeviceError{BSIM_E_UNSUPPORTED, "batch has 2^32 edges or more"};
    if (on_host) {
        // stage every graph's arrays once in device memory
        for (uint32_t g = 0; g < G; g++) {
            const bsim_graph& in = graphs[g];
            const size_t n = in.n_vertices, m = in.n_edges;
            const size_t nt = in.type_off[n];
            uint32_t* ro = arena.alloc<uint32_t>(n + 1);
            uint32_t* to = arena.alloc<uint32_t>(n + 1);
            uint32_t* tg = arena.alloc<uint32_t>(m + 1);
            uint8_t* lab = arena.alloc<uint8_t>(m * lb + 4);
            uint32_t* ti = arena.alloc<uint32_t>(nt + 1);
            uint8_t* al = in.alive ? arena.alloc<uint8_t>(n + 1) : nullptr;
            hip_check(hipMemcpyAsync(ro, in.row_off, (n + 1) * 4, hipMemcpyHostToDevice, s), "upload");
            hip_check(hipMemcpyAsync(to, in.type_off, (n + 1) * 4, hipMemcpyHostToDevice, s), "upload");
            if (m) {
                hip_check(hipMemcpyAsync(tg, in.targets, m * 4, hipMemcpyHostToDevice, s), "upload");
                hip_check(hipMemcpyAsync(lab, in.labels, m * lb, hipMemcpyHostToDevice, s), "upload");
            }
            if (nt) hip_check(hipMemcpyAsync(ti, in.type_ids, nt * 4, hipMemcpyHostToDevice, s), "upload");
            if (al) hip_check(hipMemcpyAsync(al, in.alive, n, hipMemcpyHostToDevice, s), "upload");
            gp[g] = GraphPtrs{ro, tg, lab, to, ti, al, in.n_vertices, 0};
            toff[g + 1] = toff[g] + nt;
        }
    } else {
        for (uint32_t g = 0; g < G; g++) {
            const bsim_graph& in = graphs[g];
            gp[g] = GraphPtrs{in.row_off, in.targets, in.labels, in.type_off, in.type_ids, in.alive, in.n_vertices, 0};
        }
    }
    GraphPtrs* d_gp = upload_vec(arena, gp, s);
    if (!on_host) {
        uint32_t* cnt = arena.alloc<uint32_t>(G);
        k_type_counts<<<grid_for(G), kBlock, 0, s>>>(d_gp, G, cnt);
        std::vector<uint32_t> h(G);
        hip_check(hipMemcpyAsync(h.data(), cnt, G * 4ull, hipMemcpyDeviceToHost, s), "type counts");
        hip_check(hipStreamSynchronize(s), "type counts");
        for (uint32_t g = 0; g < G; g++) toff[g + 1] = toff[g] + h[g];
    }
    if (toff[G] >= (1ull << 32)) throw DeviceError{BSIM_E_UNSUPPORTED, "batch has too many type entries"};
    const uint32_t n = static_cast<uint32_t>(voff[G]);
    const uint32_t m = static_cast<uint32_t>(eoff[G]);
    const uint32_t nt = static_cast<uint32_t>(toff[G]);
    uint64_t* d_voff = upload_vec(arena, voff, s);
    uint64_t* d_eoff = upload_vec(arena, eoff, s);
    uint64_t* d_toff = upload_vec(arena, toff, s);
    uint32_t* row_off = arena.alloc<uint32_t>(n + 1ull);
    uint32_t* type_off = arena.alloc<uint32_t>(n + 1ull);
    uint32_t* tgt = arena.alloc<uint32_t>(m + 1ull);
    uint8_t* lab = arena.alloc<uint8_t>((m + 1ull) * lb);
    uint32_t* ids = arena.alloc<uint32_t>(nt + 1ull);
    uint8_t* alive = arena.alloc<uint8_t>(n + 1ull);
    gid = arena.alloc<uint32_t>(n + 1ull);
    hip_check(hipMemsetAsync(status, 0, sizeof(RunStatus), s), "status");
    hip_check(hipMemsetD32Async(reinterpret_cast<hipDeviceptr_t>(row_off + n), static_cast<int>(m), 1, s), "end");
    hip_check(hipMemsetD32Async(reinterpret_cast<hipDeviceptr_t>(type_off + n), static_cast<int>(nt), 1, s), "end");
    if (n)
        k_union_vertices<<<grid_for(n), kBlock, 0, s>>>(d_gp, d_voff, d_eoff, d_toff, G, n, row_off, type_off, alive,
                                                        gid, status);
    if (m) {
        if (lb == 2)
            k_union_edges<uint16_t><<<grid_for(m), kBlock, 0, s>>>(d_gp, d_eoff, d_voff, G, m, tgt,
                                                                 reinterpret_cast<uint16_t*>(lab), status);
        else
            k_union_edges<uint32_t><<<grid_for(m), kBlock, 0, s>>>(d_gp, d_eoff, d_voff, G, m, tgt,
                                                                 reinterpret_cast<uint32_t*>(lab), status);
    }
    if (nt) k_union_types<<<grid_for(nt), kBlock, 0, s>>>(d_gp, d_toff, G, nt, ids);
    hip_check(hipGetLastError(), "union launch");
    hip_check(hipMemcpyAsync(status_host, status, sizeof(RunStatus), hipMemcpyDeviceToHost, s), "union status");
    hip_check(hipStreamSynchronize(s), "union sync");
    if (status_host->error & kErrRange) throw DeviceError{BSIM_E_RANGE, "an edge target is out of its graph's range"};
    if (status_host->error & kErrInvalid) throw DeviceError{BSIM_E_INVALID, "a graph's offsets are malformed"};
    u.n = n;
    u.m = m;
    u.label_bytes = lb;
    u.row_off = row_off;
    u.tgt = tgt;
    u.lab = lab;
    u.type_off = type_off;
    u.type_ids = ids;
    u.alive = alive;
}

// Capacities of a small-graph workgroup on this device: at most 1,024
// vertices and 1,535 edges (below the hub degree, so a small graph has no
// hub) when the device gives a workgroup the LDS for them, else half; and
// the persistent grid (the workgroups that fit the CUs at once).
void small_capacity(int device, uint32_t* max_v, uint32_t* max_e, uint32_t* grid) {
    int lds = 0, cus = 0;
    if (hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, device) != hipSuccess) lds = 65536;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess) cus = 64;
    uint32_t v = 1024, e = kHubMinDegree - 1;
    while (v > 64 && small_graph_lds_bytes(v, e, nullptr) + 1024 > static_cast<uint64_t>(lds)) {
        v /= 2;
        e /= 2;
    }
    *max_v = v;
    *max_e = e;
    const uint64_t per_cu = std::max<uint64_t>(1, (160ull << 10) / (small_graph_lds_bytes(v, e, nullptr) + 1024));
    *grid = static_cast<uint32_t>(std::max(cus, 1) * per_cu);
}

}  // namespace

void batch_summarize(bsim_ctx* ctx, const bsim_graph* graphs, uint32_t G, const bsim_params& p,
                     bsim_result** outs, uint64_t small_edges) {
    hipStream_t s = ctx->stream;
    if (p.flags & BSIM_PREV_LEVEL_EDGES)
        throw DeviceError{BSIM_E_UNSUPPORTED, "BSIM_PREV_LEVEL_EDGES is supported by single-graph calls only"};
    for (uint32_t g = 0; g < G; g++) {
        validate_params(graphs[g], p, true);
        if (graphs[g].label_bytes != graphs[0].label_bytes || graphs[g].mem_kind != graphs[0].mem_kind)
            throw DeviceError{BSIM_E_INVALID, "all graphs of a batch need the same label_bytes and mem_kind"};
    }
    Arena arena(s);
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
    Staged u;
    uint32_t* gid = nullptr;
    RunStatus* ustat = arena.alloc<RunStatus>(1);
    build_union(graphs, G, u, gid, ustat, &ctx->status_host[3], arena, s);
    u.hub_table_slots = ctx->hub_table_slots;
    stage_graph(u, ustat, &ctx->status_host[3], arena, s);
    // direction parameterization: the view of a disjoint union is the
    // disjoint union of the graphs' views
    const bool view = (p.flags & (BSIM_BACKWARD | BSIM_BOTH_DIRECTIONS)) != 0;
    DirectedView dv;
    if (view) {
        direction_view(u, p.flags, nullptr, dv, arena, s);
        stage_graph(dv.h, ustat, &ctx->status_host[3], arena, s);
    }
    const Staged& ur = view ? dv.h : u;
    const Staged& uf = view ? dv.f : u;
    const bool stop = (p.flags & BSIM_STOP_AT_FIXPOINT) != 0;
    RunBuffers rb;
    alloc_run_buffers(ur, p.k_max, stop, rb, arena, s);
    rb.bc.gid = gid;
    rb.bc.n_graphs = G;
    rb.bc.virt_base = u.n;
    rb.bc.hist_cap = 64;
    rb.bc.done_level = arena.alloc<uint32_t>(G);
    rb.bc.fix = arena.alloc<uint32_t>(G);
    rb.bc.n_done = arena.alloc<uint32_t>(1);
    rb.bc.hist = arena.alloc<uint32_t>(static_cast<size_t>(rb.bc.hist_cap) * G);
    hip_check(hipMemsetAsync(rb.bc.done_level, 0xFF, G * 4ull, s), "done levels");
    hip_check(hipMemsetAsync(rb.bc.fix, 0, G * 4ull, s), "fix");
    hip_check(hipMemsetAsync(rb.bc.n_done, 0, 4, s), "done count");
    hip_check(hipMemsetAsync(rb.bc.hist, 0, static_cast<size_t>(rb.bc.hist_cap) * G * 4, s), "history");
    // small graphs: refined to their stop levels by the persistent launch,
    // each inside one workgroup's LDS (not with a direction view, whose
    // per-graph edge counts differ from the graphs' own)
    if (!view && small_edges > 0 && (stop || p.k_max <= 4096)) {
        uint32_t max_v = 0, max_e = 0, grid = 0;
        small_capacity(ctx->device, &max_v, &max_e, &grid);
        std::vector<uint32_t> list;
        std::vector<uint8_t> ext(G, 0);
        uint32_t max_n = 0;
        for (uint32_t g = 0; g < G; g++) {
            const bsim_graph& in = graphs[g];
            if (in.n_vertices <= max_v && in.n_edges <= std::min<uint64_t>(max_e, small_edges)) {
                list.push_back(g);
                ext[g] = 1;
                max_n = std::max(max_n, in.n_vertices);
            }
        }
        if (!list.empty()) {
            std::stable_sort(list.begin(), list.end(),
                             [&](uint32_t x, uint32_t y) { return graphs[x].n_edges > graphs[y].n_edges; });
            std::vector<uint64_t> voff(G + 1, 0);
            for (uint32_t g = 0; g < G; g++) voff[g + 1] = voff[g] + graphs[g].n_vertices;
            rb.small.glist = upload_vec(arena, list, s);
            rb.small.n_small = static_cast<uint32_t>(list.size());
            rb.small.voff = upload_vec(arena, voff, s);
            rb.small.queue = arena.alloc<uint32_t>(1);
            rb.small.max_v = max_v;
            rb.small.max_e = max_e;
            rb.small.max_n = max_n;
            rb.small.grid = grid;
            rb.bc.ext = upload_vec(arena, ext, s);
        }
    }
    hip_check(hipEventRecord(ev[1], s), "event");
    LoopResult lr = run_refinement(ctx, ur, p, rb, nullptr, arena);
    hip_check(hipEventRecord(ev[2], s), "event");

    // per-graph stop levels and class counts
    std::vector<uint32_t> done(G), fix(G);
    hip_check(hipMemcpyAsync(done.data(), rb.bc.done_level, G * 4ull, hipMemcpyDeviceToHost, s), "done levels");
    hip_check(hipMemcpyAsync(fix.data(), rb.bc.fix, G * 4ull, hipMemcpyDeviceToHost, s), "fix");
    hip_check(hipStreamSynchronize(s), "batch sync");
    uint32_t top = 0;
    for (uint32_t g = 0; g < G; g++) top = std::max(top, done[g]);
    std::vector<uint32_t> hist(static_cast<size_t>(top + 1) * G);
    hip_check(hipMemcpyAsync(hist.data(), rb.bc.hist, hist.size() * 4, hipMemcpyDeviceToHost, s), "history");
    hip_check(hipStreamSynchronize(s), "history sync");
    std::vector<uint64_t> bbase(G + 1, 0);
    std::vector<std::vector<uint32_t>> bpi(G);
    for (uint32_t g = 0; g < G; g++) {
        uint32_t run = 0;
        for (uint32_t j = 0; j <= done[g]; j++) bpi[g].push_back(run += hist[static_cast<size_t>(j) * G + g]);
        bbase[g + 1] = bbase[g] + run;
    }

    Arena keep(s);
    FinalOut fo;
    finalize(uf, rb.rep, !(p.flags & BSIM_NO_SUMMARY_EDGES), fo, arena, keep, s);
    if (fo.n_blocks != bbase[G]) throw DeviceError{BSIM_E_DEVICE, "internal: class count mismatch in batch finalize"};
    uint64_t* d_bbase = upload_vec(arena, bbase, s);
    uint64_t* hashes = keep.alloc<uint64_t>(u.n + 1ull);
    if (u.n)
        k_rebase_vertices<<<grid_for(u.n), kBlock, 0, s>>>(gid, rb.bc.done_level, d_bbase, rb.h[0], rb.h[1], u.n,
                                                           fo.block_ids, hashes);
    std::vector<uint64_t> seoff(G + 1, 0);
    const uint32_t nse = static_cast<uint32_t>(fo.n_se);
    if (nse) {
        uint64_t* d_seoff = arena.alloc<uint64_t>(G + 1);
        k_edge_starts<<<grid_for(G + 1ull), kBlock, 0, s>>>(fo.se_src, nse, d_bbase, G, d_seoff);
        k_rebase_edges<<<grid_for(nse), kBlock, 0, s>>>(d_seoff, d_bbase, G, nse, fo.se_src, fo.se_dst);
        hip_check(hipMemcpyAsync(seoff.data(), d_seoff, (G + 1) * 8ull, hipMemcpyDeviceToHost, s), "edge starts");
    }
    hip_check(hipGetLastError(), "batch rebase");
    hip_check(hipStreamSynchronize(s), "batch rebase sync");
    seoff[G] = nse;

    // shared arrays: on the device, or copied to the host once
    auto shared = std::make_shared<SharedArrays>();
    shared->device = ctx->device;
    shared->stream = s;
    void* dev[6] = {hashes, fo.block_ids, fo.block_sizes, fo.se_src, fo.se_label, fo.se_dst};
    const size_t sizes[6] = {u.n * 8ull, u.n * 4ull, fo.n_blocks * 4ull, nse * 4ull, nse * 4ull, nse * 4ull};
    void* base[6];
    const bool host = (p.flags & BSIM_RESULT_ON_HOST) != 0;
    for (int i = 0; i < 6; i++) {
        if (host) {
            base[i] = malloc(sizes[i] ? sizes[i] : 8);
            if (!base[i]) throw DeviceError{BSIM_E_NOMEM, "host result allocation failed"};
            shared->host_ptrs.push_back(base[i]);
            if (sizes[i]) hip_check(hipMemcpyAsync(base[i], dev[i], sizes[i], hipMemcpyDeviceToHost, s), "result copy");
        } else {
            base[i] = dev[i];
            keep.detach(dev[i]);
            shared->device_ptrs.push_back(dev[i]);
        }
    }
    hip_check(hipEventRecord(ev[3], s), "event");
    hip_check(hipEventSynchronize(ev[3]), "event");
    float ms[4] = {0, 0, 0, 0};
    (void)hipEventElapsedTime(&ms[0], ev[0], ev[1]);
    (void)hipEventElapsedTime(&ms[1], ev[1], ev[2]);
    (void)hipEventElapsedTime(&ms[2], ev[2], ev[3]);
    (void)hipEventElapsedTime(&ms[3], ev[0], ev[3]);
    uint64_t voff = 0;
    for (uint32_t g = 0; g < G; g++) {
        bsim_result* r = new bsim_result();
        memset(r, 0, sizeof(*r));
        ResultPriv* pr = new ResultPriv();
        r->priv = pr;
        pr->device = ctx->device;
        pr->stream = s;
        pr->shared = shared;
        pr->blocks_per_iter = bpi[g];
        r->n_vertices = graphs[g].n_vertices;
        r->k_done = done[g];
        r->fixpoint = fix[g];
        r->n_blocks = static_cast<uint32_t>(bbase[g + 1] - bbase[g]);
        r->n_summary_edges = seoff[g + 1] - seoff[g];
        r->mem_kind = host ? BSIM_MEM_HOST : BSIM_MEM_DEVICE;
        r->n_iter_launches = lr.launches;
        r->hashes = static_cast<uint64_t*>(base[0]) + voff;
        r->block_ids = static_cast<uint32_t*>(base[1]) + voff;
        r->block_sizes = static_cast<uint32_t*>(base[2]) + bbase[g];
        r->blocks_per_iter = pr->blocks_per_iter.data();
        r->se_src = static_cast<uint32_t*>(base[3]) + seoff[g];
        r->se_label = static_cast<uint32_t*>(base[4]) + seoff[g];
        r->se_dst = static_cast<uint32_t*>(base[5]) + seoff[g];
        r->ms_stage = ms[0];
        r->ms_iterate = ms[1];
        r->ms_finalize = ms[2];
        r->ms_total = ms[3];
        r->ms_iter_kernels = lr.ms_kernels;
        r->ms_hub_kernels = lr.ms_hub_kernels;
        r->n_timed_launches = lr.n_timed;
        outs[g] = r;
        voff += graphs[g].n_vertices;
    }
    ctx_note_demand(ctx, arena);
}

}  // namespace bsim

namespace bsim {
namespace {

// Size class of a batch for the autotuner's cache: graph count, total and
// largest edge counts (powers of two), label width, memory kind and flags.
uint64_t size_class(const bsim_graph* graphs, uint32_t G, const bsim_params& p) {
    uint64_t total = 0, largest = 0;
    for (uint32_t g = 0; g < G; g++) {
        total += graphs[g].n_edges;
        largest = std::max<uint64_t>(largest, graphs[g].n_edges);
    }
    return (static_cast<uint64_t>(bit_width(G)) << 56) | (static_cast<uint64_t>(bit_width(total)) << 48) |
           (static_cast<uint64_t>(bit_width(largest)) << 40) | (static_cast<uint64_t>(graphs[0].label_bytes) << 36) |
           (static_cast<uint64_t>(graphs[0].mem_kind) << 32) | p.flags;
}

// The autotuner: the first batched call of a size class on a context runs
// every candidate schedule on the batch itself, keeps the fastest for the
// class, and returns the results of a run with it.  A schedule never changes
// a result (every graph's result equals its own summarization), only the
// time.  Candidates: the small-graph launch off or on (graphs of up to the
// workgroup capacity), and hub-bucket tables of 4,096 or 16,384 LDS slots.
void tuned_batch(bsim_ctx* ctx, const bsim_graph* graphs, uint32_t G, const bsim_params& p, bsim_result** outs) {
    const uint32_t hub_default = ctx->hub_table_slots;
    bsim_ctx::BatchTune pick{ctx->autotune ? ~0ull : ctx->fixed_small_edges, hub_default};
    const uint64_t key = size_class(graphs, G, p);
    auto it = ctx->batch_tune.find(key);
    if (it != ctx->batch_tune.end()) {
        pick = it->second;
    } else if (ctx->autotune) {
        std::vector<bsim_ctx::BatchTune> cand;
        for (uint64_t small : {0ull, ~0ull})
            for (uint32_t hub : {4096u, 16384u})
                if (hub <= query_hub_table_slots(ctx->device, true)) cand.push_back({small, hub});
        double best = 0;
        // a ctx that has not yet sized its work buffer runs the first
        // candidate once untimed, so that no candidate pays for the pool
        // allocations the others are spared
        const bool size_work = ctx->keep_work && ctx->work_want == 0;
        for (size_t i = size_work && !cand.empty() ? 0 : 1; i <= cand.size(); i++) {
            const auto& c = cand[i ? i - 1 : 0];
            std::vector<bsim_result*> tmp(G, nullptr);
            ctx->hub_table_slots = c.hub_table_slots;
            const auto t0 = std::chrono::steady_clock::now();
            try {
                batch_summarize(ctx, graphs, G, p, tmp.data(), c.small_edges);
            } catch (...) {
                ctx->hub_table_slots = hub_default;
                for (bsim_result* r : tmp)
                    if (r) bsim_result_free(r);
                throw;
            }
            const double dt = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
            for (bsim_result* r : tmp)
                if (r) bsim_result_free(r);
            if (i && (best == 0 || dt < best)) {
                best = dt;
                pick = c;
            }
        }
        ctx->batch_tune[key] = pick;
    }
    ctx->hub_table_slots = pick.hub_table_slots;
    ctx->last_batch = pick;
    try {
        batch_summarize(ctx, graphs, G, p, outs, pick.small_edges);
    } catch (...) {
        ctx->hub_table_slots = hub_default;
        throw;
    }
    ctx->hub_table_slots = hub_default;
}

}  // namespace
}  // namespace bsim

extern "C" int bsim_batch_summarize(bsim_ctx* ctx, const bsim_graph* graphs, uint32_t n_graphs,
                                    const bsim_params* params, bsim_result** outs) {
    if (!ctx || !params || !outs || (n_graphs && !graphs)) return BSIM_E_INVALID;
    for (uint32_t g = 0; g < n_graphs; g++) outs[g] = nullptr;
    if (n_graphs == 0) return BSIM_OK;
    try {
        bsim::hip_check(hipSetDevice(ctx->device), "set device");
        bsim::tuned_batch(ctx, graphs, n_graphs, *params, outs);
        return BSIM_OK;
    } catch (const bsim::DeviceError& e) {
        ctx->err = e.msg;
        (void)hipStreamSynchronize(ctx->stream);
        for (uint32_t g = 0; g < n_graphs; g++) {
            if (outs[g]) bsim_result_free(outs[g]);
            outs[g] = nullptr;
        }
        return e.status;
    } catch (const std::bad_alloc&) {
        ctx->err = "host allocation failed";
        return BSIM_E_NOMEM;
    }
}
