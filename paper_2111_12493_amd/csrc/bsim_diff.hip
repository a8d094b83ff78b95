// Change detection from two snapshots without a change log (Sec. 3.2: the
// change classes between the graph at time t and at t+1).  Produces the
// ordered update batch that turns `before` into `after`:
//   ADD_V  every new id before.n .. after.n - 1, with after's type list;
//   MOD_V  every vertex alive in both whose type set changed;
//   DEL_E  every distinct triple of before missing from after, both
//          endpoints alive after, in order of its first copy in before;
//   ADD_E  every distinct triple of after missing from before, in order of
//          its first copy in after;
//   DEL_V  every vertex alive before (or new) and dead after.
// The edge sets are compared with one open-addressing table per snapshot:
// a slot holds an edge index + 1, the triple is read back from the edge
// arrays, and the smallest index of a triple's copies wins (atomicMin), so
// each distinct triple has one deterministic representative.
#include <cstdlib>
#include <cstring>

#include "bsim_api_internal.h"

namespace bsim {
namespace {

struct EdgeSet {
    const uint32_t* src;
    const uint32_t* tgt;
    const void* lab;
    uint32_t label_bytes;
    uint32_t m;
    uint32_t* table;  // mask + 1 slots: 0 empty, else edge index + 1
    uint32_t mask;
};

__device__ __forceinline__ uint32_t label_at(const EdgeSet& g, uint32_t e) {
    return g.label_bytes == 2 ? static_cast<const uint16_t*>(g.lab)[e] : static_cast<const uint32_t*>(g.lab)[e];
}

__device__ __forceinline__ uint32_t triple_home(uint32_t u, uint32_t l, uint32_t w, uint32_t mask) {
    return static_cast<uint32_t>(mix64(((static_cast<uint64_t>(u) << 32) | w) ^ mix64(kCL + l))) & mask;
}

__device__ __forceinline__ bool same_triple(const EdgeSet& g, uint32_t f, uint32_t u, uint32_t l, uint32_t w) {
    return g.src[f] == u && g.tgt[f] == w && label_at(g, f) == l;
}

// The row of each edge: the largest v with row_off[v] <= e.
__global__ void __launch_bounds__(kBlock) k_edge_rows(const uint32_t* __restrict__ row_off, uint32_t n, uint32_t m,
                                                      uint32_t* __restrict__ src) {
    const uint32_t e = blockIdx.x * kBlock + threadIdx.x;
    if (e >= m) return;
    uint32_t lo = 0, hi = n;
    while (hi - lo > 1) {
        const uint32_t mid = lo + (hi - lo) / 2;
        if (row_off[mid] <= e) lo = mid; else hi = mid;
    }
    src[e] = lo;
}

// Every edge joins the slot of its triple; the smallest index stays.  The
// table has at least twice as many slots as edges, so a probe ends.
__global__ void __launch_bounds__(kBlock) k_triple_insert(EdgeSet g) {
    const uint32_t e = blockIdx.x * kBlock + threadIdx.x;
    if (e >= g.m) return;
    const uint32_t u = g.src[e], l = label_at(g, e), w = g.tgt[e];
    uint32_t slot = triple_home(u, l, w, g.mask);
    for (;;) {
        uint32_t cur = g.table[slot];  // a stale 0 only costs the CAS
        if (cur == 0) {
            cur = atomicCAS(&g.table[slot], 0u, e + 1);
            if (cur == 0) return;
        }
        if (same_triple(g, cur - 1, u, l, w)) {
            atomicMin(&g.table[slot], e + 1);
            return;
        }
        slot = (slot + 1) & g.mask;
    }
}

// flag[e] = 1 when e represents its triple in `own` and the triple is absent
// from `other` (and, with keep_alive, both endpoints are alive there).
__global__ void __launch_bounds__(kBlock) k_triple_missing(EdgeSet own, EdgeSet other,
                                                           const uint8_t* __restrict__ keep_alive,
                                                           uint32_t* __restrict__ flag) {
    const uint32_t e = blockIdx.x * kBlock + threadIdx.x;
    if (e >= own.m) return;
    const uint32_t u = own.src[e], l = label_at(own, e), w = own.tgt[e];
    // the triple's slot: every slot before it on the probe path was filled
    // before it was taken, and slots never empty again
    uint32_t slot = triple_home(u, l, w, own.mask);
    uint32_t rep = 0;
    for (;;) {
        const uint32_t cur = own.table[slot];
        if (cur == 0) break;  // not reached: the insert launch placed every edge
        if (same_triple(own, cur - 1, u, l, w)) {
            rep = cur;
            break;
        }
        slot = (slot + 1) & own.mask;
    }
    uint32_t out = 0;
    if (rep == e + 1 && (!keep_alive || (keep_alive[u] && keep_alive[w]))) {
        bool found = false;
        if (other.m) {
            uint32_t s2 = triple_home(u, l, w, other.mask);
            for (;;) {
                const uint32_t cur = other.table[s2];
                if (cur == 0) break;
                if (same_triple(other, cur - 1, u, l, w)) {
                    found = true;
                    break;
                }
                s2 = (s2 + 1) & other.mask;
            }
        }
        out = found ? 0u : 1u;
    }
    flag[e] = out;
}

// Per vertex of after: kind[v] = 1 for MOD_V, 2 for DEL_V (ADD_V is every
// id >= n0); *err = 1 when a vertex dead before is alive after.
__global__ void __launch_bounds__(kBlock) k_vertex_changes(uint32_t n0, uint32_t n1,
                                                           const uint8_t* __restrict__ alive0,
                                                           const uint8_t* __restrict__ alive1,
                                                           const uint32_t* __restrict__ toff0,
                                                           const uint32_t* __restrict__ tids0,
                                                           const uint32_t* __restrict__ toff1,
                                                           const uint32_t* __restrict__ tids1,
                                                           uint8_t* __restrict__ kind, uint32_t* __restrict__ err) {
    const uint32_t v = blockIdx.x * kBlock + threadIdx.x;
    if (v >= n1) return;
    const bool a0 = v >= n0 || !alive0 || alive0[v];
    const bool a1 = !alive1 || alive1[v];
    uint8_t k = 0;
    if (v < n0 && !a0 && a1) atomicOr(err, 1u);
    if (a0 && !a1) {
        k = 2;
    } else if (v < n0 && a0 && a1) {
        const uint32_t b0 = toff0[v], e0 = toff0[v + 1], b1 = toff1[v], e1 = toff1[v + 1];
        bool same = true;
        for (uint32_t i = b0; i < e0 && same; i++) {
            bool in = false;
            for (uint32_t j = b1; j < e1 && !in; j++) in = tids1[j] == tids0[i];
            same = in;
        }
        for (uint32_t j = b1; j < e1 && same; j++) {
            bool in = false;
            for (uint32_t i = b0; i < e0 && !in; i++) in = tids0[i] == tids1[j];
            same = in;
        }
        if (!same) k = 1;
    }
    kind[v] = k;
}

__global__ void __launch_bounds__(kBlock) k_gather_flagged(EdgeSet g, const uint32_t* __restrict__ flag,
                                                           const uint32_t* __restrict__ pos,
                                                           uint32_t* __restrict__ out) {
    const uint32_t e = blockIdx.x * kBlock + threadIdx.x;
    if (e >= g.m || !flag[e]) return;
    const uint64_t p = 3ull * pos[e];
    out[p] = g.src[e];
    out[p + 1] = label_at(g, e);
    out[p + 2] = g.tgt[e];
}

template <typename T>
std::vector<T> to_host(const T* p, size_t count, hipStream_t s) {
    std::vector<T> h(count);
    if (count) hip_check(hipMemcpyAsync(h.data(), p, count * sizeof(T), hipMemcpyDeviceToHost, s), "diff copy");
    return h;
}

// The (u, l, w) triples of the flagged edges, in edge order, compacted on
// the device (a scan) and copied to the host.
std::vector<uint32_t> flagged_triples(const EdgeSet& g, const uint32_t* flag, Arena& arena, hipStream_t s) {
    if (g.m == 0) return {};
    uint32_t* pos = arena.alloc<uint32_t>(static_cast<size_t>(g.m) + 1);
    uint32_t* total = arena.alloc<uint32_t>(1);
    scan_exclusive(flag, pos, g.m, total, arena, s);
    const std::vector<uint32_t> cnt = to_host(total, 1, s);
    hip_check(hipStreamSynchronize(s), "diff sync");
    uint32_t* out = arena.alloc<uint32_t>(3ull * cnt[0] + 3);
    k_gather_flagged<<<ceil_div(g.m, kBlock), kBlock, 0, s>>>(g, flag, pos, out);
    hip_check(hipGetLastError(), "diff gather");
    std::vector<uint32_t> h = to_host(out, 3ull * cnt[0], s);
    hip_check(hipStreamSynchronize(s), "diff sync");
    return h;
}

EdgeSet edge_set(const Staged& g, Arena& arena, hipStream_t s) {
    EdgeSet es{};
    es.m = static_cast<uint32_t>(g.m);
    es.tgt = g.tgt;
    es.lab = g.lab;
    es.label_bytes = g.label_bytes;
    uint32_t* src = arena.alloc<uint32_t>(static_cast<size_t>(es.m) + 1);
    if (es.m) k_edge_rows<<<ceil_div(es.m, kBlock), kBlock, 0, s>>>(g.row_off, g.n, es.m, src);
    es.src = src;
    const uint64_t cap = table_slots(2ull * es.m + 2, 64, "the edge-triple table of a snapshot");
    es.table = arena.alloc<uint32_t>(cap);
    es.mask = static_cast<uint32_t>(cap - 1);
    hip_check(hipMemsetAsync(es.table, 0, static_cast<size_t>(cap) * 4, s), "triple table");
    if (es.m) k_triple_insert<<<ceil_div(es.m, kBlock), kBlock, 0, s>>>(es);
    hip_check(hipGetLastError(), "triple table launch");
    return es;
}

bsim_update* diff_snapshots(bsim_ctx* ctx, const bsim_graph& b, const bsim_graph& a, uint64_t* n_ops) {
    const bsim_params p{0, 0};
    validate_params(b, p);
    validate_params(a, p);
    if (a.n_vertices < b.n_vertices)
        throw DeviceError{BSIM_E_INVALID, "the later snapshot has fewer vertex ids"};
    hipStream_t s = ctx->stream;
    Arena arena(s);
    Staged g0, g1;
    upload_graph(b, g0, arena, s);
    upload_graph(a, g1, arena, s);
    RunStatus* st = arena.alloc<RunStatus>(1);
    stage_graph(g0, st, &ctx->status_host[3], arena, s);  // validates
    stage_graph(g1, st, &ctx->status_host[3], arena, s);
    const uint32_t n0 = g0.n, n1 = g1.n;
    const EdgeSet e0 = edge_set(g0, arena, s);
    const EdgeSet e1 = edge_set(g1, arena, s);
    uint32_t* del_flag = arena.alloc<uint32_t>(static_cast<size_t>(e0.m) + 1);
    uint32_t* add_flag = arena.alloc<uint32_t>(static_cast<size_t>(e1.m) + 1);
    if (e0.m) k_triple_missing<<<ceil_div(e0.m, kBlock), kBlock, 0, s>>>(e0, e1, g1.alive, del_flag);
    if (e1.m) k_triple_missing<<<ceil_div(e1.m, kBlock), kBlock, 0, s>>>(e1, e0, nullptr, add_flag);
    uint8_t* kind = arena.alloc<uint8_t>(static_cast<size_t>(n1) + 1);
    uint32_t* err = arena.alloc<uint32_t>(1);
    hip_check(hipMemsetAsync(err, 0, 4, s), "diff error");
    if (n1)
        k_vertex_changes<<<ceil_div(n1, kBlock), kBlock, 0, s>>>(n0, n1, g0.alive, g1.alive, g0.type_off, g0.type_ids,
                                                                g1.type_off, g1.type_ids, kind, err);
    hip_check(hipGetLastError(), "diff launch");
    const std::vector<uint8_t> kh = to_host(kind, n1, s);
    const std::vector<uint32_t> eh = to_host(err, 1, s);
    hip_check(hipStreamSynchronize(s), "diff sync");
    if (eh[0]) throw DeviceError{BSIM_E_INVALID, "a vertex dead in the earlier snapshot is alive in the later one"};
    const std::vector<uint32_t> del = flagged_triples(e0, del_flag, arena, s);
    const std::vector<uint32_t> add = flagged_triples(e1, add_flag, arena, s);
    // the vertices that take a type list, and after's type lists
    std::vector<uint32_t> typed;
    for (uint32_t v = n0; v < n1; v++) typed.push_back(v);
    for (uint32_t v = 0; v < n0; v++)
        if (kh[v] == 1) typed.push_back(v);
    std::vector<uint32_t> toff, tids;
    if (!typed.empty()) {
        toff = to_host(g1.type_off, static_cast<size_t>(n1) + 1, s);
        hip_check(hipStreamSynchronize(s), "diff sync");
        tids = to_host(g1.type_ids, toff[n1], s);
        hip_check(hipStreamSynchronize(s), "diff sync");
    }
    uint64_t n_del_v = 0, pool = 0;
    for (uint32_t v = 0; v < n1; v++) n_del_v += kh[v] == 2;
    for (uint32_t v : typed) pool += toff[v + 1] - toff[v];
    const uint64_t n = typed.size() + del.size() / 3 + add.size() / 3 + n_del_v;
    // one host block: the ops, then the pool of type ids they point into
    char* mem = static_cast<char*>(malloc(n * sizeof(bsim_update) + pool * 4 + 8));
    if (!mem) throw std::bad_alloc();
    bsim_update* ops = reinterpret_cast<bsim_update*>(mem);
    uint32_t* tp = reinterpret_cast<uint32_t*>(mem + n * sizeof(bsim_update));
    uint64_t i = 0;
    auto typed_op = [&](uint32_t op, uint32_t v) {
        bsim_update& o = ops[i++];
        memset(&o, 0, sizeof(o));
        o.op = op;
        o.u = v;
        const uint32_t len = toff[v + 1] - toff[v];
        if (len) memcpy(tp, tids.data() + toff[v], static_cast<size_t>(len) * 4);
        o.n_types = len;
        o.types = tp;
        tp += len;
    };
    for (uint32_t v = n0; v < n1; v++) typed_op(BSIM_OP_ADD_V, v);
    for (uint32_t v = 0; v < n0; v++)
        if (kh[v] == 1) typed_op(BSIM_OP_MOD_V, v);
    auto edge_op = [&](uint32_t op, uint32_t u, uint32_t l, uint32_t w) {
        bsim_update& o = ops[i++];
        memset(&o, 0, sizeof(o));
        o.op = op;
        o.u = u;
        o.label = l;
        o.w = w;
    };
    for (size_t j = 0; j < del.size(); j += 3) edge_op(BSIM_OP_DEL_E, del[j], del[j + 1], del[j + 2]);
    for (size_t j = 0; j < add.size(); j += 3) edge_op(BSIM_OP_ADD_E, add[j], add[j + 1], add[j + 2]);
    for (uint32_t v = 0; v < n1; v++)
        if (kh[v] == 2) {
            bsim_update& o = ops[i++];
            memset(&o, 0, sizeof(o));
            o.op = BSIM_OP_DEL_V;
            o.u = v;
        }
    *n_ops = n;
    return ops;
}

}  // namespace
}  // namespace bsim

using namespace bsim;

int bsim_diff_snapshots(bsim_ctx* ctx, const bsim_graph* before, const bsim_graph* after, bsim_update** ops,
                        uint64_t* n_ops) {
    if (ops) *ops = nullptr;
    if (n_ops) *n_ops = 0;
    if (!ctx || !before || !after || !ops || !n_ops) return BSIM_E_INVALID;
    try {
        hip_check(hipSetDevice(ctx->device), "set device");
        *ops = diff_snapshots(ctx, *before, *after, n_ops);
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

void bsim_updates_free(bsim_update* ops) { free(ops); }
