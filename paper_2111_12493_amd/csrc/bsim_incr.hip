// bsim_incr.hip -- incremental summarization (a9): a resident state that keeps
// the graph and every level h^0..h^K in HBM, and update batches that re-hash
// only the vertices a change can reach (Sec. 3.2; Theorem 2 states that the
// result then equals a batch run on the updated graph).
//
// State layout (device): the out-edges as CSR plus a per-edge source array
// (COO order = CSR order), the type lists likewise, a reverse adjacency
// (in-neighbour lists) that may hold stale extra entries, the alive mask and
// the levels.  Vertex ids are stable: deleted vertices keep their id, with
// no edges, no types, hash 0 and no block.
//
// An update batch:
//   1. host: validate the ordered operations and resolve them into the net
//      change of every touched (u, label, w) triple -- "deleted" (some
//      deletion of the triple happened, so its old copies go) and
//      "present" (the triple exists at the end) -- plus the final type set of
//      every touched vertex;
//   2. device: rebuild the CSR (edge-parallel: old edges that survive are
//      moved by a prefix sum, new triples are appended to their row), the
//      type lists and the reverse adjacency;
//   3. device: level 0 recomputes t(v) for the vertices whose types changed;
//      level j recomputes h^j on the frontier F_j = B u in(C_{j-1}), where B
//      holds the vertices whose own inputs changed (types or out-edge set)
//      and C_{j-1} the vertices whose h^{j-1} changed.  Every other vertex
//      keeps h^j: all its inputs are unchanged;
//      A level whose frontier passes the ctx's limits (a share of the
//      vertices or of the out-edges) is recomputed for all vertices, and so
//      is every later one;
//   4. device: the class index of every level (bsim_cindex.hip) follows the
//      vertices whose hash or previous-level class changed, or is rebuilt
//      after a level recomputed in full; then the fixpoint rule and
//      finalize (block ids, sizes, summary edges) as in batch.
#include <algorithm>
#include <chrono>
#include <cstdio>
#include <cstring>
#include <functional>
#include <unordered_map>

#include "bsim_api_internal.h"
#include "bsim_device.h"
#include "bsim_append.h"
#include "bsim_resolve.h"

using namespace bsim;

namespace bsim {
namespace {

constexpr uint32_t kFlagRows = 1u;    // dflag: the out-edge row is rebuilt
constexpr uint32_t kFlagTypes = 2u;   // dflag: the type list is replaced
constexpr uint32_t kSmallDeg = 512;   // frontier vertices handled by one wave
constexpr uint32_t kFrontLanes = 16;   // lanes per frontier vertex of at most this many out-edges
constexpr uint32_t kFrontGroups = 64 / kFrontLanes;
constexpr uint32_t kWaveSlots = 1024; // LDS de-dup slots per wave (>= 2 * kSmallDeg)
constexpr uint32_t kChunkEdges = 4096;  // edges per block of a large frontier vertex
constexpr uint32_t kInChunk = 4096;     // in-list entries per wave of a large changed vertex
constexpr uint32_t kFrontGrid = 2048;   // blocks of the frontier kernels (grid-stride)
// A large frontier vertex of degree d takes a table of next_pow2(2 d) slots
// with 32-bit slot arithmetic, which holds for d <= 2^30.
constexpr uint64_t kMaxStateEdges = 1ull << 30;

// Device counters of one update batch.
constexpr uint32_t kInStripes = 64;     // striped in-degree sums of a level's changed vertices

struct IncCounters {
    uint32_t b_count;      // base frontier list
    uint32_t f_count[2];   // frontier of a level (by parity)
    uint32_t big_count;    // large frontier vertices deferred to chunk blocks
    uint32_t chunk_count;
    uint32_t in_chunk_count;  // chunks of the in-lists of large changed vertices
    uint64_t slot_top;     // scratch table slots handed out
    // sum of the in-degrees of the vertices whose hash changed at a level
    // (by parity, striped by vertex id): bounds the next level's frontier
    uint64_t in_sum[2][kInStripes];
    // sum of the out-degrees of a level's frontier (striped by block): the
    // edges its re-hash reads
    uint64_t out_sum[2][kInStripes];
};

struct BigEntry {
    uint32_t v;
    uint32_t chunk0;
    uint32_t nchunks;
    uint32_t slots;
    uint64_t slot0;
};

__device__ __forceinline__ uint32_t next_pow2_dev(uint32_t x) {
    return x <= 1 ? 1u : 1u << (32 - __clz(static_cast<int>(x - 1)));
}

// Set mark[v] once; the first setter appends v to the list (one atomic on
// the count per block; every thread of the block calls it).
__device__ __forceinline__ void block_mark_append(bool valid, uint32_t v, uint32_t* mark, uint32_t* list,
                                                  uint32_t* count, uint32_t* s_wave) {
    bool first = false;
    if (valid && *reinterpret_cast<volatile uint32_t*>(&mark[v]) == 0) first = atomicOr(&mark[v], 1u) == 0;
    const uint32_t pos = block_reserve(first, count, s_wave);
    if (first) list[pos] = v;
}

// Tag v for this level (valid lanes); the first tagger lists v through the
// wave's appender and adds v's out-degree to the lane's sum `deg`.  All
// lanes of the wave call it together.
__device__ __forceinline__ void tag_push(WaveAppender& ap, uint64_t& deg, bool valid, uint32_t v, uint32_t tag,
                                         uint32_t* mark, const uint32_t* __restrict__ row_off) {
    bool first = false;
    if (valid && *reinterpret_cast<volatile uint32_t*>(&mark[v]) != tag) first = atomicExch(&mark[v], tag) != tag;
    if (first) deg += row_off[v + 1] - row_off[v];
    ap.push(first, v);
}

// The end of a wave's tagging: its buffered list entries, and its out-degree
// sum added to one of the striped counters.
__device__ __forceinline__ void tag_finish(WaveAppender& ap, uint64_t deg, uint64_t* out_sum) {
    ap.flush();
    const uint64_t d = wave_sum_u64(deg);
    if (lane_id() == 0 && d)
        atomicAdd(reinterpret_cast<unsigned long long*>(&out_sum[blockIdx.x & (kInStripes - 1)]),
                  static_cast<unsigned long long>(d));
}

// t(v) of one vertex from its type list (set semantics), as at level 0 of a run.
__device__ uint64_t type_hash(const uint32_t* ids, uint32_t a, uint32_t b, bool untyped) {
    uint64_t sum = 0;
    if (!untyped) {
        for (uint32_t i = a; i < b; i++) {
            const uint32_t tau = ids[i];
            bool dup = false;
            for (uint32_t j = a; j < i && !dup; j++) dup = ids[j] == tau;
            if (!dup) sum += mix64(kCT ^ static_cast<uint64_t>(tau));
        }
    }
    return mix64(kCT + sum);
}

// ---------------------------------------------------------------- staging

__global__ void k_coo_owner(const uint32_t* __restrict__ off, uint32_t n, uint64_t m,
                            uint32_t* __restrict__ own) {
    const uint64_t e = static_cast<uint64_t>(blockIdx.x) * kBlock + threadIdx.x;
    if (e >= m) return;
    uint32_t lo = 0, hi = n;  // largest v with off[v] <= e
    while (hi - lo > 1) {
        const uint32_t mid = (lo + hi) >> 1;
        if (off[mid] <= e) lo = mid; else hi = mid;
    }
    own[e] = lo;
}

__global__ void k_salt_table(uint64_t* salt, uint32_t count) {
    const uint32_t l = blockIdx.x * kBlock + threadIdx.x;
    if (l < count) salt[l] = mix64(kCL + static_cast<uint64_t>(l));
}

__global__ void k_alive_all(uint8_t* alive, const uint8_t* src, uint32_t n) {
    const uint32_t v = blockIdx.x * kBlock + threadIdx.x;
    if (v < n) alive[v] = src ? (src[v] ? 1 : 0) : 1;
}

// Reverse adjacency from keys (target << 32 | source) sorted ascending.
__global__ void k_rev_split(const uint64_t* __restrict__ keys, uint32_t m, uint32_t* __restrict__ own,
                            uint32_t* __restrict__ srcs) {
    const uint32_t i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= m) return;
    own[i] = static_cast<uint32_t>(keys[i] >> 32);
    srcs[i] = static_cast<uint32_t>(keys[i]);
}

// rev_off[w] = first entry whose owner is >= w, for w = 0..n.
__global__ void k_rev_offsets(const uint32_t* __restrict__ own, uint32_t m, uint32_t n,
                              uint32_t* __restrict__ off) {
    const uint32_t i = blockIdx.x * kBlock + threadIdx.x;
    if (i > m) return;
    const uint32_t hi = i < m ? own[i] : n;
    const int64_t lo = i > 0 ? static_cast<int64_t>(own[i - 1]) : -1;
    for (int64_t w = lo + 1; w <= static_cast<int64_t>(hi); w++) off[w] = i;
}

__global__ void k_edge_keys_rev(const uint32_t* __restrict__ src, const uint32_t* __restrict__ tgt,
                                uint32_t m, uint64_t* __restrict__ keys) {
    const uint32_t e = blockIdx.x * kBlock + threadIdx.x;
    if (e < m) keys[e] = (static_cast<uint64_t>(tgt[e]) << 32) | src[e];
}

// ---------------------------------------------------------------- marking

__global__ void k_set_dead(const uint32_t* __restrict__ dead, uint32_t nd, uint8_t* alive) {
    const uint32_t i = blockIdx.x * kBlock + threadIdx.x;
    if (i < nd) alive[dead[i]] = 0;
}

// Explicit change groups: per source u its range of changes; u's row is rebuilt.
__global__ void k_mark_groups(const uint32_t* __restrict__ gsrc, const uint32_t* __restrict__ gbeg,
                              const uint32_t* __restrict__ gend, uint32_t ng, uint32_t* dflag,
                              uint32_t* chg_lo, uint32_t* chg_hi, uint32_t* bmark, uint32_t* blist,
                              IncCounters* cnt) {
    __shared__ uint32_t s_wave[kBlock / 64 + 1];
    const uint32_t i = blockIdx.x * kBlock + threadIdx.x;
    const bool valid = i < ng;
    uint32_t u = 0;
    if (valid) {
        u = gsrc[i];
        atomicOr(&dflag[u], kFlagRows);
        chg_lo[u] = gbeg[i];
        chg_hi[u] = gend[i];
    }
    block_mark_append(valid, u, bmark, blist, &cnt->b_count, s_wave);
}

__global__ void k_clear_groups(const uint32_t* __restrict__ gsrc, uint32_t ng, uint32_t* chg_lo,
                               uint32_t* chg_hi) {
    const uint32_t i = blockIdx.x * kBlock + threadIdx.x;
    if (i < ng) {
        chg_lo[gsrc[i]] = 0;
        chg_hi[gsrc[i]] = 0;
    }
}

// A deleted vertex d: its own row goes, and every in-neighbour's row is
// rebuilt without the edges to d (one wave per deleted vertex).
__global__ void k_mark_dead(const uint32_t* __restrict__ dead, uint32_t nd,
                            const uint32_t* __restrict__ rev_off, const uint32_t* __restrict__ rev_src,
                            uint32_t n_rev, uint32_t* dflag, uint32_t* bmark, uint32_t* blist,
                            IncCounters* cnt) {
    __shared__ uint32_t s_app[kBlock / 64][kAppendBuf];
    const uint32_t lane = lane_id();
    const uint32_t wave = (blockIdx.x * kBlock + threadIdx.x) >> 6;
    if (wave >= nd) return;  // the whole wave
    const uint32_t d = dead[wave];
    if (lane == 0) atomicOr(&dflag[d], kFlagRows);
    if (d >= n_rev) return;  // the whole wave
    WaveAppender ap{s_app[threadIdx.x >> 6], blist, &cnt->b_count, 0};
    const uint32_t a = rev_off[d], b = rev_off[d + 1];
    for (uint32_t j0 = a; j0 < b; j0 += 64) {
        const uint32_t j = j0 + lane;
        const bool valid = j < b;
        bool first = false;
        uint32_t s = 0;
        if (valid) {
            s = rev_src[j];
            if ((*reinterpret_cast<volatile uint32_t*>(&dflag[s]) & kFlagRows) == 0)
                atomicOr(&dflag[s], kFlagRows);
            first = *reinterpret_cast<volatile uint32_t*>(&bmark[s]) == 0 && atomicOr(&bmark[s], 1u) == 0;
        }
        ap.push(first, s);
    }
    ap.flush();
}

// Vertices whose type set changes (new, modified, deleted).
__global__ void k_mark_types(const uint32_t* __restrict__ tl, uint32_t nT, uint32_t* dflag,
                             uint32_t* tidx, uint32_t* bmark, uint32_t* blist, IncCounters* cnt) {
    __shared__ uint32_t s_wave[kBlock / 64 + 1];
    const uint32_t i = blockIdx.x * kBlock + threadIdx.x;
    const bool valid = i < nT;
    uint32_t v = 0;
    if (valid) {
        v = tl[i];
        atomicOr(&dflag[v], kFlagTypes);
        tidx[v] = i + 1;
    }
    block_mark_append(valid, v, bmark, blist, &cnt->b_count, s_wave);
}

__global__ void k_clear_tidx(const uint32_t* __restrict__ tl, uint32_t nT, uint32_t* tidx) {
    const uint32_t i = blockIdx.x * kBlock + threadIdx.x;
    if (i < nT) tidx[tl[i]] = 0;
}

// ---------------------------------------------------------------- out-edge merge

// keep[e] (written to kpos before the scan): does old edge e survive?
template <typename LabT>
__global__ void k_fwd_keep(const uint32_t* __restrict__ src, const uint32_t* __restrict__ tgt,
                           const LabT* __restrict__ lab, uint32_t m, const uint32_t* __restrict__ dflag,
                           const uint8_t* __restrict__ alive, const uint32_t* __restrict__ chg_lo,
                           const uint32_t* __restrict__ chg_hi, const uint32_t* __restrict__ cw,
                           const uint32_t* __restrict__ cl, const uint32_t* __restrict__ cf,
                           uint32_t* __restrict__ exist, uint32_t* __restrict__ keep) {
    const uint32_t e = blockIdx.x * kBlock + threadIdx.x;
    if (e >= m) return;
    const uint32_t v = src[e];
    uint32_t k = 1;
    if (dflag[v] & kFlagRows) {
        const uint32_t w = tgt[e];
        if (!alive[v] || !alive[w]) {
            k = 0;
        } else {
            uint32_t lo = chg_lo[v], hi = chg_hi[v];
            const uint32_t l = static_cast<uint32_t>(lab[e]);
            // changes of v are sorted by (w, l)
            while (lo < hi) {
                const uint32_t mid = (lo + hi) >> 1;
                const uint32_t mw = cw[mid], ml = cl[mid];
                if (mw < w || (mw == w && ml < l)) lo = mid + 1; else hi = mid;
            }
            if (lo < chg_hi[v] && cw[lo] == w && cl[lo] == l) {
                if (cf[lo] & kChgDeleted) k = 0;
                else exist[lo] = 1;
            }
        }
    }
    keep[e] = k;
}

// Is change c appended as a new edge?
__global__ void k_app_flags(const uint32_t* __restrict__ cf, const uint32_t* __restrict__ exist,
                            uint32_t nc, uint32_t* __restrict__ app) {
    const uint32_t c = blockIdx.x * kBlock + threadIdx.x;
    if (c >= nc) return;
    const uint32_t f = cf[c];
    app[c] = ((f & kChgPresent) && ((f & kChgDeleted) || !exist[c])) ? 1u : 0u;
}

__global__ void k_fwd_deg(uint32_t n_new, uint32_t n_old, const uint32_t* __restrict__ off_old,
                          const uint32_t* __restrict__ kpos, const uint32_t* __restrict__ chg_lo,
                          const uint32_t* __restrict__ chg_hi, const uint32_t* __restrict__ apos,
                          uint32_t* __restrict__ kept, uint32_t* __restrict__ deg) {
    const uint32_t v = blockIdx.x * kBlock + threadIdx.x;
    if (v >= n_new) return;
    const uint32_t k = v < n_old ? kpos[off_old[v + 1]] - kpos[off_old[v]] : 0u;
    const uint32_t a = apos[chg_hi[v]] - apos[chg_lo[v]];
    kept[v] = k;
    deg[v] = k + a;
}

template <typename LabT>
__global__ void k_fwd_copy(const uint32_t* __restrict__ src, const uint32_t* __restrict__ tgt,
                           const LabT* __restrict__ lab, uint32_t m, const uint32_t* __restrict__ off_old,
                           const uint32_t* __restrict__ kpos, const uint32_t* __restrict__ off_new,
                           uint32_t* __restrict__ src2, uint32_t* __restrict__ tgt2, LabT* __restrict__ lab2) {
    const uint32_t e = blockIdx.x * kBlock + threadIdx.x;
    if (e >= m) return;
    const uint32_t ke = kpos[e];
    if (kpos[e + 1] == ke) return;
    const uint32_t v = src[e];
    const uint32_t p = off_new[v] + (ke - kpos[off_old[v]]);
    src2[p] = v;
    tgt2[p] = tgt[e];
    lab2[p] = lab[e];
}

template <typename LabT>
__global__ void k_fwd_append(const uint32_t* __restrict__ cu, const uint32_t* __restrict__ cw,
                             const uint32_t* __restrict__ cl, uint32_t nc, const uint32_t* __restrict__ apos,
                             const uint32_t* __restrict__ off_new, const uint32_t* __restrict__ kept,
                             const uint32_t* __restrict__ chg_lo, uint32_t* __restrict__ src2,
                             uint32_t* __restrict__ tgt2, LabT* __restrict__ lab2) {
    const uint32_t c = blockIdx.x * kBlock + threadIdx.x;
    if (c >= nc || apos[c + 1] == apos[c]) return;
    const uint32_t u = cu[c];
    const uint32_t p = off_new[u] + kept[u] + (apos[c] - apos[chg_lo[u]]);
    src2[p] = u;
    tgt2[p] = cw[c];
    lab2[p] = static_cast<LabT>(cl[c]);
}

// ---------------------------------------------------------------- type lists

__global__ void k_typ_keep(const uint32_t* __restrict__ own, uint32_t nt, const uint32_t* __restrict__ dflag,
                           uint32_t* __restrict__ keep) {
    const uint32_t i = blockIdx.x * kBlock + threadIdx.x;
    if (i < nt) keep[i] = (dflag[own[i]] & kFlagTypes) ? 0u : 1u;
}

__global__ void k_typ_deg(uint32_t n_new, uint32_t n_old, const uint32_t* __restrict__ off_old,
                          const uint32_t* __restrict__ kpos, const uint32_t* __restrict__ tidx,
                          const uint32_t* __restrict__ tl_off, uint32_t* __restrict__ deg) {
    const uint32_t v = blockIdx.x * kBlock + threadIdx.x;
    if (v >= n_new) return;
    const uint32_t ti = tidx[v];
    if (ti) deg[v] = tl_off[ti] - tl_off[ti - 1];
    else deg[v] = v < n_old ? kpos[off_old[v + 1]] - kpos[off_old[v]] : 0u;
}

__global__ void k_typ_copy(const uint32_t* __restrict__ own, const uint32_t* __restrict__ ids, uint32_t nt,
                           const uint32_t* __restrict__ off_old, const uint32_t* __restrict__ kpos,
                           const uint32_t* __restrict__ off_new, uint32_t* __restrict__ own2,
                           uint32_t* __restrict__ ids2) {
    const uint32_t i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= nt) return;
    const uint32_t ki = kpos[i];
    if (kpos[i + 1] == ki) return;
    const uint32_t v = own[i];
    const uint32_t p = off_new[v] + (ki - kpos[off_old[v]]);
    own2[p] = v;
    ids2[p] = ids[i];
}

__global__ void k_typ_write(const uint32_t* __restrict__ tl, uint32_t nT, const uint32_t* __restrict__ tl_off,
                            const uint32_t* __restrict__ tl_ids, const uint32_t* __restrict__ off_new,
                            uint32_t* __restrict__ own2, uint32_t* __restrict__ ids2) {
    const uint32_t i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= nT) return;
    const uint32_t v = tl[i];
    const uint32_t p = off_new[v];
    for (uint32_t j = tl_off[i]; j < tl_off[i + 1]; j++) {
        own2[p + j - tl_off[i]] = v;
        ids2[p + j - tl_off[i]] = tl_ids[j];
    }
}

// Level 0 on the vertices whose types changed: C_0 = those whose t changed.
// A changed vertex adds its in-list length to the striped counters, the
// bound on the in-neighbours that level 1's frontier would take in.
__global__ void k_level0(const uint32_t* __restrict__ tl, uint32_t nT, const uint32_t* __restrict__ type_off,
                         const uint32_t* __restrict__ type_ids, const uint8_t* __restrict__ alive,
                         int untyped, uint64_t* __restrict__ t, uint32_t* cflag, uint32_t tag,
                         const uint32_t* __restrict__ rev_off, uint32_t n_rev, uint64_t* in_sum) {
    const uint32_t i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= nT) return;
    const uint32_t v = tl[i];
    const uint64_t tv = alive[v] ? type_hash(type_ids, type_off[v], type_off[v + 1], untyped != 0) : 0;
    if (tv != t[v]) {
        t[v] = tv;
        cflag[v] = tag;
        if (v < n_rev)
            atomicAdd(reinterpret_cast<unsigned long long*>(&in_sum[v & (kInStripes - 1)]),
                      static_cast<unsigned long long>(rev_off[v + 1] - rev_off[v]));
    }
}

// ---------------------------------------------------------------- reverse lists

__global__ void k_rev_deg(uint32_t n_new, uint32_t n_old, const uint32_t* __restrict__ off_old,
                          const uint32_t* __restrict__ r_lo, const uint32_t* __restrict__ r_hi,
                          uint32_t* __restrict__ deg) {
    const uint32_t w = blockIdx.x * kBlock + threadIdx.x;
    if (w >= n_new) return;
    deg[w] = (w < n_old ? off_old[w + 1] - off_old[w] : 0u) + (r_hi[w] - r_lo[w]);
}

__global__ void k_rev_copy(const uint32_t* __restrict__ own, const uint32_t* __restrict__ srcs, uint32_t rm,
                           const uint32_t* __restrict__ off_old, const uint32_t* __restrict__ off_new,
                           uint32_t* __restrict__ own2, uint32_t* __restrict__ srcs2) {
    const uint32_t e = blockIdx.x * kBlock + threadIdx.x;
    if (e >= rm) return;
    const uint32_t w = own[e];
    const uint32_t p = off_new[w] + (e - off_old[w]);
    own2[p] = w;
    srcs2[p] = srcs[e];
}

__global__ void k_rev_append(const uint32_t* __restrict__ rw, const uint32_t* __restrict__ ru, uint32_t nr,
                             uint32_t n_old, const uint32_t* __restrict__ off_old,
                             const uint32_t* __restrict__ off_new, const uint32_t* __restrict__ r_lo,
                             uint32_t* __restrict__ own2, uint32_t* __restrict__ srcs2) {
    const uint32_t c = blockIdx.x * kBlock + threadIdx.x;
    if (c >= nr) return;
    const uint32_t w = rw[c];
    const uint32_t od = w < n_old ? off_old[w + 1] - off_old[w] : 0u;
    const uint32_t p = off_new[w] + od + (c - r_lo[w]);
    own2[p] = w;
    srcs2[p] = ru[c];
}

// ---------------------------------------------------------------- frontier levels

__global__ void k_level_reset(IncCounters* cnt, uint32_t parity) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        cnt->f_count[parity] = 0;
        cnt->big_count = 0;
        cnt->chunk_count = 0;
        cnt->in_chunk_count = 0;
        cnt->slot_top = 0;
    }
    for (uint32_t i = threadIdx.x; i < kInStripes; i += blockDim.x) {
        cnt->in_sum[parity][i] = 0;
        cnt->out_sum[parity][i] = 0;
    }
}

// F_j starts as the base set B.
__global__ void k_front_base(const uint32_t* __restrict__ blist, IncCounters* cnt, uint32_t parity, uint32_t tag,
                             uint32_t* fmark, uint32_t* flist, const uint32_t* __restrict__ row_off) {
    __shared__ uint32_t s_app[kBlock / 64][kAppendBuf];
    WaveAppender ap{s_app[threadIdx.x >> 6], flist, &cnt->f_count[parity], 0};
    uint64_t deg = 0;
    const uint32_t nb = cnt->b_count;
    for (uint32_t i0 = blockIdx.x * kBlock; i0 < nb; i0 += gridDim.x * kBlock) {
        const uint32_t i = i0 + threadIdx.x;
        const bool valid = i < nb;
        tag_push(ap, deg, valid, valid ? blist[i] : 0u, tag, fmark, row_off);
    }
    tag_finish(ap, deg, cnt->out_sum[parity]);
}

// F_j grows by the in-neighbours of C_{j-1}: the vertices of the previous
// list whose change tag is prev_tag (one wave per listed vertex).  The
// in-list of a vertex with more than kInChunk in-neighbours (a changed hub)
// is cut into chunks, listed as (vertex << 32 | chunk) in `chunks` (room for
// chunk_cap), and walked by k_front_inchunks, many waves at once; a wave
// whose chunks find no room walks its list itself, and the slots it took
// within the room hold ~0 (skipped).
__global__ void k_front_innbrs(const uint32_t* __restrict__ prev, const uint32_t* prev_count, uint32_t prev_n,
                               const uint32_t* __restrict__ cflag, uint32_t prev_tag,
                               const uint32_t* __restrict__ rev_off, const uint32_t* __restrict__ rev_src,
                               uint32_t tag, uint32_t* fmark, uint32_t* flist, IncCounters* cnt, uint32_t parity,
                               const uint32_t* __restrict__ row_off, uint64_t* chunks, uint64_t chunk_cap) {
    __shared__ uint32_t s_app[kBlock / 64][kAppendBuf];
    WaveAppender ap{s_app[threadIdx.x >> 6], flist, &cnt->f_count[parity], 0};
    uint64_t deg = 0;
    const uint32_t np = prev_count ? *prev_count : prev_n;
    const uint32_t lane = lane_id();
    const uint32_t waves = gridDim.x * (kBlock / 64);
    for (uint32_t i = (blockIdx.x * kBlock + threadIdx.x) >> 6; i < np; i += waves) {
        const uint32_t w = prev[i];
        if (cflag[w] != prev_tag) continue;
        const uint32_t a = rev_off[w], b = rev_off[w + 1];
        if (b - a > kInChunk) {
            const uint32_t nch = (b - a + kInChunk - 1) / kInChunk;
            uint32_t c0 = 0;
            if (lane == 0) c0 = atomicAdd(&cnt->in_chunk_count, nch);
            c0 = __shfl(c0, 0);
            const bool room = static_cast<uint64_t>(c0) + nch <= chunk_cap;
            for (uint32_t c = lane; c < nch && static_cast<uint64_t>(c0) + c < chunk_cap; c += 64)
                chunks[c0 + c] = room ? (static_cast<uint64_t>(w) << 32 | c) : ~0ull;
            if (room) continue;
        }
        for (uint32_t j0 = a; j0 < b; j0 += 64) {
            const uint32_t j = j0 + lane;
            const bool valid = j < b;
            tag_push(ap, deg, valid, valid ? rev_src[j] : 0u, tag, fmark, row_off);
        }
    }
    tag_finish(ap, deg, cnt->out_sum[parity]);
}

// The chunks that k_front_innbrs listed: one wave per chunk of kInChunk
// in-list entries.
__global__ void k_front_inchunks(const uint64_t* __restrict__ chunks, uint64_t chunk_cap,
                                 const uint32_t* __restrict__ rev_off, const uint32_t* __restrict__ rev_src,
                                 uint32_t tag, uint32_t* fmark, uint32_t* flist, IncCounters* cnt, uint32_t parity,
                                 const uint32_t* __restrict__ row_off) {
    __shared__ uint32_t s_app[kBlock / 64][kAppendBuf];
    WaveAppender ap{s_app[threadIdx.x >> 6], flist, &cnt->f_count[parity], 0};
    uint64_t deg = 0;
    const uint32_t nc = static_cast<uint32_t>(min(static_cast<uint64_t>(cnt->in_chunk_count), chunk_cap));
    const uint32_t lane = lane_id();
    const uint32_t waves = gridDim.x * (kBlock / 64);
    for (uint32_t i = (blockIdx.x * kBlock + threadIdx.x) >> 6; i < nc; i += waves) {
        const uint64_t item = chunks[i];
        if (item == ~0ull) continue;
        const uint32_t w = static_cast<uint32_t>(item >> 32);
        const uint32_t a = rev_off[w] + static_cast<uint32_t>(item) * kInChunk;
        const uint32_t b = min(rev_off[w + 1], a + kInChunk);
        for (uint32_t j0 = a; j0 < b; j0 += 64) {
            const uint32_t j = j0 + lane;
            const bool valid = j < b;
            tag_push(ap, deg, valid, valid ? rev_src[j] : 0u, tag, fmark, row_off);
        }
    }
    tag_finish(ap, deg, cnt->out_sum[parity]);
}

struct FrontArgs {
    const uint32_t* row_off;
    const uint32_t* tgt;
    const void* lab;
    const uint64_t* t;
    const uint64_t* salt;
    const uint64_t* h_prev;
    uint64_t* h_cur;
    const uint8_t* alive;
    const uint32_t* flist;
    const uint32_t* f_count;
    uint32_t* cflag;
    uint32_t tag;
    IncCounters* cnt;
    BigEntry* big;
    uint32_t* chunk_owner;
    uint64_t* big_acc;
    uint32_t* big_done;
    uint64_t* scratch;
    const uint32_t* rev_off;  // in-neighbour list offsets
    uint32_t n_rev;
    uint64_t* in_sum;         // kInStripes counters of this level
};

// Store h^j(v); a changed value tags v for the next level's frontier.
// Returns v's in-degree when the value changed (the caller adds it to the
// bound on that frontier), else 0.
__device__ __forceinline__ uint64_t publish(const FrontArgs& a, uint32_t v, uint64_t h) {
    if (a.h_cur[v] != h) {
        a.h_cur[v] = h;
        a.cflag[v] = a.tag;
        if (v < a.n_rev) return a.rev_off[v + 1] - a.rev_off[v];
    }
    return 0;
}

__device__ __forceinline__ void add_in_sum(const FrontArgs& a, uint64_t x) {
    if (x) atomicAdd(reinterpret_cast<unsigned long long*>(&a.in_sum[blockIdx.x & (kInStripes - 1)]),
                     static_cast<unsigned long long>(x));
}

__device__ __forceinline__ uint64_t shfl_u64(uint64_t x, uint32_t src) {
    const uint32_t lo = static_cast<uint32_t>(__shfl(static_cast<int>(static_cast<uint32_t>(x)), static_cast<int>(src), 64));
    const uint32_t hi = static_cast<uint32_t>(__shfl(static_cast<int>(static_cast<uint32_t>(x >> 32)), static_cast<int>(src), 64));
    return (static_cast<uint64_t>(hi) << 32) | lo;
}

// h^j of one alive frontier vertex with the whole wave: its pair keys
// de-duplicated in the wave's LDS region (degree <= kSmallDeg), or the
// vertex deferred to the chunk blocks with a global table (larger).  All
// lanes of the wave call it with the same v.
template <typename LabT>
__device__ void front_vertex_wave(const FrontArgs& a, const LabT* __restrict__ lab, volatile uint64_t* tab,
                                  uint32_t v, uint32_t lane, uint64_t& ins) {
    const uint32_t e0 = a.row_off[v], deg = a.row_off[v + 1] - e0;
    if (deg > kSmallDeg) {
        if (lane == 0) {
            const uint32_t nch = (deg + kChunkEdges - 1) / kChunkEdges;
            const uint32_t slots = next_pow2_dev(2 * deg);
            const uint32_t bi = atomicAdd(&a.cnt->big_count, 1u);
            const uint32_t c0 = atomicAdd(&a.cnt->chunk_count, nch);
            const uint64_t s0 = atomicAdd(reinterpret_cast<unsigned long long*>(&a.cnt->slot_top),
                                          static_cast<unsigned long long>(slots));
            a.big[bi] = BigEntry{v, c0, nch, slots, s0};
            a.big_acc[bi] = 0;
            a.big_done[bi] = 0;
            for (uint32_t c = 0; c < nch; c++) a.chunk_owner[c0 + c] = bi;
        }
        return;
    }
    const uint32_t slots = max(64u, next_pow2_dev(2 * deg));
    for (uint32_t j = lane; j < slots; j += 64) tab[j] = 0;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    uint64_t acc = 0;
    for (uint32_t j = lane; j < deg; j += 64) {
        const uint32_t w = a.tgt[e0 + j];
        const uint32_t l = static_cast<uint32_t>(lab[e0 + j]);
        const uint64_t f = mix64((a.h_prev[w] ^ a.salt[l]) ^ kCE);
        if (f != 0 && lds_insert(const_cast<uint64_t*>(tab), static_cast<uint32_t>(f) & (slots - 1), 0, slots, f))
            acc += f;
    }
    acc = wave_sum_u64(acc);
    if (lane == 0) ins += publish(a, v, mix64(a.t[v] ^ mix64(kCS + acc)));
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// h^j of every frontier vertex.  A wave takes kFrontGroups consecutive
// frontier vertices at a time, kFrontLanes lanes each: a dead vertex, or
// one of at most kFrontLanes out-edges, is done by its lane group alone
// (one edge per lane, its keys de-duplicated by comparing every lane with
// the earlier lanes of its group, the distinct keys summed across the
// group).  The others then take the whole wave one after another
// (front_vertex_wave).
template <typename LabT>
__global__ void __launch_bounds__(kBlock) k_front_hash(FrontArgs a) {
    __shared__ uint64_t s_tab[kBlock / 64][kWaveSlots];
    const uint32_t lane = lane_id(), wid = threadIdx.x >> 6;
    volatile uint64_t* tab = s_tab[wid];
    const uint32_t nf = *a.f_count;
    const uint32_t waves = gridDim.x * (kBlock / 64);
    const LabT* __restrict__ lab = static_cast<const LabT*>(a.lab);
    const uint32_t j = lane % kFrontLanes, gbase = lane - j;
    uint64_t ins = 0;  // in-degrees of the vertices whose hash changed
    for (uint32_t i0 = ((blockIdx.x * kBlock + threadIdx.x) >> 6) * kFrontGroups; i0 < nf;
         i0 += waves * kFrontGroups) {
        const uint32_t i = i0 + lane / kFrontLanes;
        const bool valid = i < nf;
        const uint32_t v = valid ? a.flist[i] : 0u;
        const bool live = valid && a.alive[v] != 0;
        uint32_t e0 = 0, deg = 0;
        if (live) {
            e0 = a.row_off[v];
            deg = a.row_off[v + 1] - e0;
        }
        const bool small = valid && deg <= kFrontLanes;
        uint64_t f = 0;
        if (small && j < deg) {
            const uint32_t w = a.tgt[e0 + j];
            const uint32_t l = static_cast<uint32_t>(lab[e0 + j]);
            f = mix64((a.h_prev[w] ^ a.salt[l]) ^ kCE);
        }
        // a key counts at the first lane of its group that holds it (a key
        // of 0 adds nothing either way)
        bool dup = false;
#pragma unroll
        for (uint32_t t = 0; t < kFrontLanes; t++) {
            const uint64_t o = shfl_u64(f, gbase + t);
            dup |= t < j && o == f;
        }
        uint64_t acc = dup ? 0ull : f;
#pragma unroll
        for (int d = 1; d < static_cast<int>(kFrontLanes); d <<= 1) acc += shfl_xor_u64(acc, d);
        if (small && j == 0) ins += publish(a, v, live ? mix64(a.t[v] ^ mix64(kCS + acc)) : 0ull);
        uint64_t rest = __ballot(j == 0 && valid && !small);
        while (rest) {
            const uint32_t src = static_cast<uint32_t>(__ffsll(static_cast<long long>(rest)) - 1);
            rest &= rest - 1;
            const uint32_t vb = static_cast<uint32_t>(__shfl(static_cast<int>(v), static_cast<int>(src), 64));
            front_vertex_wave<LabT>(a, lab, tab, vb, lane, ins);
        }
    }
    ins = wave_sum_u64(ins);
    if (lane == 0) add_in_sum(a, ins);
}

__global__ void k_big_clear(IncCounters* cnt, uint64_t* scratch) {
    const uint64_t top = cnt->slot_top;
    for (uint64_t j = static_cast<uint64_t>(blockIdx.x) * kBlock + threadIdx.x; j < top;
         j += static_cast<uint64_t>(gridDim.x) * kBlock)
        scratch[j] = 0;
}

template <typename LabT>
__global__ void __launch_bounds__(kBlock) k_big_chunks(FrontArgs a) {
    __shared__ uint64_t s_red[kBlock / 64];
    __shared__ uint32_t s_last;
    const uint32_t nch = a.cnt->chunk_count;
    const LabT* __restrict__ lab = static_cast<const LabT*>(a.lab);
    for (uint32_t c = blockIdx.x; c < nch; c += gridDim.x) {
        const uint32_t bi = a.chunk_owner[c];
        const BigEntry be = a.big[bi];
        const uint32_t v = be.v;
        const uint32_t vb = a.row_off[v], ve = a.row_off[v + 1];
        const uint32_t e0 = vb + (c - be.chunk0) * kChunkEdges;
        const uint32_t e1 = min(ve, e0 + kChunkEdges);
        uint64_t* tab = a.scratch + be.slot0;
        const uint32_t mask = be.slots - 1;
        uint64_t acc = 0;
        for (uint32_t e = e0 + threadIdx.x; e < e1; e += kBlock) {
            const uint32_t w = a.tgt[e];
            const uint32_t l = static_cast<uint32_t>(lab[e]);
            const uint64_t f = mix64((a.h_prev[w] ^ a.salt[l]) ^ kCE);
            if (f == 0) continue;
            uint32_t slot = static_cast<uint32_t>(f) & mask;
            for (;;) {
                uint64_t cur = *reinterpret_cast<volatile uint64_t*>(&tab[slot]);
                if (cur == f) break;
                if (cur == 0) {
                    cur = atomicCAS(reinterpret_cast<unsigned long long*>(&tab[slot]), 0ull,
                                    static_cast<unsigned long long>(f));
                    if (cur == 0) {
                        acc += f;
                        break;
                    }
                    if (cur == f) break;
                }
                slot = (slot + 1) & mask;
            }
        }
        const uint64_t sum = block_sum_u64(acc, s_red);
        if (threadIdx.x == 0) {
            atomicAdd(reinterpret_cast<unsigned long long*>(&a.big_acc[bi]), static_cast<unsigned long long>(sum));
            __threadfence();
            s_last = atomicAdd(&a.big_done[bi], 1u) == be.nchunks - 1 ? 1u : 0u;
            if (s_last) {
                __threadfence();
                const uint64_t total = atomicAdd(reinterpret_cast<unsigned long long*>(&a.big_acc[bi]), 0ull);
                add_in_sum(a, publish(a, v, mix64(a.t[v] ^ mix64(kCS + total))));
            }
        }
        __syncthreads();
    }
}

}  // namespace
}  // namespace bsim

// ======================================================================== host

namespace bsim {
namespace {

// A device array owned by a resident state; grows by copying.
template <typename T>
struct DevBuf {
    T* p = nullptr;
    size_t cap = 0;
    void ensure(size_t n, size_t keep, hipStream_t s) {
        if (p && n <= cap) return;
        // headroom, so that the small growth of most batches allocates nothing
        const size_t nc = std::max<size_t>({n + n / 8, cap + cap / 2, 64});
        T* q = nullptr;
        if (device_alloc(reinterpret_cast<void**>(&q), nc * sizeof(T), s) != hipSuccess)
            throw DeviceError{BSIM_E_NOMEM, "state allocation of " + std::to_string(nc * sizeof(T)) + " bytes failed"};
        if (p && keep)
            hip_check(hipMemcpyAsync(q, p, std::min(keep, cap) * sizeof(T), hipMemcpyDeviceToDevice, s), "state grow");
        if (p) (void)hipFreeAsync(p, s);
        p = q;
        cap = nc;
    }
    void release(hipStream_t s) {
        if (p) (void)hipFreeAsync(p, s);
        p = nullptr;
        cap = 0;
    }
};

template <typename T>
T* upload(Arena& arena, const std::vector<T>& v, hipStream_t s) {
    T* d = arena.alloc<T>(v.size() + 1);
    if (!v.empty()) hip_check(hipMemcpyAsync(d, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, s), "upload");
    return d;
}

inline uint32_t grid_for(uint64_t n) { return std::max<uint32_t>(ceil_div(n, kBlock), 1); }


}  // namespace
}  // namespace bsim

struct bsim_state {
    bsim_ctx* ctx = nullptr;
    hipStream_t s = nullptr;
    uint32_t K = 0, flags = 0, label_bytes = 4;
    bool untyped = false;
    uint32_t n = 0, n_rev = 0;
    uint64_t m = 0, nt = 0, rm = 0;
    uint32_t max_label = 0;
    int cur = 0, tcur = 0, rcur = 0;
    DevBuf<uint32_t> row_off[2], src[2], tgt[2];
    DevBuf<uint8_t> lab[2];
    DevBuf<uint32_t> type_off[2], type_own[2], type_ids[2];
    DevBuf<uint32_t> rev_off[2], rev_own[2], rev_src[2];
    DevBuf<uint8_t> alive;
    std::vector<DevBuf<uint64_t>> levels;
    DevBuf<uint64_t> salt;
    DevBuf<uint32_t> dflag, bmark, fmark, chg_lo, chg_hi, tidx, kept, deg, blist, flist[2], cflag;
    uint32_t tag_base = 0;  // change / frontier tags of the next batch start above this
    // class index (bsim_cindex.hip), one per level: tables of ci_cap slots,
    // the class slot of every vertex; per level the counters (classes,
    // claimed slots); the vertex list of an update and the lists of the
    // vertices whose class changed (by level parity), with their counts
    std::vector<DevBuf<uint64_t>> ci_slot;
    std::vector<DevBuf<uint32_t>> ci_cnt, ci_cid;
    uint64_t ci_cap = 0;
    DevBuf<uint64_t> ci_ctr;
    DevBuf<uint32_t> ci_dmark, ci_d, ci_q[2], ci_n;  // ci_n: lengths of ci_d, ci_q[0], ci_q[1]
    uint32_t ci_rebuild_from = 0;  // levels from this one on are rebuilt at the next update (> K: none)
    DevBuf<uint32_t> kpos, chunk_owner, big_done;
    DevBuf<BigEntry> big;
    DevBuf<uint64_t> big_acc, scratch;
    DevBuf<IncCounters> cnt;
    DevBuf<RunStatus> status;
    std::vector<uint8_t> alive_host;
    std::vector<uint32_t> blocks_per_iter;
    // host scratch of the op resolution, all zero between batches: a
    // touched vertex's state after the batch so far (1 alive, 2 deleted) and
    // 1 + the index of its latest type list
    ResolveScratch rs;  // per-vertex marks of the op resolution
    // class-index rebuilds run on a second stream, each after an event that
    // follows the launches writing its level, so they overlap the next levels
    hipStream_t s2 = nullptr;
    hipEvent_t ev_level = nullptr, ev_classes = nullptr;
    // per level: the member counts of the class index are up to date (a
    // rebuild leaves them to the first update that moves vertices there)
    std::vector<uint8_t> ci_counted;
    // backing of an update's temporary arrays, grown to the largest demand
    // seen: large temporaries then never pass through the stream-ordered
    // pool, which can return freed memory to the driver (tens of ms) and map
    // it again in a later update
    DevBuf<uint8_t> work;
    size_t work_want = 0;

    void release() {
        if (s2) (void)hipStreamSynchronize(s2);
        for (int i = 0; i < 2; i++) {
            row_off[i].release(s), src[i].release(s), tgt[i].release(s), lab[i].release(s);
            type_off[i].release(s), type_own[i].release(s), type_ids[i].release(s);
            rev_off[i].release(s), rev_own[i].release(s), rev_src[i].release(s);
            flist[i].release(s);
        }
        alive.release(s);
        for (auto& l : levels) l.release(s);
        salt.release(s), dflag.release(s), bmark.release(s), fmark.release(s), cflag.release(s);
        chg_lo.release(s), chg_hi.release(s), tidx.release(s), kept.release(s), deg.release(s);
        blist.release(s), kpos.release(s), chunk_owner.release(s);
        big_done.release(s), big.release(s), big_acc.release(s), scratch.release(s), cnt.release(s);
        status.release(s), work.release(s);
        for (auto& b : ci_slot) b.release(s);
        for (auto& b : ci_cnt) b.release(s);
        for (auto& b : ci_cid) b.release(s);
        ci_ctr.release(s), ci_dmark.release(s), ci_d.release(s), ci_q[0].release(s), ci_q[1].release(s);
        ci_n.release(s);
        (void)hipStreamSynchronize(s);
        if (ev_level) (void)hipEventDestroy(ev_level);
        if (ev_classes) (void)hipEventDestroy(ev_classes);
        if (s2) (void)hipStreamDestroy(s2);
        ev_level = nullptr, ev_classes = nullptr, s2 = nullptr;
    }
};

namespace bsim {
namespace {

// Vertex-indexed arrays for n vertices (kept contents: the first n_keep).
void ensure_vertices(bsim_state* st, uint32_t n_new) {
    hipStream_t s = st->s;
    const size_t nv = static_cast<size_t>(n_new) + 1;
    const size_t keep_v = st->n, keep_o = static_cast<size_t>(st->n) + 1;
    st->row_off[st->cur].ensure(nv, keep_o, s);
    st->row_off[st->cur ^ 1].ensure(nv, 0, s);
    st->type_off[st->tcur].ensure(nv, keep_o, s);
    st->type_off[st->tcur ^ 1].ensure(nv, 0, s);
    st->rev_off[st->rcur].ensure(nv, static_cast<size_t>(st->n_rev) + 1, s);
    st->rev_off[st->rcur ^ 1].ensure(nv, 0, s);
    st->alive.ensure(nv, keep_v, s);
    for (auto& l : st->levels) l.ensure(nv, keep_v, s);
    // chg_lo / chg_hi / tidx are zero outside a batch, fmark / cflag hold
    // tags of earlier batches: keep them
    st->chg_lo.ensure(nv, keep_v, s);
    st->chg_hi.ensure(nv, keep_v, s);
    st->tidx.ensure(nv, keep_v, s);
    st->fmark.ensure(nv, keep_v, s);
    st->cflag.ensure(nv, keep_v, s);
    for (DevBuf<uint32_t>* b : {&st->dflag, &st->bmark, &st->kept, &st->deg, &st->blist, &st->flist[0],
                                &st->flist[1], &st->big_done, &st->chunk_owner})
        b->ensure(nv, 0, s);
    st->big.ensure(nv, 0, s);
    st->big_acc.ensure(nv, 0, s);
    // class index: the new vertices have no class and no list mark yet
    const size_t L = static_cast<size_t>(st->K) + 1;
    st->ci_slot.resize(L), st->ci_cnt.resize(L), st->ci_cid.resize(L);
    st->ci_counted.resize(L, 0);
    for (auto& c : st->ci_cid) {
        c.ensure(nv, keep_v, s);
        hip_check(hipMemsetAsync(c.p + keep_v, 0xFF, (nv - keep_v) * 4, s), "new classes");
    }
    st->ci_dmark.ensure(nv, keep_v, s);
    hip_check(hipMemsetAsync(st->ci_dmark.p + keep_v, 0, (nv - keep_v) * 4, s), "new list marks");
    for (DevBuf<uint32_t>* b : {&st->ci_d, &st->ci_q[0], &st->ci_q[1]}) b->ensure(nv, 0, s);
    st->ci_n.ensure(4, 0, s);
    st->ci_ctr.ensure(2 * L, 2 * L, s);
    // a table holds the classes of n vertices at load <= 2/3 and the slots
    // that later batches claim; a larger one starts over
    const uint64_t want = split_table_slots(static_cast<uint64_t>(n_new));
    if (want > st->ci_cap) {
        for (size_t j = 0; j < L; j++) {
            st->ci_slot[j].ensure(2 * want, 0, s);
            st->ci_cnt[j].ensure(want, 0, s);
        }
        st->ci_cap = want;
        st->ci_rebuild_from = 0;
    }
}

void ensure_salt(bsim_state* st, uint32_t max_label) {
    if (st->salt.p && max_label < st->salt.cap) return;
    const uint64_t count = next_pow2(static_cast<uint64_t>(max_label) + 1);  // labels < 2^24
    st->salt.ensure(count, 0, st->s);
    k_salt_table<<<grid_for(st->salt.cap), kBlock, 0, st->s>>>(st->salt.p, static_cast<uint32_t>(st->salt.cap));
    hip_check(hipGetLastError(), "salt launch");
}

uint32_t read_u32(const uint32_t* dev, hipStream_t s) {
    uint32_t v = 0;
    hip_check(hipMemcpyAsync(&v, dev, 4, hipMemcpyDeviceToHost, s), "read count");
    hip_check(hipStreamSynchronize(s), "read count sync");
    return v;
}

// Reverse lists from the current out-edges (sorted by target, then source).
void rebuild_reverse(bsim_state* st, Arena& arena) {
    hipStream_t s = st->s;
    const uint32_t n = st->n, m = static_cast<uint32_t>(st->m);
    const int r = st->rcur;
    st->rev_own[r].ensure(std::max<uint64_t>(m, 1), 0, s);
    st->rev_src[r].ensure(std::max<uint64_t>(m, 1), 0, s);
    st->rev_own[r ^ 1].ensure(std::max<uint64_t>(m, 1), 0, s);
    st->rev_src[r ^ 1].ensure(std::max<uint64_t>(m, 1), 0, s);
    st->rev_off[r].ensure(static_cast<size_t>(n) + 1, 0, s);
    if (m) {
        uint64_t* ka = arena.alloc<uint64_t>(m);
        uint64_t* kb = arena.alloc<uint64_t>(m);
        k_edge_keys_rev<<<grid_for(m), kBlock, 0, s>>>(st->src[st->cur].p, st->tgt[st->cur].p, m, ka);
        uint64_t* sorted = radix_sort(ka, kb, m, 32 + std::max(1, bit_width(n)), arena, s);
        k_rev_split<<<grid_for(m), kBlock, 0, s>>>(sorted, m, st->rev_own[r].p, st->rev_src[r].p);
    }
    k_rev_offsets<<<grid_for(static_cast<uint64_t>(m) + 1), kBlock, 0, s>>>(st->rev_own[r].p, m, n,
                                                                            st->rev_off[r].p);
    hip_check(hipGetLastError(), "reverse build");
    st->rm = m;
    st->n_rev = n;
}


__global__ void k_set_ranges(const uint32_t* __restrict__ gk, const uint32_t* __restrict__ gb,
                             const uint32_t* __restrict__ ge, uint32_t ng, uint32_t* lo, uint32_t* hi) {
    const uint32_t i = blockIdx.x * kBlock + threadIdx.x;
    if (i < ng) {
        lo[gk[i]] = gb[i];
        hi[gk[i]] = ge[i];
    }
}

template <typename LabT>
void merge_edges(bsim_state* st, const HostBatch& hb, uint32_t n_old, Arena& arena) {
    hipStream_t s = st->s;
    const uint32_t n_new = hb.n_new;
    const uint32_t m_old = static_cast<uint32_t>(st->m);
    const uint32_t nc = static_cast<uint32_t>(hb.cu.size());
    const int c = st->cur;
    const uint64_t m_cap = static_cast<uint64_t>(m_old) + hb.n_present;
    if (m_cap > kMaxStateEdges)
        throw DeviceError{BSIM_E_UNSUPPORTED, "a resident state holds at most 2^30 edges"};
    st->src[c ^ 1].ensure(m_cap + 1, 0, s);
    st->tgt[c ^ 1].ensure(m_cap + 1, 0, s);
    st->lab[c ^ 1].ensure((m_cap + 1) * sizeof(LabT), 0, s);
    st->kpos.ensure(std::max<uint64_t>(m_old, st->nt) + 1, 0, s);
    uint32_t* d_cu = upload(arena, hb.cu, s);
    uint32_t* d_cw = upload(arena, hb.cw, s);
    uint32_t* d_cl = upload(arena, hb.cl, s);
    uint32_t* d_cf = upload(arena, hb.cf, s);
    uint32_t* exist = arena.alloc<uint32_t>(nc + 1);
    uint32_t* apos = arena.alloc<uint32_t>(nc + 1);
    hip_check(hipMemsetAsync(exist, 0, (nc + 1) * 4ull, s), "exist");
    hip_check(hipMemsetAsync(apos, 0, (nc + 1) * 4ull, s), "apos");
    uint32_t* kpos = st->kpos.p;
    const LabT* lab = reinterpret_cast<const LabT*>(st->lab[c].p);
    hip_check(hipMemsetAsync(kpos, 0, (m_old + 1) * 4ull, s), "kpos");
    if (m_old) {
        k_fwd_keep<LabT><<<grid_for(m_old), kBlock, 0, s>>>(st->src[c].p, st->tgt[c].p, lab, m_old, st->dflag.p,
                                                          st->alive.p, st->chg_lo.p, st->chg_hi.p, d_cw, d_cl,
                                                          d_cf, exist, kpos);
        scan_exclusive(kpos, kpos, m_old, kpos + m_old, arena, s);
    }
    if (nc) {
        k_app_flags<<<grid_for(nc), kBlock, 0, s>>>(d_cf, exist, nc, apos);
        scan_exclusive(apos, apos, nc, apos + nc, arena, s);
    }
    k_fwd_deg<<<grid_for(n_new), kBlock, 0, s>>>(n_new, n_old, st->row_off[c].p, kpos, st->chg_lo.p,
                                                 st->chg_hi.p, apos, st->kept.p, st->deg.p);
    uint32_t* off_new = st->row_off[c ^ 1].p;
    scan_exclusive(st->deg.p, off_new, n_new, off_new + n_new, arena, s);
    const uint32_t m_new = read_u32(off_new + n_new, s);
    if (m_old)
        k_fwd_copy<LabT><<<grid_for(m_old), kBlock, 0, s>>>(st->src[c].p, st->tgt[c].p, lab, m_old,
                                                          st->row_off[c].p, kpos, off_new, st->src[c ^ 1].p,
                                                          st->tgt[c ^ 1].p,
                                                          reinterpret_cast<LabT*>(st->lab[c ^ 1].p));
    if (nc)
        k_fwd_append<LabT><<<grid_for(nc), kBlock, 0, s>>>(d_cu, d_cw, d_cl, nc, apos, off_new, st->kept.p,
                                                         st->chg_lo.p, st->src[c ^ 1].p, st->tgt[c ^ 1].p,
                                                         reinterpret_cast<LabT*>(st->lab[c ^ 1].p));
    hip_check(hipGetLastError(), "edge merge");
    st->cur ^= 1;
    st->m = m_new;
}

void merge_types(bsim_state* st, const HostBatch& hb, uint32_t n_old, Arena& arena) {
    hipStream_t s = st->s;
    const uint32_t n_new = hb.n_new;
    const uint32_t nt_old = static_cast<uint32_t>(st->nt);
    const uint32_t nT = static_cast<uint32_t>(hb.tl.size());
    const int c = st->tcur;
    const uint64_t cap = static_cast<uint64_t>(nt_old) + hb.tl_ids.size();
    if (cap >= (1ull << 32)) throw DeviceError{BSIM_E_UNSUPPORTED, "too many type entries"};
    st->type_own[c ^ 1].ensure(cap + 1, 0, s);
    st->type_ids[c ^ 1].ensure(cap + 1, 0, s);
    st->kpos.ensure(std::max<uint64_t>(st->m, nt_old) + 1, 0, s);
    uint32_t* kpos = st->kpos.p;
    uint32_t* d_tl = upload(arena, hb.tl, s);
    uint32_t* d_off = upload(arena, hb.tl_off, s);
    uint32_t* d_ids = upload(arena, hb.tl_ids, s);
    hip_check(hipMemsetAsync(kpos, 0, (nt_old + 1) * 4ull, s), "kpos");
    if (nt_old) {
        k_typ_keep<<<grid_for(nt_old), kBlock, 0, s>>>(st->type_own[c].p, nt_old, st->dflag.p, kpos);
        scan_exclusive(kpos, kpos, nt_old, kpos + nt_old, arena, s);
    }
    k_typ_deg<<<grid_for(n_new), kBlock, 0, s>>>(n_new, n_old, st->type_off[c].p, kpos, st->tidx.p, d_off,
                                                 st->deg.p);
    uint32_t* off_new = st->type_off[c ^ 1].p;
    scan_exclusive(st->deg.p, off_new, n_new, off_new + n_new, arena, s);
    if (nt_old)
        k_typ_copy<<<grid_for(nt_old), kBlock, 0, s>>>(st->type_own[c].p, st->type_ids[c].p, nt_old,
                                                       st->type_off[c].p, kpos, off_new, st->type_own[c ^ 1].p,
                                                       st->type_ids[c ^ 1].p);
    if (nT)
        k_typ_write<<<grid_for(nT), kBlock, 0, s>>>(d_tl, nT, d_off, d_ids, off_new, st->type_own[c ^ 1].p,
                                                    st->type_ids[c ^ 1].p);
    hip_check(hipGetLastError(), "type merge");
    st->tcur ^= 1;
    st->nt = read_u32(off_new + n_new, s);
}

void merge_reverse(bsim_state* st, const HostBatch& hb, Arena& arena) {
    hipStream_t s = st->s;
    const uint32_t n_new = hb.n_new, n_old = st->n_rev;
    const uint32_t nr = static_cast<uint32_t>(hb.rw.size());
    const uint32_t ng = static_cast<uint32_t>(hb.rgw.size());
    const int c = st->rcur;
    const uint64_t cap = st->rm + nr;
    if (cap >= (1ull << 32)) throw DeviceError{BSIM_E_UNSUPPORTED, "reverse lists too long"};
    st->rev_own[c ^ 1].ensure(cap + 1, 0, s);
    st->rev_src[c ^ 1].ensure(cap + 1, 0, s);
    uint32_t* d_rw = upload(arena, hb.rw, s);
    uint32_t* d_ru = upload(arena, hb.ru, s);
    uint32_t* d_gw = upload(arena, hb.rgw, s);
    uint32_t* d_gb = upload(arena, hb.rgbeg, s);
    uint32_t* d_ge = upload(arena, hb.rgend, s);
    if (ng) k_set_ranges<<<grid_for(ng), kBlock, 0, s>>>(d_gw, d_gb, d_ge, ng, st->chg_lo.p, st->chg_hi.p);
    k_rev_deg<<<grid_for(n_new), kBlock, 0, s>>>(n_new, n_old, st->rev_off[c].p, st->chg_lo.p, st->chg_hi.p,
                                                 st->deg.p);
    uint32_t* off_new = st->rev_off[c ^ 1].p;
    scan_exclusive(st->deg.p, off_new, n_new, off_new + n_new, arena, s);
    if (st->rm)
        k_rev_copy<<<grid_for(st->rm), kBlock, 0, s>>>(st->rev_own[c].p, st->rev_src[c].p,
                                                       static_cast<uint32_t>(st->rm), st->rev_off[c].p, off_new,
                                                       st->rev_own[c ^ 1].p, st->rev_src[c ^ 1].p);
    if (nr)
        k_rev_append<<<grid_for(nr), kBlock, 0, s>>>(d_rw, d_ru, nr, n_old, st->rev_off[c].p, off_new,
                                                     st->chg_lo.p, st->rev_own[c ^ 1].p, st->rev_src[c ^ 1].p);
    if (ng) k_clear_groups<<<grid_for(ng), kBlock, 0, s>>>(d_gw, ng, st->chg_lo.p, st->chg_hi.p);
    hip_check(hipGetLastError(), "reverse merge");
    st->rcur ^= 1;
    st->rm = cap;
    st->n_rev = n_new;
}

// The class passes of an update, level by level as the levels become final.
CiLevel ci_level(bsim_state* st, uint32_t j) {
    CiLevel L;
    L.slot = st->ci_slot[j].p;
    L.cnt = st->ci_cnt[j].p;
    L.cid = st->ci_cid[j].p;
    L.mask = static_cast<uint32_t>(st->ci_cap - 1);
    return L;
}

// Level j's class index from scratch, on the second stream once the
// launches that write h^j (queued on the state's stream) are done, so it
// overlaps the later levels' launches.  Every later level is rebuilt too:
// the class slots of level j are new.
void index_rebuild(bsim_state* st, uint32_t j) {
    st->ci_rebuild_from = std::min(st->ci_rebuild_from, j);
    hip_check(hipEventRecord(st->ev_level, st->s), "level event");
    hip_check(hipStreamWaitEvent(st->s2, st->ev_level, 0), "level wait");
    // the member counts matter only to a later update that moves vertices
    // of this level, and their atomics cost about as much as the rest of
    // the rebuild (and slow the refinement launches beside it): they are
    // counted by the first update that needs them (ci_count), so a level
    // that is recomputed in full again never counts them
    ci_rebuild(ci_level(st, j), st->ci_cap, j ? st->ci_cid[j - 1].p : nullptr, st->levels[j].p, st->alive.p, st->n,
               st->ci_ctr.p + 2 * j, st->s2);
    st->ci_counted[j] = 0;
}

// Level j's class index once h^j is final: rebuilt (from ci_rebuild_from
// on), else updated for the vertices whose h^j changed (candidates of list
// a with flag[v] == tag, or all of a when flag is null) or whose level j-1
// class changed (list b).  The vertices whose level-j class changes are
// listed for level j+1.
void index_level(bsim_state* st, uint32_t j, const uint32_t* a, uint32_t na, const uint32_t* na_dev,
                 const uint32_t* flag, uint32_t tag, const uint32_t* b, uint32_t nb, const uint32_t* nb_dev,
                 Arena& arena) {
    if (j >= st->ci_rebuild_from) {
        index_rebuild(st, j);
        return;
    }
    hipStream_t s = st->s;
    uint32_t* counts = st->ci_n.p;  // [0] the update's list, [1 + parity] the moved lists, [3] errors
    ci_list(a, na, na_dev, flag, tag, b, nb, nb_dev, st->ci_dmark.p, tag, st->ci_d.p, counts, kFrontGrid, s);
    uint32_t* hw = st->ctx->count_host;
    uint64_t used = 0;
    hip_check(hipMemcpyAsync(hw, counts, 4, hipMemcpyDeviceToHost, s), "class list length");
    hip_check(hipMemcpyAsync(&used, st->ci_ctr.p + 2 * j + 1, 8, hipMemcpyDeviceToHost, s), "claimed slots");
    hip_check(hipStreamSynchronize(s), "class list sync");
    const uint32_t nd = *hw;
    // each listed vertex may claim one slot: past 85 % of the table, start over
    if ((used + nd) * 20 > st->ci_cap * 17) {
        index_rebuild(st, j);
        return;
    }
    const CiLevel L = ci_level(st, j);
    if (!st->ci_counted[j]) {
        // the level was rebuilt without its counts (they are cleared); the
        // rebuild stream was joined by the end of the update that rebuilt it
        ci_count(L, st->n, s);
        st->ci_counted[j] = 1;
    }
    ci_update(L, j ? st->ci_cid[j - 1].p : nullptr, st->levels[j].p, st->alive.p, st->ci_d.p, nd,
              st->ci_ctr.p + 2 * j, st->ci_q[j & 1].p, counts + 1 + (j & 1), counts + 3, hw, arena, s);
}

// After the last level: join the rebuild stream; per level the classes and
// the claimed slots.
std::vector<uint64_t> index_end(bsim_state* st) {
    hip_check(hipEventRecord(st->ev_classes, st->s2), "classes event");
    hip_check(hipStreamWaitEvent(st->s, st->ev_classes, 0), "classes wait");
    std::vector<uint64_t> c(2ull * (st->K + 1));
    uint32_t err = 0;
    hip_check(hipMemcpyAsync(c.data(), st->ci_ctr.p, c.size() * 8, hipMemcpyDeviceToHost, st->s), "class counts");
    hip_check(hipMemcpyAsync(&err, st->ci_n.p + 3, 4, hipMemcpyDeviceToHost, st->s), "class index errors");
    hip_check(hipStreamSynchronize(st->s), "class sync");
    if (err) {
        // cannot happen while index_level keeps free slots; rebuild next time
        st->ci_rebuild_from = 0;
        throw DeviceError{BSIM_E_DEVICE, "internal: a class index table ran full"};
    }
    return c;
}

// The most out-edges a frontier level may read before the level is
// recomputed for all vertices (the deferred large vertices' table slots,
// at most 4 per edge, are sized from it).
uint64_t frontier_edge_limit(const bsim_ctx* ctx, uint64_t m) {
    return ctx->frontier_limit_pct ? m * ctx->frontier_edge_pct / 100 + 4096 : 4096;
}

// Levels j0..K for every vertex with the refinement kernels (hash-only
// mode): used when a frontier covers a large share of the graph, and as the
// plain form (full recomputation per update).
void full_levels(bsim_state* st, uint32_t j0, Arena& arena) {
    hipStream_t s = st->s;
    Staged g;
    g.n = st->n;
    g.m = st->m;
    g.label_bytes = st->label_bytes;
    g.row_off = st->row_off[st->cur].p;
    g.tgt = st->tgt[st->cur].p;
    g.lab = st->lab[st->cur].p;
    g.type_off = st->type_off[st->tcur].p;
    g.type_ids = st->type_ids[st->tcur].p;
    g.alive = st->alive.p;
    g.hub_table_slots = st->ctx->hub_table_slots;
    g.max_label = st->max_label;
    g.trusted = true;
    RunStatus* sd = arena.alloc<RunStatus>(1);
    stage_graph(g, sd, &st->ctx->status_host[3], arena, s);
    HashScratch hs;
    alloc_hash_scratch(g, hs, arena, s);
    for (uint32_t j = j0; j <= st->K; j++) {
        launch_hash_level(g, st->levels[0].p, st->levels[j - 1].p, st->levels[j].p, hs, j, s);
        index_rebuild(st, j);
    }
}

// Re-hash levels 1..K on the frontiers of the batch (level 0 already done:
// the vertices of `tl` whose t changed carry tag `tag0` in cflag).  A level
// whose frontier exceeds the ctx's frontier limit, and every level after
// it, is recomputed for all vertices instead.
void propagate(bsim_state* st, const uint32_t* d_tl, uint32_t nT, uint32_t tag0, Arena& arena) {
    hipStream_t s = st->s;
    const uint32_t n = st->n;
    const uint64_t limit = static_cast<uint64_t>(n) * st->ctx->frontier_limit_pct / 100;
    const uint64_t edge_limit = frontier_edge_limit(st->ctx, st->m);
    if (st->ctx->frontier_limit_pct == 0) {
        if (st->K >= 1) full_levels(st, 1, arena);
        return;
    }
    st->chunk_owner.ensure(static_cast<size_t>(n) + st->m / kChunkEdges + 2, 0, s);
    const int lb = st->label_bytes;
    uint32_t fcount = 0;
    for (uint32_t j = 1; j <= st->K; j++) {
        const uint32_t par = j & 1;
        const uint32_t tag = tag0 + j;
        if (st->ctx->frontier_limit_pct < 100) {
            // F_j holds at most B plus the in-neighbours of C_{j-1} (C_0: the
            // type changes): when that bound is far past the limit (a changed
            // hub), the expansion would only confirm that the level goes to
            // the full kernels
            uint64_t in_sum[kInStripes];
            uint32_t nb = 0;
            hip_check(hipMemcpyAsync(in_sum, st->cnt.p->in_sum[par ^ 1], sizeof(in_sum), hipMemcpyDeviceToHost, s),
                      "frontier bound");
            hip_check(hipMemcpyAsync(&nb, &st->cnt.p->b_count, 4, hipMemcpyDeviceToHost, s), "base count");
            hip_check(hipStreamSynchronize(s), "frontier bound sync");
            uint64_t bound = nb;
            for (uint32_t i = 0; i < kInStripes; i++) bound += in_sum[i];
            if (bound > 4 * limit + 1024) {
                full_levels(st, j, arena);
                return;
            }
        }
        k_level_reset<<<1, 64, 0, s>>>(st->cnt.p, par);
        const uint32_t* row_off = st->row_off[st->cur].p;
        k_front_base<<<256, kBlock, 0, s>>>(st->blist.p, st->cnt.p, par, tag, st->fmark.p, st->flist[par].p,
                                            row_off);
        // the scratch table is free until k_front_hash hands out its slots
        uint64_t* in_chunks = st->scratch.p;
        const uint64_t in_cap = st->scratch.cap;
        if (j == 1)
            k_front_innbrs<<<kFrontGrid, kBlock, 0, s>>>(d_tl, nullptr, nT, st->cflag.p, tag0, st->rev_off[st->rcur].p,
                                                         st->rev_src[st->rcur].p, tag, st->fmark.p, st->flist[par].p,
                                                         st->cnt.p, par, row_off, in_chunks, in_cap);
        else
            k_front_innbrs<<<kFrontGrid, kBlock, 0, s>>>(st->flist[par ^ 1].p, &st->cnt.p->f_count[par ^ 1], 0,
                                                         st->cflag.p, tag - 1, st->rev_off[st->rcur].p,
                                                         st->rev_src[st->rcur].p, tag, st->fmark.p, st->flist[par].p,
                                                         st->cnt.p, par, row_off, in_chunks, in_cap);
        k_front_inchunks<<<kFrontGrid, kBlock, 0, s>>>(in_chunks, in_cap, st->rev_off[st->rcur].p,
                                                       st->rev_src[st->rcur].p, tag, st->fmark.p, st->flist[par].p,
                                                       st->cnt.p, par, row_off);
        hip_check(hipGetLastError(), "frontier marks");
        uint64_t out_sum[kInStripes];
        hip_check(hipMemcpyAsync(&fcount, &st->cnt.p->f_count[par], 4, hipMemcpyDeviceToHost, s), "frontier count");
        hip_check(hipMemcpyAsync(out_sum, st->cnt.p->out_sum[par], sizeof(out_sum), hipMemcpyDeviceToHost, s),
                  "frontier edges");
        hip_check(hipStreamSynchronize(s), "frontier sync");
        uint64_t fedges = 0;
        for (uint32_t i = 0; i < kInStripes; i++) fedges += out_sum[i];
        // the frontier kernels read an edge several times slower than the
        // full-level kernels: past 3 x pct % of the edges, a full level is cheaper
        if (fcount > limit || fedges > edge_limit) {
            full_levels(st, j, arena);
            return;
        }
        // the table slots of the deferred (large) frontier vertices:
        // next_pow2(2 deg) <= 4 deg each, so 4 x the frontier's edges
        st->scratch.ensure(4 * fedges + 1024, 0, s);
        FrontArgs a;
        a.row_off = st->row_off[st->cur].p;
        a.tgt = st->tgt[st->cur].p;
        a.lab = st->lab[st->cur].p;
        a.t = st->levels[0].p;
        a.salt = st->salt.p;
        a.h_prev = st->levels[j - 1].p;
        a.h_cur = st->levels[j].p;
        a.alive = st->alive.p;
        a.flist = st->flist[par].p;
        a.f_count = &st->cnt.p->f_count[par];
        a.cflag = st->cflag.p;
        a.tag = tag;
        a.cnt = st->cnt.p;
        a.big = st->big.p;
        a.chunk_owner = st->chunk_owner.p;
        a.big_acc = st->big_acc.p;
        a.big_done = st->big_done.p;
        a.scratch = st->scratch.p;
        a.rev_off = st->rev_off[st->rcur].p;
        a.n_rev = st->n_rev;
        a.in_sum = st->cnt.p->in_sum[par];
        const uint32_t grid =
            std::max<uint32_t>(std::min<uint32_t>(ceil_div(fcount, kBlock / 64 * kFrontGroups), kFrontGrid), 1);
        if (lb == 2) k_front_hash<uint16_t><<<grid, kBlock, 0, s>>>(a);
        else k_front_hash<uint32_t><<<grid, kBlock, 0, s>>>(a);
        k_big_clear<<<256, kBlock, 0, s>>>(st->cnt.p, st->scratch.p);
        if (lb == 2) k_big_chunks<uint16_t><<<512, kBlock, 0, s>>>(a);
        else k_big_chunks<uint32_t><<<512, kBlock, 0, s>>>(a);
        hip_check(hipGetLastError(), "frontier launch");
        const uint32_t qp = (j - 1) & 1;
        index_level(st, j, st->flist[par].p, 0, &st->cnt.p->f_count[par], st->cflag.p, tag, st->ci_q[qp].p, 0,
                    st->ci_n.p + 1 + qp, arena);
    }
}

// Result arrays of an update, allocated before the update changes the state
// (so an allocation failure cannot leave a half-applied batch behind).
struct ResultReserve {
    Arena* keep = nullptr;   // owns the arrays until they go to the result
    FinalOut fo;             // preset output arrays
    uint64_t* hashes = nullptr;
};

// Classes, fixpoint rule and finalize on the current levels.
bsim_result* finish(bsim_state* st, Arena& arena, float* ms_cls, ResultReserve* rr = nullptr) {
    hipStream_t s = st->s;
    const std::vector<uint64_t> c = index_end(st);
    std::vector<uint32_t> nk(st->K + 1);
    for (uint32_t j = 0; j <= st->K; j++) nk[j] = static_cast<uint32_t>(c[2 * j]);
    // the next update rebuilds the tables whose claimed slots passed 70 %
    st->ci_rebuild_from = st->K + 1;
    for (uint32_t j = 0; j <= st->K; j++)
        if (c[2 * j + 1] * 10 > st->ci_cap * 7) {
            st->ci_rebuild_from = j;
            break;
        }
    const bool stop = (st->flags & BSIM_STOP_AT_FIXPOINT) != 0;
    uint32_t k_done = st->K, fix = 0;
    for (uint32_t j = 0; j <= st->K; j++) {
        const uint32_t fx = (j >= 1 && nk[j] == nk[j - 1]) ? 1u : 0u;
        if ((stop && fx) || j >= st->K) {
            k_done = j;
            fix = fx;
            break;
        }
    }
    (void)ms_cls;
    Staged g;
    g.n = st->n;
    g.m = st->m;
    g.label_bytes = st->label_bytes;
    g.row_off = st->row_off[st->cur].p;
    g.tgt = st->tgt[st->cur].p;
    g.lab = st->lab[st->cur].p;
    g.alive = st->alive.p;
    g.src = st->src[st->cur].p;
    g.max_label = st->max_label;
    Arena own_keep(s);
    Arena& keep = rr ? *rr->keep : own_keep;
    FinalOut fo;
    if (rr) fo = rr->fo;
    // the classes of level k_done, named by their slots in that level's table
    finalize(g, st->ci_cid[k_done].p, !(st->flags & BSIM_NO_SUMMARY_EDGES), fo, arena, keep, s, st->ci_cap);
    if (fo.n_blocks != nk[k_done]) throw DeviceError{BSIM_E_DEVICE, "internal: class count mismatch in finalize"};
    LoopResult lr;
    lr.k_done = k_done;
    lr.fixpoint = fix;
    lr.blocks_per_iter.assign(nk.begin(), nk.begin() + k_done + 1);
    return make_result(st->ctx, g, lr, st->levels[k_done].p, fo, keep, st->flags, rr ? rr->hashes : nullptr);
}

// Every device allocation an update batch needs, made before the batch
// changes anything: the state's arrays at their sizes after the batch (the
// merges, the frontier scratch and counters then find them in place), a
// workspace that holds the update's temporaries, and the result's arrays.
// An allocation that fails here throws with the state as it was.
void reserve_batch(bsim_state* st, const HostBatch& hb, ResultReserve& rr) {
    hipStream_t s = st->s;
    const uint32_t n_new = hb.n_new;
    const uint64_t m_cap = st->m + hb.n_present;
    if (m_cap > kMaxStateEdges) throw DeviceError{BSIM_E_UNSUPPORTED, "a resident state holds at most 2^30 edges"};
    const uint64_t nt_cap = st->nt + hb.tl_ids.size();
    if (nt_cap >= (1ull << 32)) throw DeviceError{BSIM_E_UNSUPPORTED, "too many type entries"};
    ensure_vertices(st, n_new);
    if (!hb.gsrc.empty() || !hb.dead.empty()) {
        st->src[st->cur ^ 1].ensure(m_cap + 1, 0, s);
        st->tgt[st->cur ^ 1].ensure(m_cap + 1, 0, s);
        st->lab[st->cur ^ 1].ensure((m_cap + 1) * st->label_bytes, 0, s);
    }
    if (!hb.tl.empty()) {
        st->type_own[st->tcur ^ 1].ensure(nt_cap + 1, 0, s);
        st->type_ids[st->tcur ^ 1].ensure(nt_cap + 1, 0, s);
    }
    st->kpos.ensure(std::max(m_cap, nt_cap) + 1, 0, s);
    if (!hb.rw.empty() || n_new > st->n_rev) {
        const uint64_t cap = st->rm + hb.rw.size();
        if (cap >= (1ull << 32)) throw DeviceError{BSIM_E_UNSUPPORTED, "reverse lists too long"};
        st->rev_own[st->rcur ^ 1].ensure(cap + 1, 0, s);
        st->rev_src[st->rcur ^ 1].ensure(cap + 1, 0, s);
    }
    ensure_salt(st, std::max(st->max_label, hb.max_label));
    st->chunk_owner.ensure(static_cast<size_t>(n_new) + m_cap / kChunkEdges + 2, 0, s);
    st->scratch.ensure(4 * frontier_edge_limit(st->ctx, m_cap) + 1024, 0, s);
    // the workspace: uploads of the batch, merge flags and scans, the
    // staging of full levels, the reverse-list sort and finalize
    const uint64_t items = hb.cu.size() + hb.rw.size() + hb.rgw.size() + hb.tl.size() + hb.tl_ids.size() +
                           hb.dead.size() + 3 * hb.gsrc.size() + hb.tl_off.size();
    const uint64_t bound = 40 * m_cap + 128ull * n_new + 24 * items + (64ull << 20);
    st->work_want = std::max<uint64_t>(st->work_want, bound);
    st->work.ensure(st->work_want, 0, s);
    // the result's arrays
    Arena& keep = *rr.keep;
    rr.fo.preset = true;
    rr.fo.block_ids = keep.alloc<uint32_t>(static_cast<size_t>(n_new) + 1);
    rr.fo.block_sizes = keep.alloc<uint32_t>(static_cast<size_t>(n_new) + 1);
    const uint64_t se = (st->flags & BSIM_NO_SUMMARY_EDGES) ? 1 : m_cap + 1;
    rr.fo.se_src = keep.alloc<uint32_t>(se);
    rr.fo.se_label = keep.alloc<uint32_t>(se);
    rr.fo.se_dst = keep.alloc<uint32_t>(se);
    rr.hashes = keep.alloc<uint64_t>(static_cast<size_t>(n_new) + 1);
}

struct PhaseTimer {
    hipStream_t s;
    hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};
    explicit PhaseTimer(hipStream_t st) : s(st) {
        for (auto& e : ev) hip_check(hipEventCreate(&e), "event");
    }
    ~PhaseTimer() {
        for (auto& e : ev)
            if (e) (void)hipEventDestroy(e);
    }
    void mark(int i) { hip_check(hipEventRecord(ev[i], s), "event"); }
    void fill(bsim_result* r) {
        hip_check(hipEventSynchronize(ev[3]), "event");
        (void)hipEventElapsedTime(&r->ms_stage, ev[0], ev[1]);
        (void)hipEventElapsedTime(&r->ms_iterate, ev[1], ev[2]);
        (void)hipEventElapsedTime(&r->ms_finalize, ev[2], ev[3]);
        (void)hipEventElapsedTime(&r->ms_total, ev[0], ev[3]);
    }
};

bsim_result* apply_batch(bsim_state* st, const HostBatch& hb) {
    hipStream_t s = st->s;
    PhaseTimer tm(s);
    tm.mark(0);
    Arena keep(s);
    ResultReserve rr;
    rr.keep = &keep;
    reserve_batch(st, hb, rr);
    Arena arena(s);
    arena.back(st->work.p, st->work.cap);
    const uint32_t n_old = st->n, n_new = hb.n_new;
    const size_t grow = n_new - n_old;
    if (grow) {
        hip_check(hipMemsetAsync(st->alive.p + n_old, 1, grow, s), "new alive");
        for (auto& l : st->levels) hip_check(hipMemsetAsync(l.p + n_old, 0, grow * 8, s), "new levels");
        // a grown index array holds unset memory past the old vertices
        for (DevBuf<uint32_t>* b : {&st->chg_lo, &st->chg_hi, &st->tidx, &st->fmark, &st->cflag})
            hip_check(hipMemsetAsync(b->p + n_old, 0, (grow + 1) * 4, s), "index and tag arrays");
    }
    hip_check(hipMemsetAsync(st->dflag.p, 0, (static_cast<size_t>(n_new) + 1) * 4, s), "dflag");
    hip_check(hipMemsetAsync(st->bmark.p, 0, (static_cast<size_t>(n_new) + 1) * 4, s), "bmark");
    hip_check(hipMemsetAsync(st->cnt.p, 0, sizeof(IncCounters), s), "counters");
    uint32_t* d_dead = upload(arena, hb.dead, s);
    uint32_t* d_tl = upload(arena, hb.tl, s);
    uint32_t* d_gsrc = upload(arena, hb.gsrc, s);
    uint32_t* d_gbeg = upload(arena, hb.gbeg, s);
    uint32_t* d_gend = upload(arena, hb.gend, s);
    const uint32_t nd = static_cast<uint32_t>(hb.dead.size());
    const uint32_t nT = static_cast<uint32_t>(hb.tl.size());
    const uint32_t ng = static_cast<uint32_t>(hb.gsrc.size());
    if (nd) k_set_dead<<<grid_for(nd), kBlock, 0, s>>>(d_dead, nd, st->alive.p);
    if (ng)
        k_mark_groups<<<grid_for(ng), kBlock, 0, s>>>(d_gsrc, d_gbeg, d_gend, ng, st->dflag.p, st->chg_lo.p,
                                                      st->chg_hi.p, st->bmark.p, st->blist.p, st->cnt.p);
    if (nd)
        k_mark_dead<<<grid_for(64ull * nd), kBlock, 0, s>>>(d_dead, nd, st->rev_off[st->rcur].p,
                                                            st->rev_src[st->rcur].p, st->n_rev, st->dflag.p,
                                                            st->bmark.p, st->blist.p, st->cnt.p);
    if (nT) k_mark_types<<<grid_for(nT), kBlock, 0, s>>>(d_tl, nT, st->dflag.p, st->tidx.p, st->bmark.p,
                                                          st->blist.p, st->cnt.p);
    hip_check(hipGetLastError(), "batch marks");
    if (ng || nd) {
        if (st->label_bytes == 2) merge_edges<uint16_t>(st, hb, n_old, arena);
        else merge_edges<uint32_t>(st, hb, n_old, arena);
    } else if (grow) {
        hip_check(hipMemsetD32Async(reinterpret_cast<hipDeviceptr_t>(st->row_off[st->cur].p + n_old + 1),
                                    static_cast<int>(st->m), grow, s), "new rows");
    }
    if (ng) k_clear_groups<<<grid_for(ng), kBlock, 0, s>>>(d_gsrc, ng, st->chg_lo.p, st->chg_hi.p);
    if (nT) {
        merge_types(st, hb, n_old, arena);
        k_clear_tidx<<<grid_for(nT), kBlock, 0, s>>>(d_tl, nT, st->tidx.p);
    }
    if (!hb.rw.empty() || n_new > st->n_rev) merge_reverse(st, hb, arena);
    st->n = n_new;
    st->max_label = std::max(st->max_label, hb.max_label);
    ensure_salt(st, st->max_label);
    if (st->rm > 2 * st->m + 65536) rebuild_reverse(st, arena);
    tm.mark(1);
    // tags of this batch: tag0 for level 0, tag0 + j for level j
    if (st->tag_base > 0xFFFFFFFFu - 2 * (st->K + 2)) {
        hip_check(hipMemsetAsync(st->fmark.p, 0, st->fmark.cap * 4, s), "tags");
        hip_check(hipMemsetAsync(st->cflag.p, 0, st->cflag.cap * 4, s), "tags");
        hip_check(hipMemsetAsync(st->ci_dmark.p, 0, st->ci_dmark.cap * 4, s), "tags");
        st->tag_base = 0;
    }
    const uint32_t tag0 = st->tag_base + 1;
    st->tag_base += st->K + 2;
    if (nT)
        k_level0<<<grid_for(nT), kBlock, 0, s>>>(d_tl, nT, st->type_off[st->tcur].p, st->type_ids[st->tcur].p,
                                                 st->alive.p, st->untyped ? 1 : 0, st->levels[0].p, st->cflag.p,
                                                 tag0, st->rev_off[st->rcur].p, st->n_rev, st->cnt.p->in_sum[0]);
    hip_check(hipGetLastError(), "level 0");
    hip_check(hipMemsetAsync(st->ci_n.p + 3, 0, 4, s), "class index errors");
    index_level(st, 0, d_tl, nT, nullptr, nullptr, tag0, d_dead, nd, nullptr, arena);
    propagate(st, d_tl, nT, tag0, arena);
    tm.mark(2);
    bsim_result* r = finish(st, arena, nullptr, &rr);
    tm.mark(3);
    tm.fill(r);
    st->work_want = std::max(st->work_want, arena.demand());
    st->alive_host.resize(n_new, 1);
    for (uint32_t d : hb.dead) st->alive_host[d] = 0;
    return r;
}

// A new state from a graph.  Its levels come from the batch refinement, or,
// for a state read back from a checkpoint, from `stored_levels`, which fills
// st->levels[0..K] on the state's stream.
bsim_result* create_state(bsim_ctx* ctx, const bsim_graph& graph, const bsim_params& p, bsim_state* st,
                          const std::function<void(bsim_state*)>* stored_levels = nullptr) {
    if (p.flags & BSIM_PREV_LEVEL_EDGES)
        throw DeviceError{BSIM_E_UNSUPPORTED, "BSIM_PREV_LEVEL_EDGES is supported without a state only"};
    if (graph.n_edges > kMaxStateEdges)
        throw DeviceError{BSIM_E_UNSUPPORTED, "a resident state holds at most 2^30 edges"};
    hipStream_t s = ctx->stream;
    PhaseTimer tm(s);
    tm.mark(0);
    Arena arena(s);
    Staged g;
    upload_graph(graph, g, arena, s);
    g.hub_table_slots = ctx->hub_table_slots;
    RunStatus* stage_status = arena.alloc<RunStatus>(1);
    stage_graph(g, stage_status, &ctx->status_host[3], arena, s);
    st->ctx = ctx;
    st->s = s;
    hip_check(hipStreamCreateWithFlags(&st->s2, hipStreamNonBlocking), "class stream");
    hip_check(hipEventCreateWithFlags(&st->ev_level, hipEventDisableTiming), "level event");
    hip_check(hipEventCreateWithFlags(&st->ev_classes, hipEventDisableTiming), "classes event");
    st->K = p.k_max;
    st->flags = p.flags & ~BSIM_KEEP_LEVELS;
    st->untyped = (p.flags & BSIM_UNTYPED) != 0;
    st->label_bytes = graph.label_bytes;
    st->levels.resize(p.k_max + 1);
    st->status.ensure(1, 0, s);
    st->cnt.ensure(1, 0, s);
    hip_check(hipMemsetAsync(st->status.p, 0, sizeof(RunStatus), s), "status");
    ensure_vertices(st, g.n);
    // chg_lo / chg_hi / tidx are index arrays that every batch reads for all
    // vertices: they start at zero and batches restore the entries they set
    for (DevBuf<uint32_t>* b : {&st->chg_lo, &st->chg_hi, &st->tidx, &st->fmark, &st->cflag})
        hip_check(hipMemsetAsync(b->p, 0, b->cap * 4, s), "index and tag arrays");
    st->n = g.n;
    st->m = g.m;
    st->max_label = g.max_label;
    const uint32_t n = g.n;
    const uint32_t m = static_cast<uint32_t>(g.m);
    const int c = st->cur;
    st->src[c].ensure(m + 1ull, 0, s);
    st->tgt[c].ensure(m + 1ull, 0, s);
    st->lab[c].ensure((m + 1ull) * g.label_bytes, 0, s);
    hip_check(hipMemcpyAsync(st->row_off[c].p, g.row_off, (n + 1ull) * 4, hipMemcpyDeviceToDevice, s), "row_off");
    if (m) {
        hip_check(hipMemcpyAsync(st->tgt[c].p, g.tgt, m * 4ull, hipMemcpyDeviceToDevice, s), "targets");
        hip_check(hipMemcpyAsync(st->lab[c].p, g.lab, static_cast<size_t>(m) * g.label_bytes,
                                 hipMemcpyDeviceToDevice, s), "labels");
        k_coo_owner<<<grid_for(m), kBlock, 0, s>>>(g.row_off, n, m, st->src[c].p);
    }
    const uint32_t nt = read_u32(g.type_off + n, s);
    st->nt = nt;
    st->type_own[st->tcur].ensure(nt + 1ull, 0, s);
    st->type_ids[st->tcur].ensure(nt + 1ull, 0, s);
    hip_check(hipMemcpyAsync(st->type_off[st->tcur].p, g.type_off, (n + 1ull) * 4, hipMemcpyDeviceToDevice, s),
              "type_off");
    if (nt) {
        hip_check(hipMemcpyAsync(st->type_ids[st->tcur].p, g.type_ids, nt * 4ull, hipMemcpyDeviceToDevice, s),
                  "type ids");
        k_coo_owner<<<grid_for(nt), kBlock, 0, s>>>(g.type_off, n, nt, st->type_own[st->tcur].p);
    }
    if (n) k_alive_all<<<grid_for(n), kBlock, 0, s>>>(st->alive.p, g.alive, n);
    hip_check(hipGetLastError(), "state copy");
    st->alive_host.resize(n);
    if (n) hip_check(hipMemcpyAsync(st->alive_host.data(), st->alive.p, n, hipMemcpyDeviceToHost, s), "alive");
    // the op resolution's per-vertex scratch, sized once here (not in the
    // first batch's latency)
    st->rs.vmark.assign(static_cast<size_t>(n) + n / 8 + 1024, 0);
    st->rs.vtype.assign(st->rs.vmark.size(), 0);
    // the frontier scratch up to the frontier edge limit (4 slots per edge),
    // allocated here rather than in an update's latency
    st->scratch.ensure(4 * frontier_edge_limit(ctx, st->m) + 1024, 0, s);
    // the workspace of an update's temporary arrays (the full-level staging
    // and the merges take about 8 B per edge and 8 B per vertex), and the
    // second copies of the CSR and type arrays that the first merges write,
    // allocated here rather than inside an update's latency
    st->work_want = 12 * static_cast<size_t>(st->m) + 16 * static_cast<size_t>(n) + (64u << 20);
    st->work.ensure(st->work_want, 0, s);
    st->src[c ^ 1].ensure(m + 1ull, 0, s);
    st->tgt[c ^ 1].ensure(m + 1ull, 0, s);
    st->lab[c ^ 1].ensure((m + 1ull) * g.label_bytes, 0, s);
    st->kpos.ensure(std::max<uint64_t>(m, nt) + 1, 0, s);
    st->type_own[st->tcur ^ 1].ensure(nt + 1ull, 0, s);
    st->type_ids[st->tcur ^ 1].ensure(nt + 1ull, 0, s);
    st->chunk_owner.ensure(static_cast<size_t>(n) + st->m / kChunkEdges + 2, 0, s);
    ensure_salt(st, st->max_label);
    rebuild_reverse(st, arena);
    tm.mark(1);
    if (stored_levels) {
        (*stored_levels)(st);
    } else {
        // every level h^0..h^K by the batch refinement (no early stop)
        RunBuffers rb;
        alloc_run_buffers(g, p.k_max, false, rb, arena, s);
        LevelSink sink;
        for (auto& l : st->levels) sink.levels.push_back(l.p);
        bsim_params bp{p.k_max, p.flags & ~BSIM_STOP_AT_FIXPOINT};
        run_refinement(ctx, g, bp, rb, &sink, arena);
    }
    tm.mark(2);
    hip_check(hipMemsetAsync(st->ci_n.p, 0, 4 * 4, s), "class list counts");
    for (uint32_t j = 0; j <= st->K; j++) index_rebuild(st, j);
    bsim_result* r = finish(st, arena, nullptr);
    tm.mark(3);
    tm.fill(r);
    return r;
}

}  // namespace

int summarize_with_state(bsim_ctx* ctx, const bsim_graph& graph, const bsim_params& p, bsim_state** state_out,
                         bsim_result** out) {
    validate_params(graph, p);
    if (p.k_max > 4096)
        throw DeviceError{BSIM_E_UNSUPPORTED, "a resident state needs k_max <= 4096 (it keeps every level)"};
    bsim_state* st = new bsim_state();
    try {
        *out = create_state(ctx, graph, p, st);
    } catch (...) {
        st->s = ctx->stream;
        st->release();
        delete st;
        throw;
    }
    *state_out = st;
    return BSIM_OK;
}

uint64_t state_bytes(const bsim_state* st) {
    uint64_t b = 0;
    auto add = [&](const auto& buf) { b += buf.cap * sizeof(*buf.p); };
    for (int i = 0; i < 2; i++) {
        add(st->row_off[i]), add(st->src[i]), add(st->tgt[i]), add(st->lab[i]);
        add(st->type_off[i]), add(st->type_own[i]), add(st->type_ids[i]);
        add(st->rev_off[i]), add(st->rev_own[i]), add(st->rev_src[i]), add(st->flist[i]);
    }
    add(st->alive);
    for (const auto& l : st->levels) add(l);
    add(st->salt), add(st->dflag), add(st->bmark), add(st->fmark), add(st->chg_lo);
    add(st->chg_hi), add(st->tidx), add(st->kept), add(st->deg), add(st->blist), add(st->cflag);
    add(st->kpos), add(st->chunk_owner), add(st->big_done), add(st->big), add(st->big_acc);
    add(st->scratch), add(st->work);
    for (const auto& x : st->ci_slot) add(x);
    for (const auto& x : st->ci_cnt) add(x);
    for (const auto& x : st->ci_cid) add(x);
    add(st->ci_ctr), add(st->ci_dmark), add(st->ci_d), add(st->ci_q[0]), add(st->ci_q[1]), add(st->ci_n);
    return b;
}

bsim_ctx* state_ctx(const bsim_state* st) { return st->ctx; }

// ---------------------------------------------------------------- checkpoint
// A state on file (host byte order, little-endian on this platform): a
// 64-byte header, then row_off (n+1 u32), targets (m u32), labels (m entries
// of label_bytes), type_off (n+1 u32), type ids (nt u32), alive (n bytes) and
// the levels h^0..h^K (n u64 each), back to back.  The header's checksum
// folds every section in that order.  Loading rebuilds the state from the
// graph, with the graph checks of a summarize call, and takes the levels from
// the file instead of refining them again.
namespace {

constexpr char kCkptMagic[8] = {'B', 'S', 'I', 'M', 'S', 'T', 'A', 'T'};
constexpr uint32_t kCkptVersion = 1;

struct CkptHeader {
    char magic[8];
    uint32_t version, k_max, flags, label_bytes, n, reserved0;
    uint64_t m, nt, checksum, reserved1;
};
static_assert(sizeof(CkptHeader) == 64, "checkpoint header layout");

// Fold of 8-byte words, acc <- (acc ^ w) * P, a section's last word padded
// with zero bytes.  For a fixed word each step permutes acc, and for a fixed
// acc it permutes the word, so a change confined to one word always changes
// the result.
struct Fold {
    uint64_t acc = 0x243F6A8885A308D3ull;
    void add(const void* data, size_t bytes) {
        const uint8_t* b = static_cast<const uint8_t*>(data);
        size_t i = 0;
        for (; i + 8 <= bytes; i += 8) {
            uint64_t w;
            memcpy(&w, b + i, 8);
            acc = (acc ^ w) * 0x100000001B3ull;
        }
        if (i < bytes) {
            uint64_t w = 0;
            memcpy(&w, b + i, bytes - i);
            acc = (acc ^ w) * 0x100000001B3ull;
        }
    }
};

struct File {
    FILE* f = nullptr;
    ~File() {
        if (f) fclose(f);
    }
};

template <typename T>
std::vector<T> to_host(const T* dev, size_t count, hipStream_t s) {
    std::vector<T> h(count);
    if (count) {
        hip_check(hipMemcpyAsync(h.data(), dev, count * sizeof(T), hipMemcpyDeviceToHost, s), "checkpoint read");
        hip_check(hipStreamSynchronize(s), "checkpoint read");
    }
    return h;
}

void save_state(const bsim_state* st, const char* path) {
    hipStream_t s = st->s;
    const size_t n = st->n, m = st->m, nt = st->nt;
    CkptHeader hd{};
    memcpy(hd.magic, kCkptMagic, 8);
    hd.version = kCkptVersion;
    hd.k_max = st->K;
    hd.flags = st->flags;
    hd.label_bytes = st->label_bytes;
    hd.n = st->n;
    hd.m = m;
    hd.nt = nt;
    const std::string tmp = std::string(path) + ".tmp";
    File out;
    out.f = fopen(tmp.c_str(), "wb");
    if (!out.f) throw DeviceError{BSIM_E_IO, "cannot open " + tmp + " for writing"};
    bool ok = fwrite(&hd, sizeof(hd), 1, out.f) == 1;
    Fold fold;
    auto put = [&](const void* data, size_t bytes) {
        fold.add(data, bytes);
        if (bytes && ok) ok = fwrite(data, 1, bytes, out.f) == bytes;
    };
    {
        auto v = to_host(st->row_off[st->cur].p, n + 1, s);
        put(v.data(), v.size() * 4);
    }
    {
        auto v = to_host(st->tgt[st->cur].p, m, s);
        put(v.data(), v.size() * 4);
    }
    {
        auto v = to_host(st->lab[st->cur].p, m * st->label_bytes, s);
        put(v.data(), v.size());
    }
    {
        auto v = to_host(st->type_off[st->tcur].p, n + 1, s);
        put(v.data(), v.size() * 4);
    }
    {
        auto v = to_host(st->type_ids[st->tcur].p, nt, s);
        put(v.data(), v.size() * 4);
    }
    {
        auto v = to_host(st->alive.p, n, s);
        put(v.data(), v.size());
    }
    for (const auto& l : st->levels) {
        auto v = to_host(l.p, n, s);
        put(v.data(), v.size() * 8);
    }
    hd.checksum = fold.acc;
    if (ok) ok = fseek(out.f, 0, SEEK_SET) == 0 && fwrite(&hd, sizeof(hd), 1, out.f) == 1;
    ok = (fclose(out.f) == 0) && ok;
    out.f = nullptr;
    if (!ok || rename(tmp.c_str(), path) != 0) {
        remove(tmp.c_str());
        throw DeviceError{BSIM_E_IO, std::string("writing the state to ") + path + " failed"};
    }
}

bsim_result* load_state(bsim_ctx* ctx, const char* path, bsim_state* st) {
    File in;
    in.f = fopen(path, "rb");
    if (!in.f) throw DeviceError{BSIM_E_IO, std::string("cannot open ") + path};
    const DeviceError bad{BSIM_E_INVALID, std::string(path) + " is not a complete state file of this library"};
    CkptHeader hd{};
    if (fread(&hd, sizeof(hd), 1, in.f) != 1 || memcmp(hd.magic, kCkptMagic, 8) != 0) throw bad;
    if (hd.version != kCkptVersion)
        throw DeviceError{BSIM_E_UNSUPPORTED, "state file version " + std::to_string(hd.version)};
    if ((hd.label_bytes != 2 && hd.label_bytes != 4) || hd.n == 0xFFFFFFFFu || hd.m >= (1ull << 32) ||
        hd.nt >= (1ull << 32) || hd.k_max > 4096)
        throw bad;
    const uint64_t n = hd.n, m = hd.m, nt = hd.nt;
    const uint64_t total = sizeof(hd) + 8 * (n + 1) + m * (4 + hd.label_bytes) + 4 * nt + n +
                           8 * n * (hd.k_max + 1ull);
    if (fseeko(in.f, 0, SEEK_END) != 0 || static_cast<uint64_t>(ftello(in.f)) != total ||
        fseeko(in.f, sizeof(hd), SEEK_SET) != 0)
        throw bad;
    Fold fold;
    auto get = [&](void* data, size_t bytes) {
        if (bytes && fread(data, 1, bytes, in.f) != bytes) throw DeviceError{BSIM_E_IO, std::string("reading ") + path};
        fold.add(data, bytes);
    };
    std::vector<uint32_t> row_off(n + 1), tgt(m + 1), type_off(n + 1), type_ids(nt + 1);
    std::vector<uint8_t> lab(m * hd.label_bytes + 4), alive(n + 1);
    get(row_off.data(), (n + 1) * 4);
    get(tgt.data(), m * 4);
    get(lab.data(), m * hd.label_bytes);
    get(type_off.data(), (n + 1) * 4);
    get(type_ids.data(), nt * 4);
    get(alive.data(), n);
    // the staging checks the CSR on the device; the sizes it takes from the
    // last offsets must agree with the arrays read here
    if (row_off[n] != m || type_off[n] != nt) throw bad;
    bsim_graph g{};
    g.n_vertices = hd.n;
    g.label_bytes = hd.label_bytes;
    g.n_edges = m;
    g.row_off = row_off.data();
    g.targets = tgt.data();
    g.labels = lab.data();
    g.type_off = type_off.data();
    g.type_ids = type_ids.data();
    g.alive = alive.data();
    g.mem_kind = BSIM_MEM_HOST;
    const bsim_params p{hd.k_max, hd.flags};
    validate_params(g, p, false);
    const std::function<void(bsim_state*)> fill = [&](bsim_state* fresh) {
        std::vector<uint64_t> h(n + 1);
        for (auto& l : fresh->levels) {
            get(h.data(), n * 8);
            for (uint64_t v = 0; v < n; v++)
                if (!alive[v] && h[v]) throw bad;  // a deleted vertex has hash 0
            if (n) hip_check(hipMemcpyAsync(l.p, h.data(), n * 8, hipMemcpyHostToDevice, fresh->s), "level upload");
            hip_check(hipStreamSynchronize(fresh->s), "level upload");
        }
        if (fold.acc != hd.checksum)
            throw DeviceError{BSIM_E_INVALID, std::string(path) + ": checksum mismatch"};
    };
    return create_state(ctx, g, p, st, &fill);
}

}  // namespace

}  // namespace bsim

extern "C" {

int bsim_apply_updates(bsim_state* st, const bsim_update* ops, uint64_t n_ops, bsim_result** out) {
    if (out) *out = nullptr;
    if (!st || !out || (n_ops && !ops)) return BSIM_E_INVALID;
    try {
        hip_check(hipSetDevice(st->ctx->device), "set device");
        const auto t0 = std::chrono::steady_clock::now();
        const HostBatch& hb = resolve_ops_into(st->rs.hb, st->n, st->label_bytes, st->alive_host, st->rs, ops, n_ops);
        const float ms_resolve = std::chrono::duration<float, std::milli>(std::chrono::steady_clock::now() - t0).count();
        *out = apply_batch(st, hb);
        (*out)->ms_resolve = ms_resolve;
        return BSIM_OK;
    } catch (const DeviceError& e) {
        st->ctx->err = e.msg;
        (void)hipStreamSynchronize(st->s);
        return e.status;
    } catch (const std::bad_alloc&) {
        st->ctx->err = "host allocation failed";
        return BSIM_E_NOMEM;
    }
}

int bsim_state_graph(const bsim_state* st, bsim_graph* g) {
    if (!st || !g) return BSIM_E_INVALID;
    memset(g, 0, sizeof(*g));
    try {
        hip_check(hipSetDevice(st->ctx->device), "set device");
        const size_t n = st->n, m = st->m, nt = st->nt;
        void* a[6] = {malloc((n + 1) * 4), malloc(m * 4 + 4), malloc(m * st->label_bytes + 4),
                      malloc((n + 1) * 4), malloc(nt * 4 + 4), malloc(n + 1)};
        for (void* q : a)
            if (!q) {
                for (void* r : a) free(r);
                return BSIM_E_NOMEM;
            }
        hipStream_t s = st->s;
        hip_check(hipMemcpyAsync(a[0], st->row_off[st->cur].p, (n + 1) * 4, hipMemcpyDeviceToHost, s), "row_off");
        if (m) {
            hip_check(hipMemcpyAsync(a[1], st->tgt[st->cur].p, m * 4, hipMemcpyDeviceToHost, s), "targets");
            hip_check(hipMemcpyAsync(a[2], st->lab[st->cur].p, m * st->label_bytes, hipMemcpyDeviceToHost, s),
                      "labels");
        }
        hip_check(hipMemcpyAsync(a[3], st->type_off[st->tcur].p, (n + 1) * 4, hipMemcpyDeviceToHost, s), "type_off");
        if (nt) hip_check(hipMemcpyAsync(a[4], st->type_ids[st->tcur].p, nt * 4, hipMemcpyDeviceToHost, s), "types");
        if (n) hip_check(hipMemcpyAsync(a[5], st->alive.p, n, hipMemcpyDeviceToHost, s), "alive");
        hip_check(hipStreamSynchronize(s), "state graph");
        g->n_vertices = st->n;
        g->label_bytes = st->label_bytes;
        g->n_edges = st->m;
        g->row_off = static_cast<uint32_t*>(a[0]);
        g->targets = static_cast<uint32_t*>(a[1]);
        g->labels = a[2];
        g->type_off = static_cast<uint32_t*>(a[3]);
        g->type_ids = static_cast<uint32_t*>(a[4]);
        g->alive = static_cast<uint8_t*>(a[5]);
        g->mem_kind = BSIM_MEM_HOST;
        return BSIM_OK;
    } catch (const DeviceError& e) {
        st->ctx->err = e.msg;
        return e.status;
    }
}

int bsim_state_device_graph(const bsim_state* st, bsim_graph* g) {
    if (!st || !g) return BSIM_E_INVALID;
    memset(g, 0, sizeof(*g));
    g->n_vertices = st->n;
    g->label_bytes = st->label_bytes;
    g->n_edges = st->m;
    g->row_off = st->row_off[st->cur].p;
    g->targets = st->tgt[st->cur].p;
    g->labels = st->lab[st->cur].p;
    g->type_off = st->type_off[st->tcur].p;
    g->type_ids = st->type_ids[st->tcur].p;
    g->alive = st->alive.p;
    g->mem_kind = BSIM_MEM_DEVICE;
    return BSIM_OK;
}

int bsim_state_save(const bsim_state* st, const char* path) {
    if (!st || !path) return BSIM_E_INVALID;
    try {
        hip_check(hipSetDevice(st->ctx->device), "set device");
        save_state(st, path);
        return BSIM_OK;
    } catch (const DeviceError& e) {
        st->ctx->err = e.msg;
        return e.status;
    } catch (const std::bad_alloc&) {
        st->ctx->err = "host allocation failed";
        return BSIM_E_NOMEM;
    }
}

int bsim_state_load(bsim_ctx* ctx, const char* path, bsim_state** state_out, bsim_result** out) {
    if (state_out) *state_out = nullptr;
    if (out) *out = nullptr;
    if (!ctx || !path || !state_out || !out) return BSIM_E_INVALID;
    bsim_state* st = nullptr;
    try {
        hip_check(hipSetDevice(ctx->device), "set device");
        st = new bsim_state();
        *out = load_state(ctx, path, st);
        *state_out = st;
        return BSIM_OK;
    } catch (const DeviceError& e) {
        ctx->err = e.msg;
        if (st) {
            st->s = ctx->stream;
            st->release();
            delete st;
        }
        (void)hipStreamSynchronize(ctx->stream);
        return e.status;
    } catch (const std::bad_alloc&) {
        ctx->err = "host allocation failed";
        if (st) {
            st->s = ctx->stream;
            st->release();
            delete st;
        }
        return BSIM_E_NOMEM;
    }
}

void bsim_state_free(bsim_state* st) {
    if (!st) return;
    (void)hipSetDevice(st->ctx->device);
    st->release();
    delete st;
}

}  // extern "C"
