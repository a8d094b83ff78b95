// bsim_iter.hip -- the refinement loop (a2-a7).
//
// Level 0 (k_init) hashes every vertex's type set (Algorithm 4's
// initialization: the ID of the local schema) and groups vertices by it.
// Launch k >= 1 (k_iterate) runs three phases in every block:
//   0. stop test on the class count of level k-2, which is complete once
//      launch k-1 has finished; recycling of counters and of the split table
//      that level k-2 used;
//   1. split test of level k-1 for the block's own vertices: a vertex whose
//      h^{k-1} differs from its representative's joins (or founds) the class
//      (rep, h^{k-1}) in the split table; the number of founded classes is
//      n_{k-1} - n_{k-2};
//   2. h^k: a tile block gathers h^{k-1} of its out-edge targets
//      (SignalMessages), de-duplicates the (label, hash) pair keys of each
//      vertex in a per-vertex open-addressing region of an LDS table
//      (MergeMessages' hash table), sums the mixed distinct keys
//      (the order-independent Hash) and writes h^k; a hub chunk block writes
//      its mixed keys to the hub's scratch area instead.
// Then k_hub de-duplicates each hub's scratch keys bucket by bucket in LDS
// and adds each bucket's distinct sum to the hub's accumulator;
// k_hub_finish turns the sums into h^k.
//
// The stop test lags the hashes by two launches, so once the block count
// stops growing at level j, launch j+1 has computed h^{j+1} that is never
// used and launch j+2 sets the sticky done flag; every later launch returns
// at once, so the host can queue launches ahead.  A launch can also run as
// two (kPhaseSplit, then kPhaseHash): the host reads the classes that the
// split half founded before it decides on the hash half, which lets a run
// that reaches its fixpoint there hash no further level.
#include "bsim_device.h"

namespace bsim {

namespace {

// ------------------------------------------------------------ split table

// Join the class (r, key) of the level's split table, founding it if needed.
// A slot holds the owner word ((r + 1) << 32 | owner) of one class; the
// class key is the owner's own key, keys[owner], read back from the level's
// hash array (written by an earlier launch, read-only here).  Returns the
// owner word and sets *founded when this call created the class.  Slots
// only ever go from empty to filled during a launch, so every caller with
// the same (r, key) walks the same probe sequence and stops at the same
// slot; founding a class is one CAS.
__device__ uint64_t split_join(const SplitTable& T, const uint64_t* __restrict__ keys, uint32_t r, uint64_t key,
                               uint32_t v, uint32_t* founded, uint32_t* slot_out) {
    const uint64_t mine = (static_cast<uint64_t>(r + 1) << 32) | v;  // never 0: r + 1 >= 1
    *founded = 0;
    // the home slot depends on the class r as well as the key: isomorphic
    // vertices of different classes (every batched graph has vertices with
    // the same type set) share keys, and must not share one probe chain
    uint32_t slot = (static_cast<uint32_t>(key) ^
                     static_cast<uint32_t>((static_cast<uint64_t>(r) * 0x9E3779B97F4A7C15ull) >> 32)) & T.mask;
    for (;;) {
        uint64_t* p = &T.slots[slot];
        uint64_t cur = *p;  // a stale 0 only costs the CAS below
        if (cur == 0) {
            cur = atomicCAS(reinterpret_cast<unsigned long long*>(p), 0ull, static_cast<unsigned long long>(mine));
            if (cur == 0) {
                *founded = 1;
                *slot_out = slot;
                return mine;
            }
        }
        if ((cur >> 32) == static_cast<uint64_t>(r + 1) && keys[static_cast<uint32_t>(cur)] == key) {
            *slot_out = slot;
            return cur;
        }
        slot = (slot + 1) & T.mask;
    }
}

// split_join for the participating lanes of a wave, one call per distinct
// (r, key): lanes are grouped by ballots first, so a key shared by many
// vertices (every vertex without out-edges of one type set joins one class)
// reaches the table once per wave.  All lanes of the wave must call it.
// Returns the owner word for participating lanes; *founded / *slot as
// split_join for the group's leader, 0 / 0xFFFFFFFF for the others.
__device__ __forceinline__ uint64_t shfl_u64(uint64_t x, uint32_t src) {
    const int lo = __shfl(static_cast<int>(static_cast<uint32_t>(x)), static_cast<int>(src), 64);
    const int hi = __shfl(static_cast<int>(static_cast<uint32_t>(x >> 32)), static_cast<int>(src), 64);
    return (static_cast<uint64_t>(static_cast<uint32_t>(hi)) << 32) | static_cast<uint32_t>(lo);
}

__device__ uint64_t wave_split_join(const SplitTable& T, const uint64_t* __restrict__ keys, bool participant,
                                    uint32_t r, uint64_t key, uint32_t v, uint32_t* founded, uint32_t* slot_out) {
    const uint32_t lane = lane_id();
    uint32_t leader_of = lane;
    bool pending = participant;
    for (;;) {
        const uint64_t ball = __ballot(pending);
        if (!ball) break;
        const uint32_t leader = static_cast<uint32_t>(__ffsll(static_cast<long long>(ball)) - 1);
        const uint64_t lk = shfl_u64(key, leader);
        const uint32_t lr = static_cast<uint32_t>(__shfl(static_cast<int>(r), static_cast<int>(leader), 64));
        if (pending && key == lk && r == lr) {
            leader_of = leader;
            pending = false;
        }
    }
    *founded = 0;
    *slot_out = 0xFFFFFFFFu;
    uint64_t o = 0;
    if (participant && leader_of == lane) o = split_join(T, keys, r, key, v, founded, slot_out);
    return shfl_u64(o, leader_of);
}

// base[key] += 1 for every taking lane, one atomic per distinct key in the
// wave (a batched run's founders are counted per graph, and a wave's
// vertices mostly belong to one graph).  All lanes of the wave call it.
__device__ void wave_count_by_key(bool take, uint32_t key, uint32_t* base) {
    const uint32_t lane = lane_id();
    bool pending = take;
    for (;;) {
        const uint64_t ball = __ballot(pending);
        if (!ball) break;
        const uint32_t leader = static_cast<uint32_t>(__ffsll(static_cast<long long>(ball)) - 1);
        const uint32_t lk = static_cast<uint32_t>(__shfl(static_cast<int>(key), static_cast<int>(leader), 64));
        const uint64_t same = __ballot(pending && key == lk);
        if (lane == leader) atomicAdd(&base[lk], static_cast<uint32_t>(__popcll(same)));
        if (key == lk) pending = false;
    }
}

// Count the classes founded by this block at `level` (stripe counter) and
// remember their slots so the table can be cleared selectively.
__device__ void record_founders(const SplitTable& T, uint32_t* lcnt, uint32_t level,
                                uint32_t founded, uint32_t slot, uint32_t* s_red, uint32_t* s_base) {
    const uint32_t lane = lane_id(), wid = threadIdx.x >> 6;
    const uint64_t ball = __ballot(founded != 0);
    const uint32_t wcount = static_cast<uint32_t>(__popcll(ball));
    const uint32_t wrank = static_cast<uint32_t>(__popcll(ball & ((1ull << lane) - 1)));
    if (lane == 0) s_red[wid] = wcount;
    __syncthreads();
    uint32_t off = 0, tot = 0;
    for (int w = 0; w < kBlock / 64; w++) {
        if (w < static_cast<int>(wid)) off += s_red[w];
        tot += s_red[w];
    }
    const uint32_t stripe = blockIdx.x & (kStripes - 1);
    if (threadIdx.x == 0)
        *s_base = tot ? atomicAdd(&lcnt[(level & (kStripeRing - 1)) * kStripes + stripe], tot) : 0;
    __syncthreads();
    if (founded) {
        // every counted position is written
        const uint32_t pos = *s_base + off + wrank;
        if (pos < static_cast<uint32_t>(kListPerStripe)) T.list[stripe * kListPerStripe + pos] = slot;
    }
    __syncthreads();
}

// ------------------------------------------------------------ level 0

// t(v) and h^0 = t for every vertex (0 for a dead one).
__global__ void __launch_bounds__(kBlock) k_types(const uint32_t* __restrict__ type_off,
                                                  const uint32_t* __restrict__ type_ids,
                                                  const uint8_t* __restrict__ alive, uint32_t n, int untyped,
                                                  uint64_t* __restrict__ t, uint64_t* __restrict__ h0) {
    const uint32_t v = blockIdx.x * kBlock + threadIdx.x;
    if (v < n) {
        uint64_t tv = 0;
        if (!alive || alive[v]) {
            uint64_t sum = 0;
            if (!untyped) {
                const uint32_t a = type_off[v], b = type_off[v + 1];
                for (uint32_t i = a; i < b; i++) {
                    const uint32_t tau = type_ids[i];
                    bool dup = false;
                    for (uint32_t j = a; j < i && !dup; j++) dup = type_ids[j] == tau;
                    if (!dup) sum += mix64(kCT ^ static_cast<uint64_t>(tau));
                }
            }
            tv = mix64(kCT + sum);
        }
        t[v] = tv;
        h0[v] = tv;
    }
}

// Level-0 classes by t (written by k_types, the launch before): many
// vertices share a type set, so each wave's lanes are grouped by key before
// they touch the table.
__global__ void __launch_bounds__(kBlock) k_init(const uint64_t* __restrict__ t, const uint8_t* __restrict__ alive,
                                                 uint32_t n, uint32_t* __restrict__ rep, SplitTable T,
                                                 uint32_t* lcnt, BatchCtl bc) {
    __shared__ uint32_t s_red[kBlock / 64];
    __shared__ uint32_t s_base;
    const uint32_t v = blockIdx.x * kBlock + threadIdx.x;
    uint32_t founded = 0, slot = 0xFFFFFFFFu;
    uint32_t r = 0xFFFFFFFFu;
    const bool part = v < n && (!alive || alive[v]);
    const uint32_t gi = (part && bc.gid) ? bc.gid[v] : 0u;
    const uint32_t vr = bc.gid ? bc.virt_base + gi : kNoRep;
    uint64_t key = 0;
    if (part) key = t[v];
    const uint64_t o = wave_split_join(T, t, part, vr, key, v, &founded, &slot);
    if (part) r = static_cast<uint32_t>(o);
    if (bc.gid) wave_count_by_key(founded != 0, gi, bc.hist);
    if (v < n) rep[v] = r;
    record_founders(T, lcnt, 0, founded, slot, s_red, &s_base);
}

// ------------------------------------------------------------ launch k

struct IterShared {
    uint64_t tab[kTableSlots];
    uint64_t acc[kTileMaxVerts];
    uint32_t off[kTileMaxVerts + 1];
    uint32_t red[kBlock / 64];
    uint32_t ctl[4];
    alignas(8) uint8_t seg[kTileMaxEdges];
};

static_assert(offsetof(IterShared, red) >= kSoloSlots * sizeof(uint64_t),
              "a solo block's table must end before the block's control words");
static_assert(kTileMaxEdges >= (kBlock / 64) * 8, "a solo block's wave sums live in seg");

// Split test of level k-1 for one owned vertex (h_prev holds h^{k-1}).
__device__ __forceinline__ void split_test(const IterArgs& a, uint32_t v, uint32_t* founded,
                                           uint32_t* slot) {
    *founded = 0;
    *slot = 0xFFFFFFFFu;
    if (a.alive && !a.alive[v]) return;
    if (a.bc.gid && a.k - 1 > a.bc.done_level[a.bc.gid[v]]) return;
    const uint32_t r = a.rep[v];
    if (r == v) return;
    const uint64_t hv = a.h_prev[v];
    if (hv == a.h_prev[r]) return;
    a.rep[v] = static_cast<uint32_t>(split_join(a.test_tab, a.h_prev, r, hv, v, founded, slot));
    if (a.bc.gid && *founded)
        atomicAdd(&a.bc.hist[static_cast<size_t>(a.k - 1) * a.bc.n_graphs + a.bc.gid[v]], 1u);
}

// What launch k does: the split test of level k-1, the hashes h^k, and the
// stop test of level k - stop_lag (its split is complete by then).
__device__ __forceinline__ bool run_test(const IterArgs& a) {
    return !a.hash_only && a.phase != kPhaseHash && a.k >= 2 && a.k - 1 <= a.k_max;
}
__device__ __forceinline__ bool run_hash(const IterArgs& a) { return a.phase != kPhaseSplit && a.k <= a.k_max; }
__device__ __forceinline__ uint32_t stop_lag(const IterArgs& a) { return a.phase == kPhaseHash ? 1u : 2u; }

// The sticky done flag as this wave sees it (only to skip loads; see tile_block).
__device__ __forceinline__ bool early_done(const IterArgs& a) {
    return !a.hash_only && __hip_atomic_load(&a.status->done, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0;
}

// Stop test of level k - stop_lag (wave 0), from the values loaded at block start:
// S.ctl[0] = 1 when the run is done; block 0 also records n_{k-2} and, on
// stopping, the final status.  Visible to the block after its next barrier.
__device__ __forceinline__ void stop_decision(const IterArgs& a, IterShared& S, uint32_t p_done,
                                              uint32_t p_cnt, uint32_t p_tot) {
    const uint32_t tid = threadIdx.x, k = a.k;
    if (tid >= 64) return;
    uint32_t ex = p_done;
    // batched runs: the per-graph stop launch before this one sets done
    const uint32_t lag = stop_lag(a);
    if (!ex && k >= lag && !a.bc.gid && !a.hash_only) {
        const uint32_t lv = k - lag;
        const uint32_t c = wave_sum_u32(p_cnt);
        const uint32_t nl = lv == 0 ? c : p_tot + c;
        if (tid == 0) {
            if (blockIdx.x == 0) a.totals[lv] = nl;
            const uint32_t fix = (lv >= 1 && c == 0) ? 1u : 0u;
            if ((a.stop && fix) || lv >= a.k_max) {
                ex = 1;
                if (blockIdx.x == 0) {
                    a.status->k_done = lv;
                    a.status->fixpoint = fix;
                    a.status->done = 1;
                }
            }
        }
    }
    if (tid == 0) S.ctl[0] = ex;
}

// A tile block.  Its latency is a chain of dependent memory round trips, so
// every load is issued before the first barrier: tile bounds -> offsets and
// per-vertex state -> edge targets / labels and the representative's hash
// -> neighbour hashes.  Nothing is written before the stop decision.
// Returns false when the run is done.
template <typename LabT>
__device__ bool tile_block(const IterArgs& a, uint32_t tile, IterShared& S, uint32_t p_done, uint32_t p_cnt,
                           uint32_t p_tot) {
    const uint32_t tid = threadIdx.x, k = a.k;
    const bool test = run_test(a);
    const bool hash = run_hash(a);
    const uint32_t i0 = a.tile_i0[tile], nv = a.tile_i1[tile] - i0;
    const uint32_t ebase = a.tile_e0[tile];
    // A launch queued after the stop finds the sticky done flag set; every
    // block of it then takes the same stop decision, so its waves may skip
    // their loads at once (the exit itself still follows stop_decision).
    const bool skip = early_done(a);
    const uint32_t ne = skip ? 0u : a.tile_e1[tile] - ebase;
    const bool mine = !skip && tid < nv;
    const uint32_t v = mine ? a.act[i0 + tid] : 0u;
    uint32_t ro0 = 0, rv = v, gi = 0;
    uint64_t hv_own = 0, tv = 0;
    bool live = false;
    // batched runs: a graph that stopped at level L keeps its level-L state
    bool act_test = true, act_hash = true;
    if (mine) {
        ro0 = a.row_off[v];
        live = !a.alive || a.alive[v];
        if (a.bc.gid) {
            gi = a.bc.gid[v];
            const uint32_t dl = a.bc.done_level[gi];
            const bool ext = a.bc.ext && a.bc.ext[gi];
            act_test = !ext && k - 1 <= dl;
            act_hash = !ext && k <= dl;
        }
        if (test) {
            rv = a.rep[v];
            hv_own = a.h_prev[v];
        }
        if (hash) tv = a.t[v];
    }
    const LabT* __restrict__ lab = static_cast<const LabT*>(a.lab);
    uint32_t w[kEdgesPerThread];
    uint32_t l[kEdgesPerThread];
    uint64_t hv[kEdgesPerThread];
#pragma unroll
    for (int r = 0; r < kEdgesPerThread; r++) {
        const uint32_t j = tid + r * kBlock;
        w[r] = 0;
        l[r] = 0;
        if (hash && j < ne) {
            // targets and labels are read once per launch: non-temporal, so
            // they do not push the gathered hashes out of L2
            w[r] = __builtin_nontemporal_load(&a.tgt[ebase + j]);
            l[r] = static_cast<uint32_t>(__builtin_nontemporal_load(&lab[ebase + j]));
        }
    }
    // split test of level k-1: the representative's hash
    const bool probe = test && mine && live && act_test && rv != v;
    uint64_t hv_rep = 0;
    if (probe) hv_rep = a.h_prev[rv];
#pragma unroll
    for (int r = 0; r < kEdgesPerThread; r++) {
        const uint32_t j = tid + r * kBlock;
        hv[r] = (hash && j < ne) ? a.h_prev[w[r]] ^ a.salt[l[r]] : 0;
    }
    stop_decision(a, S, p_done, p_cnt, p_tot);
    if (hash) {
        if (mine) {
            S.off[tid] = ro0 - ebase;
            S.acc[tid] = 0;
        }
        if (tid == 0) S.off[nv] = ne;
    }
    __syncthreads();
    if (S.ctl[0]) return false;
    if (test) {
        // leave the class of rep[v] if h^{k-1} differs
        uint32_t founded = 0, slot = 0xFFFFFFFFu;
        if (probe && hv_own != hv_rep)
            a.rep[v] = static_cast<uint32_t>(split_join(a.test_tab, a.h_prev, rv, hv_own, v, &founded, &slot));
        if (a.bc.gid) wave_count_by_key(founded != 0, gi, a.bc.hist + static_cast<size_t>(k - 1) * a.bc.n_graphs);
        record_founders(a.test_tab, a.lcnt, k - 1, founded, slot, S.red, &S.ctl[1]);
    }
    if (!hash) return true;
    for (uint32_t j = tid; j < 2 * ne; j += kBlock) S.tab[j] = 0;
    tile_segments(nv, S.off, S.seg, S.red);
    // De-duplicate the mixed keys per vertex.  Most keys are distinct and
    // most home slots empty, so every key first tries its home slot, with
    // all of a thread's attempts in flight together; the few keys whose home
    // slot holds another key probe on from there.
    uint64_t f[kEdgesPerThread];
    uint32_t seg[kEdgesPerThread], slot[kEdgesPerThread], lo[kEdgesPerThread], hi[kEdgesPerThread];
#pragma unroll
    for (int r = 0; r < kEdgesPerThread; r++) {
        const uint32_t j = tid + r * kBlock;
        f[r] = 0;  // a zero term adds nothing to the sum, repeated or not
        if (j < ne) {
            f[r] = mix64(hv[r] ^ kCE);
            const uint32_t i = S.seg[j];
            seg[r] = i;
            lo[r] = 2 * S.off[i];
            hi[r] = 2 * S.off[i + 1];
            slot[r] = lo[r] + static_cast<uint32_t>(
                                  (static_cast<uint64_t>(static_cast<uint32_t>(f[r])) * (hi[r] - lo[r])) >> 32);
        }
    }
    uint64_t old[kEdgesPerThread];
#pragma unroll
    for (int r = 0; r < kEdgesPerThread; r++)
        if (f[r] != 0)
            old[r] = atomicCAS(reinterpret_cast<unsigned long long*>(&S.tab[slot[r]]), 0ull,
                               static_cast<unsigned long long>(f[r]));
#pragma unroll
    for (int r = 0; r < kEdgesPerThread; r++) {
        if (f[r] == 0 || old[r] == f[r]) continue;
        bool fresh = old[r] == 0;
        if (!fresh) {
            const uint32_t next = slot[r] + 1 == hi[r] ? lo[r] : slot[r] + 1;
            fresh = lds_insert(S.tab, next, lo[r], hi[r], f[r]) != 0;
        }
        if (fresh)
            atomicAdd(reinterpret_cast<unsigned long long*>(&S.acc[seg[r]]), static_cast<unsigned long long>(f[r]));
    }
    __syncthreads();
    if (mine && act_hash) a.h_next[v] = live ? mix64(tv ^ mix64(kCS + S.acc[tid])) : 0;
    return true;
}

// A hub chunk block: kTileMaxEdges edges of one hub.  Loads first, as in
// tile_block; the hub's first chunk block owns the hub vertex's split test.
template <typename LabT>
__device__ bool hub_chunk_block(const IterArgs& a, uint32_t blk, IterShared& S, uint32_t p_done, uint32_t p_cnt,
                                uint32_t p_tot) {
    const uint32_t tid = threadIdx.x, k = a.k;
    const bool test = run_test(a);
    const bool hash = run_hash(a);
    const uint32_t hi = a.hc_hub[blk];
    const uint32_t e0 = a.hc_e0[blk];
    const uint32_t v = a.hub_v[hi];
    const uint32_t logb = a.hub_logb[hi];
    const uint64_t koff = a.hub_key_off[hi];
    const uint32_t vbeg = a.row_off[v], vend = a.row_off[v + 1];
    const uint32_t ne = early_done(a) ? 0u : min(static_cast<uint32_t>(kTileMaxEdges), vend - e0);
    const LabT* __restrict__ lab = static_cast<const LabT*>(a.lab);
    uint32_t w[kEdgesPerThread];
    uint32_t l[kEdgesPerThread];
    uint64_t hv[kEdgesPerThread];
#pragma unroll
    for (int r = 0; r < kEdgesPerThread; r++) {
        const uint32_t j = tid + r * kBlock;
        w[r] = 0;
        l[r] = 0;
        if (hash && j < ne) {
            w[r] = a.tgt[e0 + j];
            l[r] = static_cast<uint32_t>(lab[e0 + j]);
        }
    }
#pragma unroll
    for (int r = 0; r < kEdgesPerThread; r++) {
        const uint32_t j = tid + r * kBlock;
        hv[r] = (hash && j < ne) ? a.h_prev[w[r]] ^ a.salt[l[r]] : 0;
    }
    stop_decision(a, S, p_done, p_cnt, p_tot);
    __syncthreads();
    if (S.ctl[0]) return false;
    if (test) {
        uint32_t founded = 0, slot = 0xFFFFFFFFu;
        if (tid == 0 && e0 == vbeg) split_test(a, v, &founded, &slot);
        record_founders(a.test_tab, a.lcnt, k - 1, founded, slot, S.red, &S.ctl[1]);
    }
    if (!hash) return true;
    uint64_t* __restrict__ out = a.hub_keys + koff + (e0 - vbeg);
    // group the chunk's nonzero keys by hash bucket (top logb bits) so each
    // hub-bucket block reads only its own keys; order within a bucket is free
    const uint32_t nb = 1u << logb;
    uint32_t* hist = reinterpret_cast<uint32_t*>(S.tab);
    for (uint32_t b = tid; b <= nb; b += kBlock) hist[b] = 0;
    __syncthreads();
    uint64_t f[kEdgesPerThread];
    uint32_t rank[kEdgesPerThread];
#pragma unroll
    for (int r = 0; r < kEdgesPerThread; r++) {
        const uint32_t j = tid + r * kBlock;
        f[r] = j < ne ? mix64(hv[r] ^ kCE) : 0;
        rank[r] = 0;
        if (f[r] != 0) {
            const uint32_t b = logb ? static_cast<uint32_t>(f[r] >> (64 - logb)) : 0u;
            rank[r] = atomicAdd(&hist[b], 1u);
        }
    }
    __syncthreads();
    if (tid == 0) {  // exclusive prefix over at most 256 buckets
        uint32_t run = 0;
        for (uint32_t b = 0; b < nb; b++) {
            const uint32_t c = hist[b];
            hist[b] = run;
            run += c;
        }
        hist[nb] = run;
    }
    __syncthreads();
    uint32_t* boff = a.hub_boff + static_cast<uint64_t>(blk) * kHubOffStride;
    for (uint32_t b = tid; b <= nb; b += kBlock) boff[b] = hist[b];
#pragma unroll
    for (int r = 0; r < kEdgesPerThread; r++) {
        if (f[r] != 0) {
            const uint32_t b = logb ? static_cast<uint32_t>(f[r] >> (64 - logb)) : 0u;
            out[hist[b] + rank[r]] = f[r];
        }
    }
    return true;
}

// A solo hub block: one hub vertex of at most kSoloMaxEdges edges, all its
// pair keys de-duplicated in the whole LDS table.
template <typename LabT>
__device__ bool solo_block(const IterArgs& a, uint32_t v, IterShared& S, uint32_t p_done, uint32_t p_cnt,
                           uint32_t p_tot) {
    const uint32_t tid = threadIdx.x, k = a.k;
    const bool test = run_test(a);
    const bool hash = run_hash(a);
    const uint32_t e0 = a.row_off[v];
    const uint32_t ne = early_done(a) ? 0u : a.row_off[v + 1] - e0;
    bool act_hash = true;
    if (a.bc.gid) act_hash = k <= a.bc.done_level[a.bc.gid[v]];
    const uint64_t tv = hash ? a.t[v] : 0;
    const LabT* __restrict__ lab = static_cast<const LabT*>(a.lab);
    uint32_t w[kSoloPerThread];
    uint32_t l[kSoloPerThread];
    uint64_t hv[kSoloPerThread];
#pragma unroll
    for (int r = 0; r < kSoloPerThread; r++) {
        const uint32_t j = tid + r * kBlock;
        w[r] = 0;
        l[r] = 0;
        if (hash && j < ne) {
            w[r] = a.tgt[e0 + j];
            l[r] = static_cast<uint32_t>(lab[e0 + j]);
        }
    }
#pragma unroll
    for (int r = 0; r < kSoloPerThread; r++) {
        const uint32_t j = tid + r * kBlock;
        hv[r] = (hash && j < ne) ? a.h_prev[w[r]] ^ a.salt[l[r]] : 0;
    }
    // the table spans tab, acc and off (the arrays a tile block uses)
    uint64_t* tab = S.tab;
    stop_decision(a, S, p_done, p_cnt, p_tot);
    for (uint32_t j = tid; j < kSoloSlots; j += kBlock) tab[j] = 0;
    __syncthreads();
    if (S.ctl[0]) return false;
    if (test) {
        uint32_t founded = 0, slot = 0xFFFFFFFFu;
        if (tid == 0) split_test(a, v, &founded, &slot);
        record_founders(a.test_tab, a.lcnt, k - 1, founded, slot, S.red, &S.ctl[1]);
    }
    if (!hash) return true;
    // home-slot attempts first, all in flight together (see tile_block)
    uint64_t acc = 0;
    uint64_t f[kSoloPerThread], old[kSoloPerThread];
#pragma unroll
    for (int r = 0; r < kSoloPerThread; r++) {
        const uint32_t j = tid + r * kBlock;
        f[r] = j < ne ? mix64(hv[r] ^ kCE) : 0;
    }
    // double hashing: home slot from the low key bits, step from the high
    // bits; the table size is prime, so every step visits every slot
    uint32_t home[kSoloPerThread];
#pragma unroll
    for (int r = 0; r < kSoloPerThread; r++)
        home[r] = static_cast<uint32_t>((static_cast<uint64_t>(static_cast<uint32_t>(f[r])) * kSoloSlots) >> 32);
#pragma unroll
    for (int r = 0; r < kSoloPerThread; r++)
        if (f[r] != 0)
            old[r] = atomicCAS(reinterpret_cast<unsigned long long*>(&tab[home[r]]), 0ull,
                               static_cast<unsigned long long>(f[r]));
#pragma unroll
    for (int r = 0; r < kSoloPerThread; r++) {
        if (f[r] == 0 || old[r] == f[r]) continue;
        bool fresh = old[r] == 0;
        if (!fresh) {
            const uint32_t step = 1u + static_cast<uint32_t>(f[r] >> 32) % (kSoloSlots - 1);
            fresh = lds_insert_step(tab, home[r], step, kSoloSlots, f[r]) != 0;
        }
        if (fresh) acc += f[r];
    }
    acc = wave_sum_u64(acc);
    uint64_t* wsum = reinterpret_cast<uint64_t*>(S.seg);  // outside the table
    if (lane_id() == 0) wsum[tid >> 6] = acc;
    __syncthreads();
    if (tid == 0 && act_hash) {
        uint64_t sum = 0;
        for (int i = 0; i < kBlock / 64; i++) sum += wsum[i];
        a.h_next[v] = mix64(tv ^ mix64(kCS + sum));
    }
    return true;
}

// kIsoPerBlock vertices without out-edges: split test, and h^k = M(t ^
// M(C_S)) where the hash buffer still needs it.
__device__ bool iso_block(const IterArgs& a, uint32_t blk, IterShared& S, uint32_t p_done, uint32_t p_cnt,
                          uint32_t p_tot) {
    const uint32_t tid = threadIdx.x, k = a.k;
    const bool test = run_test(a);
    const bool hash = run_hash(a) && (k <= 2 || a.all_levels);
    uint32_t v[kIsoPerThread], rv[kIsoPerThread], gi[kIsoPerThread];
    uint64_t hv_own[kIsoPerThread], hv_rep[kIsoPerThread], tv[kIsoPerThread];
    bool mine[kIsoPerThread], live[kIsoPerThread], probe[kIsoPerThread], act_hash[kIsoPerThread];
#pragma unroll
    for (int r = 0; r < kIsoPerThread; r++) {
        const uint32_t i = blk * kIsoPerBlock + r * kBlock + tid;
        mine[r] = i < a.n_iso;
        v[r] = mine[r] ? a.iso[i] : 0u;
        rv[r] = v[r];
        gi[r] = 0;
        hv_own[r] = tv[r] = hv_rep[r] = 0;
        live[r] = false;
        act_hash[r] = true;
        bool act_test = true;
        if (mine[r]) {
            live[r] = !a.alive || a.alive[v[r]];
            if (a.bc.gid) {
                gi[r] = a.bc.gid[v[r]];
                const uint32_t dl = a.bc.done_level[gi[r]];
                const bool ext = a.bc.ext && a.bc.ext[gi[r]];
                act_test = !ext && k - 1 <= dl;
                act_hash[r] = !ext && k <= dl;
            }
            if (test) {
                rv[r] = a.rep[v[r]];
                hv_own[r] = a.h_prev[v[r]];
            }
            if (hash) tv[r] = a.t[v[r]];
        }
        probe[r] = test && mine[r] && live[r] && act_test && rv[r] != v[r];
    }
#pragma unroll
    for (int r = 0; r < kIsoPerThread; r++)
        if (probe[r]) hv_rep[r] = a.h_prev[rv[r]];
    stop_decision(a, S, p_done, p_cnt, p_tot);
    __syncthreads();
    if (S.ctl[0]) return false;
    if (test) {
        for (int r = 0; r < kIsoPerThread; r++) {
            // vertices without out-edges of one type set and one class all
            // carry the same key: group them per wave before the table
            uint32_t founded = 0, slot = 0xFFFFFFFFu;
            const bool part = probe[r] && hv_own[r] != hv_rep[r];
            const uint64_t o = wave_split_join(a.test_tab, a.h_prev, part, rv[r], hv_own[r], v[r], &founded, &slot);
            if (part) a.rep[v[r]] = static_cast<uint32_t>(o);
            if (a.bc.gid)
                wave_count_by_key(founded != 0, gi[r], a.bc.hist + static_cast<size_t>(k - 1) * a.bc.n_graphs);
            record_founders(a.test_tab, a.lcnt, k - 1, founded, slot, S.red, &S.ctl[1]);
        }
    }
    if (hash) {
#pragma unroll
        for (int r = 0; r < kIsoPerThread; r++)
            if (mine[r] && act_hash[r]) a.h_next[v[r]] = live[r] ? mix64(tv[r] ^ mix64(kCS)) : 0;
    }
    return true;
}

// A block with no tile (an empty graph still needs its stop test).
__device__ bool null_block(const IterArgs& a, IterShared& S, uint32_t p_done, uint32_t p_cnt, uint32_t p_tot) {
    stop_decision(a, S, p_done, p_cnt, p_tot);
    __syncthreads();
    return S.ctl[0] == 0;
}

// Recycling, after the block's own work: counters of level k-3 and the
// split table that level k-2 filled (launch k+1 tests level k in it).
__device__ void recycle(const IterArgs& a) {
    const uint32_t tid = threadIdx.x, k = a.k;
    if (blockIdx.x == 0 && tid < kStripes && k >= 3)
        a.lcnt[((k - 3) & (kStripeRing - 1)) * kStripes + tid] = 0;
    if (k < 2) return;
    const uint32_t* cnt = a.lcnt + ((k - 2) & (kStripeRing - 1)) * kStripes;
    bool overflow = false;
    for (int st = 0; st < kStripes; st++) overflow |= cnt[st] > static_cast<uint32_t>(kListPerStripe);
    if (overflow) {
        const uint64_t cap = static_cast<uint64_t>(a.clr_tab.mask) + 1;
        const uint64_t per = (cap + gridDim.x - 1) / gridDim.x;
        const uint64_t lo = per * blockIdx.x, hi = min(cap, lo + per);
        for (uint64_t j = lo + tid; j < hi; j += kBlock) a.clr_tab.slots[j] = 0;
    } else {
        const uint64_t items = static_cast<uint64_t>(kStripes) * kListPerStripe;
        for (uint64_t i = static_cast<uint64_t>(blockIdx.x) * kBlock + tid; i < items;
             i += static_cast<uint64_t>(gridDim.x) * kBlock) {
            const uint32_t st = static_cast<uint32_t>(i / kListPerStripe);
            const uint32_t e = static_cast<uint32_t>(i % kListPerStripe);
            if (e < cnt[st]) {
                const uint32_t idx = a.clr_tab.list[i];
                if (idx <= a.clr_tab.mask) a.clr_tab.slots[idx] = 0;
            }
        }
    }
}

template <typename LabT>
__global__ void __launch_bounds__(kBlock) k_iterate(IterArgs a) {
    __shared__ IterShared S;
    const uint32_t tid = threadIdx.x;
    const uint32_t k = a.k;
    // stop-test inputs (level k - stop_lag), loaded together with everything else
    uint32_t p_done = 0, p_cnt = 0, p_tot = 0;
    if (tid < 64) {
        p_done = __hip_atomic_load(&a.status->done, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        const uint32_t lag = stop_lag(a);
        if (k >= lag && !a.bc.gid && !a.hash_only) {
            const uint32_t lv = k - lag;
            p_cnt = a.lcnt[(lv & (kStripeRing - 1)) * kStripes + tid];
            p_tot = lv ? a.totals[lv - 1] : 0u;
        }
    }
    bool go;
    const uint32_t b = blockIdx.x;
    if (a.stop_only)
        go = null_block(a, S, p_done, p_cnt, p_tot);
    else if (b < a.n_hub_chunks)
        go = hub_chunk_block<LabT>(a, b, S, p_done, p_cnt, p_tot);
    else if (b - a.n_hub_chunks < a.n_solo)
        go = solo_block<LabT>(a, a.solo_v[b - a.n_hub_chunks], S, p_done, p_cnt, p_tot);
    else if (b - a.n_hub_chunks - a.n_solo < a.n_iso_blocks)
        go = iso_block(a, b - a.n_hub_chunks - a.n_solo, S, p_done, p_cnt, p_tot);
    else if (b - a.n_hub_chunks - a.n_solo - a.n_iso_blocks < a.n_tiles)
        go = tile_block<LabT>(a, b - a.n_hub_chunks - a.n_solo - a.n_iso_blocks, S, p_done, p_cnt, p_tot);
    else
        go = null_block(a, S, p_done, p_cnt, p_tot);
    // the hash half of a split launch recycles nothing: its split half did
    if (go && !a.hash_only && a.phase != kPhaseHash) recycle(a);
}

// ------------------------------------------------------------ hub buckets

constexpr int kMaxHubRuns = 256;  // chunk runs staged in LDS at a time

// Stage the runs of chunks [cb, cb+ncb) of this bucket: s_src[i] = scratch
// offset of run i, s_run = exclusive prefix of run lengths (s_run[ncb] = total).
__device__ void stage_runs(const HubArgs& a, uint32_t c0, uint32_t cb, uint32_t ncb, uint32_t bucket,
                           uint32_t e_first, uint32_t* s_run, uint32_t* s_src) {
    const uint32_t tid = threadIdx.x;
    __syncthreads();
    if (tid < ncb) {
        const uint32_t blk = c0 + cb + tid;
        const uint32_t* boff = a.hub_boff + static_cast<uint64_t>(blk) * kHubOffStride;
        s_src[tid] = (a.hc_e0[blk] - e_first) + boff[bucket];
        s_run[tid + 1] = boff[bucket + 1] - boff[bucket];
    }
    __syncthreads();
    if (tid == 0) {
        s_run[0] = 0;
        for (uint32_t i = 1; i <= ncb; i++) s_run[i] += s_run[i - 1];
    }
    __syncthreads();
}

__global__ void __launch_bounds__(kHubBlock) k_hub(HubArgs a) {
    extern __shared__ uint64_t s_tab[];
    __shared__ uint64_t s_red64[kHubBlock / 64];
    __shared__ uint32_t s_ctl[4];
    __shared__ uint32_t s_run[kMaxHubRuns + 1];   // prefix of run lengths
    __shared__ uint32_t s_src[kMaxHubRuns];       // scratch offset of each run
    const uint32_t tid = threadIdx.x;
    if (*reinterpret_cast<volatile uint32_t*>(&a.status->done)) return;
    const uint32_t hi = a.hb_hub[blockIdx.x];
    const uint32_t bucket = a.hb_bucket[blockIdx.x];
    const uint32_t logb = a.hub_logb[hi];
    const uint32_t c0 = a.hub_chunk0[hi], nc = a.hub_nchunks[hi];
    const uint64_t* __restrict__ keys = a.hub_keys + a.hub_key_off[hi];
    const uint32_t mask = a.table_slots - 1;
    volatile uint32_t* ctl = s_ctl;
    const uint32_t e_first = a.hc_e0[c0];

    // The bucket's keys form one run per chunk of the hub.  They are inserted
    // into one LDS table (runs staged kMaxHubRuns chunks at a time).  Only
    // distinct keys occupy slots; a bucket with more distinct keys than the
    // table limit is re-split by further hash bits and re-read, which ends
    // because distinct keys differ in some bit (depth capped for safety).
    uint64_t sum = 0;
    for (uint32_t extra = 0;; extra++) {
        if (extra > kMaxHubExtraBits) {
            if (tid == 0) atomicOr(&a.status->error, kErrHubSplit);
            break;
        }
        sum = 0;
        bool overflow = false;
        const uint32_t bits = logb + extra;
        for (uint32_t sub = 0; sub < (1u << extra) && !overflow; sub++) {
            const uint64_t want = (static_cast<uint64_t>(bucket) << extra) | sub;
            __syncthreads();
            for (uint32_t j = tid; j < a.table_slots; j += kHubBlock) s_tab[j] = 0;
            if (tid == 0) {
                ctl[1] = 0;  // distinct keys inserted
                ctl[2] = 0;  // overflow
            }
            for (uint32_t cb = 0; cb < nc && !overflow; cb += kMaxHubRuns) {
                const uint32_t ncb = min(static_cast<uint32_t>(kMaxHubRuns), nc - cb);
                stage_runs(a, c0, cb, ncb, bucket, e_first, s_run, s_src);
                const uint32_t total = s_run[ncb];
                for (uint32_t j0 = 0; j0 < total; j0 += 4 * kHubBlock) {
                    if (ctl[2]) break;
                    uint64_t f[4];
#pragma unroll
                    for (int r = 0; r < 4; r++) {
                        const uint32_t j = j0 + r * kHubBlock + tid;
                        f[r] = 0;
                        if (j < total) {
                            // run containing j: binary search over the run prefix
                            uint32_t lo = 0, hi2 = ncb;
                            while (hi2 - lo > 1) {
                                const uint32_t mid = (lo + hi2) >> 1;
                                if (s_run[mid] <= j) lo = mid; else hi2 = mid;
                            }
                            f[r] = keys[s_src[lo] + (j - s_run[lo])];
                        }
                    }
#pragma unroll
                    for (int r = 0; r < 4; r++) {
                        if (f[r] == 0) continue;
                        if (extra && (f[r] >> (64 - bits)) != want) continue;
                        const uint32_t got =
                            lds_insert_bounded(s_tab, static_cast<uint32_t>(f[r]) & mask, a.table_slots, f[r]);
                        if (got == 1u) {
                            sum += f[r];
                            // count distinct keys only: duplicates never overflow
                            if (atomicAdd(const_cast<uint32_t*>(&ctl[1]), 1u) + 1 >= a.table_limit) ctl[2] = 1;
                        } else if (got == 2u) {
                            ctl[2] = 1;
                        }
                    }
                }
                __syncthreads();
                overflow = ctl[2] != 0;
            }
        }
        if (!overflow) break;
    }
    __syncthreads();
    // block sum
    uint64_t x = wave_sum_u64(sum);
    if (lane_id() == 0) s_red64[tid >> 6] = x;
    __syncthreads();
    if (tid == 0) {
        uint64_t bsum = 0;
        for (int i = 0; i < kHubBlock / 64; i++) bsum += s_red64[i];
        __hip_atomic_fetch_add(&a.hub_acc[hi], bsum, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
}

// h^k of each chunked hub from the sum of its buckets' distinct keys.  The
// sums are read here, one launch after the bucket blocks added them, so the
// bucket blocks need no fence or completion count (an agent-scope fence on
// this chip writes back or invalidates the whole L2 of the block's XCD);
// each sum is cleared for the next level.
__global__ void __launch_bounds__(kBlock) k_hub_finish(const uint64_t* t, const uint32_t* hub_v, uint64_t* hub_acc,
                                                       uint32_t n_big, uint64_t* h_next, const RunStatus* status,
                                                       uint32_t k, BatchCtl bc) {
    const uint32_t i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= n_big || status->done) return;  // a done run added nothing
    const uint64_t acc = hub_acc[i];
    hub_acc[i] = 0;
    const uint32_t v = hub_v[i];
    if (!bc.gid || k <= bc.done_level[bc.gid[v]]) h_next[v] = mix64(t[v] ^ mix64(kCS + acc));
}

// ------------------------------------------------------------ batched stop

// Launch k of a batched run begins with this: graph g stops at level k-2
// when its class count did not grow there (fixpoint) or k-2 reaches k_max.
__global__ void __launch_bounds__(kBlock) k_graph_stop(BatchCtl bc, uint32_t k, uint32_t k_max, uint32_t stop,
                                                       RunStatus* status) {
    const uint32_t g = blockIdx.x * kBlock + threadIdx.x;
    if (g >= bc.n_graphs || k < 2 || bc.done_level[g] != 0xFFFFFFFFu) return;
    const uint32_t lv = k - 2;
    const uint32_t c = bc.hist[static_cast<size_t>(lv) * bc.n_graphs + g];
    const uint32_t fx = (lv >= 1 && c == 0) ? 1u : 0u;
    if ((stop && fx) || lv >= k_max) {
        bc.done_level[g] = lv;
        bc.fix[g] = fx;
        if (atomicAdd(bc.n_done, 1u) + 1 == bc.n_graphs) {
            status->k_done = lv;
            status->fixpoint = fx;
            status->done = 1;
        }
    }
}

// ------------------------------------------------------------ level classes
//
// The classes of stored levels h^0..h^K, level by level (used by the
// resident state, whose levels change under update batches): level 0 groups
// alive vertices by t(v); level j >= 1 splits every class by h^j with the
// same split test as launch j+1 of the refinement loop.

}  // namespace

uint32_t query_hub_table_slots(int device, bool device_max) {
    int bytes = 0;
    if (hipDeviceGetAttribute(&bytes, hipDeviceAttributeMaxSharedMemoryPerBlock, device) != hipSuccess)
        bytes = 65536;
    // keep room for the block's static LDS.  Keys arrive grouped by bucket,
    // so small tables cost no extra reads and let several blocks share a CU.
    uint64_t avail = bytes > 4096 ? static_cast<uint64_t>(bytes) - 4096 : 4096;
    uint64_t slots = std::min<uint64_t>(avail / 8, device_max ? 16384 : kHubTableDefault);
    uint32_t p = 1;
    while (2ull * p <= slots) p <<= 1;
    return p;
}

static SplitTable make_table(Arena& arena, uint64_t cap) {
    SplitTable T;
    T.slots = arena.alloc<uint64_t>(cap);
    T.list = arena.alloc<uint32_t>(static_cast<size_t>(kStripes) * kListPerStripe);
    T.mask = static_cast<uint32_t>(cap - 1);
    return T;
}

void alloc_run_buffers(const Staged& g, uint32_t k_max, bool stop, RunBuffers& rb, Arena& arena,
                       hipStream_t s) {
    const uint32_t n = g.n;
    rb.t = arena.alloc<uint64_t>(n);
    rb.h[0] = arena.alloc<uint64_t>(n);
    rb.h[1] = arena.alloc<uint64_t>(n);
    rb.rep = arena.alloc<uint32_t>(n);
    const uint64_t cap = split_table_slots(n);
    for (int i = 0; i < 2; i++) {
        rb.tab[i] = make_table(arena, cap);
        hip_check(hipMemsetAsync(rb.tab[i].slots, 0, static_cast<size_t>(cap) * sizeof(uint64_t), s),
                  "clear split table");
    }
    rb.lcnt = arena.alloc<uint32_t>(kStripeRing * kStripes);
    // level j's count is written by launch j+2 <= k_done+2; k_done <= max(n, 1)
    // when stopping at the fixpoint, else k_max
    const uint64_t kc = stop ? std::min<uint64_t>(k_max, static_cast<uint64_t>(n) + 1) : k_max;
    rb.k_cap = static_cast<uint32_t>(kc) + 3;
    rb.totals = arena.alloc<uint32_t>(rb.k_cap);
    rb.hub_keys = arena.alloc<uint64_t>(g.hub_keys_total + 1);
    rb.hub_boff = arena.alloc<uint32_t>((static_cast<size_t>(g.n_hub_chunks) + 1) * kHubOffStride);
    rb.hub_acc = arena.alloc<uint64_t>(g.n_hubs + 1);
    rb.status = arena.alloc<RunStatus>(1);
    hip_check(hipMemsetAsync(rb.lcnt, 0, kStripeRing * kStripes * 4, s), "clear counters");
    hip_check(hipMemsetAsync(rb.totals, 0, rb.k_cap * 4, s), "clear totals");
    hip_check(hipMemsetAsync(rb.hub_acc, 0, (g.n_hubs + 1) * 8, s), "clear hub acc");
    hip_check(hipMemsetAsync(rb.status, 0, sizeof(RunStatus), s), "clear status");
}

void launch_init(const Staged& g, const RunBuffers& rb, bool untyped, hipStream_t s) {
    const uint32_t n = g.n;
    const uint32_t grid = std::max<uint32_t>(ceil_div(n, kBlock), 1);
    k_types<<<grid, kBlock, 0, s>>>(g.type_off, g.type_ids, g.alive, n, untyped ? 1 : 0, rb.t, rb.h[0]);
    k_init<<<grid, kBlock, 0, s>>>(rb.t, g.alive, n, rb.rep, rb.tab[0], rb.lcnt, rb.bc);
    hip_check(hipGetLastError(), "init launch");
}

void launch_iteration(const Staged& g, const RunBuffers& rb, uint32_t k, uint32_t k_max,
                      bool stop, bool all_levels, hipStream_t s, uint32_t phase, bool stop_only) {
    IterArgs a{};
    a.phase = phase;
    a.stop_only = stop_only ? 1u : 0u;
    a.row_off = g.row_off;
    a.tgt = g.tgt;
    a.lab = g.lab;
    a.t = rb.t;
    a.salt = g.salt;
    a.h_prev = rb.h[(k - 1) & 1];
    a.h_next = rb.h[k & 1];
    a.alive = g.alive;
    a.rep = rb.rep;
    a.tile_i0 = g.tile_i0;
    a.tile_i1 = g.tile_i1;
    a.tile_e0 = g.tile_e0;
    a.tile_e1 = g.tile_e1;
    a.act = g.act;
    a.iso = g.iso;
    a.n_iso = g.n_iso;
    a.n_iso_blocks = ceil_div(g.n_iso, kIsoPerBlock);
    a.hc_hub = g.hc_hub;
    a.hc_e0 = g.hc_e0;
    a.hub_v = g.hub_v;
    a.hub_logb = g.hub_logb;
    a.hub_key_off = g.hub_key_off;
    a.hub_keys = rb.hub_keys;
    a.hub_boff = rb.hub_boff;
    a.test_tab = rb.tab[(k - 1) & 1];
    a.clr_tab = rb.tab[k & 1];
    a.lcnt = rb.lcnt;
    a.totals = rb.totals;
    a.status = rb.status;
    a.n_tiles = g.n_tiles;
    a.n_hub_chunks = g.n_hub_chunks;
    a.n_solo = g.n_solo;
    a.solo_v = g.hub_v ? g.hub_v + (g.n_hubs - g.n_solo) : nullptr;
    a.k = k;
    a.k_max = k_max;
    a.stop = stop ? 1u : 0u;
    a.all_levels = all_levels ? 1u : 0u;
    a.bc = rb.bc;
    const uint32_t grid =
        stop_only ? 1u : std::max<uint32_t>(g.n_hub_chunks + g.n_solo + a.n_iso_blocks + g.n_tiles, 1);
    if (g.label_bytes == 2)
        k_iterate<uint16_t><<<grid, kBlock, 0, s>>>(a);
    else
        k_iterate<uint32_t><<<grid, kBlock, 0, s>>>(a);
    hip_check(hipGetLastError(), "iteration launch");
}

void launch_hubs(const Staged& g, const RunBuffers& rb, uint32_t k, hipStream_t s) {
    if (g.n_hub_blocks == 0) return;
    HubArgs a{};
    a.t = rb.t;
    a.hub_keys = rb.hub_keys;
    a.hub_key_off = g.hub_key_off;
    a.hub_boff = rb.hub_boff;
    a.hub_chunk0 = g.hub_chunk0;
    a.hub_nchunks = g.hub_nchunks;
    a.hc_e0 = g.hc_e0;
    a.hub_v = g.hub_v;
    a.hub_deg = g.hub_deg;
    a.hub_logb = g.hub_logb;
    a.hb_hub = g.hb_hub;
    a.hb_bucket = g.hb_bucket;
    a.hub_acc = rb.hub_acc;
    a.h_next = rb.h[k & 1];
    a.status = rb.status;
    a.table_slots = g.hub_table_slots;
    a.table_limit = (g.hub_table_slots / 8) * 7;
    a.k = k;
    a.bc = rb.bc;
    k_hub<<<g.n_hub_blocks, kHubBlock, static_cast<size_t>(g.hub_table_slots) * 8, s>>>(a);
    hip_check(hipGetLastError(), "hub launch");
    const uint32_t n_big = g.n_hubs - g.n_solo;
    k_hub_finish<<<ceil_div(n_big, kBlock), kBlock, 0, s>>>(rb.t, g.hub_v, rb.hub_acc, n_big, rb.h[k & 1],
                                                              rb.status, k, rb.bc);
    hip_check(hipGetLastError(), "hub finish launch");
}

void alloc_hash_scratch(const Staged& g, HashScratch& hs, Arena& arena, hipStream_t s) {
    hs.hub_keys = arena.alloc<uint64_t>(g.hub_keys_total + 1);
    hs.hub_boff = arena.alloc<uint32_t>((static_cast<size_t>(g.n_hub_chunks) + 1) * kHubOffStride);
    hs.hub_acc = arena.alloc<uint64_t>(g.n_hubs + 1);
    hs.status = arena.alloc<RunStatus>(1);
    hip_check(hipMemsetAsync(hs.hub_acc, 0, (g.n_hubs + 1) * 8ull, s), "hub acc");
    hip_check(hipMemsetAsync(hs.status, 0, sizeof(RunStatus), s), "status");
}

void launch_hash_level(const Staged& g, const uint64_t* t, const uint64_t* h_prev, uint64_t* h_next,
                       const HashScratch& hs, uint32_t level, hipStream_t s) {
    IterArgs a{};
    a.row_off = g.row_off;
    a.tgt = g.tgt;
    a.lab = g.lab;
    a.t = t;
    a.salt = g.salt;
    a.h_prev = h_prev;
    a.h_next = h_next;
    a.alive = g.alive;
    a.tile_i0 = g.tile_i0;
    a.tile_i1 = g.tile_i1;
    a.tile_e0 = g.tile_e0;
    a.tile_e1 = g.tile_e1;
    a.act = g.act;
    a.iso = g.iso;
    a.n_iso = g.n_iso;
    a.n_iso_blocks = ceil_div(g.n_iso, kIsoPerBlock);
    a.hc_hub = g.hc_hub;
    a.hc_e0 = g.hc_e0;
    a.hub_v = g.hub_v;
    a.hub_logb = g.hub_logb;
    a.hub_key_off = g.hub_key_off;
    a.hub_keys = hs.hub_keys;
    a.hub_boff = hs.hub_boff;
    a.status = hs.status;
    a.n_tiles = g.n_tiles;
    a.n_hub_chunks = g.n_hub_chunks;
    a.n_solo = g.n_solo;
    a.solo_v = g.hub_v ? g.hub_v + (g.n_hubs - g.n_solo) : nullptr;
    a.k = level;
    a.k_max = 0xFFFFFFFFu;
    a.hash_only = 1;
    a.all_levels = 1;
    const uint32_t grid = std::max<uint32_t>(g.n_hub_chunks + g.n_solo + a.n_iso_blocks + g.n_tiles, 1);
    if (g.label_bytes == 2)
        k_iterate<uint16_t><<<grid, kBlock, 0, s>>>(a);
    else
        k_iterate<uint32_t><<<grid, kBlock, 0, s>>>(a);
    hip_check(hipGetLastError(), "hash level launch");
    if (g.n_hub_blocks == 0) return;
    HubArgs h{};
    h.t = t;
    h.hub_keys = hs.hub_keys;
    h.hub_key_off = g.hub_key_off;
    h.hub_boff = hs.hub_boff;
    h.hub_chunk0 = g.hub_chunk0;
    h.hub_nchunks = g.hub_nchunks;
    h.hc_e0 = g.hc_e0;
    h.hub_v = g.hub_v;
    h.hub_deg = g.hub_deg;
    h.hub_logb = g.hub_logb;
    h.hb_hub = g.hb_hub;
    h.hb_bucket = g.hb_bucket;
    h.hub_acc = hs.hub_acc;
    h.h_next = h_next;
    h.status = hs.status;
    h.table_slots = g.hub_table_slots;
    h.table_limit = (g.hub_table_slots / 8) * 7;
    h.k = level;
    k_hub<<<g.n_hub_blocks, kHubBlock, static_cast<size_t>(g.hub_table_slots) * 8, s>>>(h);
    hip_check(hipGetLastError(), "hash level hub launch");
    const uint32_t n_big = g.n_hubs - g.n_solo;
    k_hub_finish<<<ceil_div(n_big, kBlock), kBlock, 0, s>>>(t, g.hub_v, hs.hub_acc, n_big, h_next, hs.status,
                                                              level, BatchCtl{});
    hip_check(hipGetLastError(), "hash level hub finish launch");
}

void launch_graph_stop(const RunBuffers& rb, uint32_t k, uint32_t k_max, bool stop, hipStream_t s) {
    k_graph_stop<<<ceil_div(rb.bc.n_graphs, kBlock), kBlock, 0, s>>>(rb.bc, k, k_max, stop ? 1u : 0u, rb.status);
    hip_check(hipGetLastError(), "graph stop launch");
}

}  // namespace bsim
