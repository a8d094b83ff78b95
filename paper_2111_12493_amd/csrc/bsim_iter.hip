// bsim_iter.hip -- the refinement loop (a2-a7).
//
// Iteration 0 hashes every vertex's type set (Algorithm 4's initialization:
// the ID of the local schema).  Iteration k >= 1 is one launch of
// k_iterate: every block first evaluates the stop test on the counts of the
// previous launch, then either
//   * a tile block: gathers h^{k-1} of its tile's out-edge targets
//     (SignalMessages), de-duplicates the (label, hash) pair keys of each
//     vertex in a per-vertex open-addressing region of an LDS table
//     (MergeMessages' hash table), sums the mixed distinct keys per vertex
//     (the order-independent Hash), and writes h^k; or
//   * a hub chunk block: the same for up to kTileMaxEdges edges of one hub,
//     de-duplicating into the hub's region of a global table; partial sums
//     meet in a global accumulator and the hub's last chunk block finishes
//     the hash and clears the region.
// Every new h^k is inserted into a key-only count table; the number of new
// keys is n_k, the block count of the k-partition.  The launch after the
// one where n_k == n_{k-1} (or k > k_max) sets a sticky done flag and every
// later launch returns at once, so the host can queue launches ahead.
#include "bsim_device.h"

namespace bsim {

namespace {

__global__ void __launch_bounds__(kBlock) k_type_hash(
    const uint32_t* __restrict__ type_off, const uint32_t* __restrict__ type_ids,
    const uint8_t* __restrict__ alive, uint32_t n, int untyped, uint64_t* __restrict__ t,
    uint64_t* __restrict__ h0, uint64_t* tab, uint32_t mask, uint32_t* zflag, uint32_t* stripes) {
    __shared__ uint32_t s_red[kBlock / 64];
    const uint32_t v = blockIdx.x * kBlock + threadIdx.x;
    uint32_t fresh = 0;
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
            fresh = count_insert(tab, mask, zflag, tv);
        }
        t[v] = tv;
        h0[v] = tv;
    }
    uint32_t c = block_sum_u32(fresh, s_red);
    if (threadIdx.x == 0) add_block_count(stripes, 0, c);
}

struct IterShared {
    uint64_t tab[kTableSlots];
    uint64_t acc[kTileMaxVerts];
    uint64_t red64[kBlock / 64];
    uint32_t off[kTileMaxVerts + 1];
    uint32_t red[kBlock / 64];
    uint32_t ctl[4];
    alignas(8) uint8_t seg[kTileMaxEdges];
};

template <typename LabT>
__device__ void tile_block(const IterArgs& a, uint32_t tile, IterShared& S) {
    const uint32_t tid = threadIdx.x;
    const uint32_t v0 = a.tile_v0[tile], v1 = a.tile_v1[tile];
    const uint32_t nv = v1 - v0;
    const uint32_t ebase = a.row_off[v0];
    for (uint32_t i = tid; i <= nv; i += kBlock) S.off[i] = a.row_off[v0 + i] - ebase;
    for (uint32_t i = tid; i < nv; i += kBlock) S.acc[i] = 0;
    __syncthreads();
    const uint32_t ne = S.off[nv];
    for (uint32_t j = tid; j < 2 * ne; j += kBlock) S.tab[j] = 0;
    tile_segments(nv, S.off, S.seg, S.red);

    const LabT* __restrict__ lab = static_cast<const LabT*>(a.lab);
    // stage all loads first so the gathers of one thread are in flight together
    uint32_t w[kEdgesPerThread];
    uint32_t l[kEdgesPerThread];
#pragma unroll
    for (int r = 0; r < kEdgesPerThread; r++) {
        const uint32_t j = tid + r * kBlock;
        if (j < ne) {
            w[r] = a.tgt[ebase + j];
            l[r] = static_cast<uint32_t>(lab[ebase + j]);
        }
    }
    uint64_t hv[kEdgesPerThread];
#pragma unroll
    for (int r = 0; r < kEdgesPerThread; r++) {
        const uint32_t j = tid + r * kBlock;
        if (j < ne) hv[r] = a.h_prev[w[r]] ^ a.salt[l[r]];
    }
#pragma unroll
    for (int r = 0; r < kEdgesPerThread; r++) {
        const uint32_t j = tid + r * kBlock;
        if (j < ne) {
            const uint64_t f = mix64(hv[r] ^ kCE);
            if (f != 0) {  // a zero term adds nothing to the sum, repeated or not
                const uint32_t i = S.seg[j];
                const uint32_t base = 2 * S.off[i];
                const uint32_t span = 2 * (S.off[i + 1] - S.off[i]);
                const uint32_t slot = base + static_cast<uint32_t>(
                                                 (static_cast<uint64_t>(static_cast<uint32_t>(f)) * span) >> 32);
                if (lds_insert(S.tab, slot, base, base + span, f))
                    atomicAdd(reinterpret_cast<unsigned long long*>(&S.acc[i]),
                              static_cast<unsigned long long>(f));
            }
        }
    }
    __syncthreads();
    uint32_t fresh = 0;
    if (tid < nv) {
        const uint32_t v = v0 + tid;
        if (!a.alive || a.alive[v]) {
            const uint64_t h = mix64(a.t[v] ^ mix64(kCS + S.acc[tid]));
            a.h_next[v] = h;
            fresh = count_insert(a.tab_ins, a.tab_mask, a.zflag_ins, h);
        } else {
            a.h_next[v] = 0;
        }
    }
    const uint32_t c = block_sum_u32(fresh, S.red);
    if (tid == 0) add_block_count(a.stripes, a.k, c);
}

// Insert a nonzero key into a region [base, base+span) of a global table;
// returns 1 if it was not present.  Read before CAS as in count_insert.
__device__ __forceinline__ uint32_t global_region_insert(uint64_t* tab, uint64_t base, uint32_t span,
                                                         uint64_t f) {
    uint32_t off = static_cast<uint32_t>((static_cast<uint64_t>(static_cast<uint32_t>(f)) * span) >> 32);
    for (;;) {
        uint64_t* p = tab + base + off;
        const uint64_t cur = *p;
        if (cur == f) return 0u;
        if (cur == 0) {
            unsigned long long old = atomicCAS(reinterpret_cast<unsigned long long*>(p), 0ull,
                                               static_cast<unsigned long long>(f));
            if (old == 0ull) return 1u;
            if (old == f) return 0u;
        }
        if (++off == span) off = 0;
    }
}

template <typename LabT>
__device__ void hub_chunk_block(const IterArgs& a, uint32_t blk, IterShared& S) {
    const uint32_t tid = threadIdx.x;
    const uint32_t hi = a.hc_hub[blk];
    const uint32_t e0 = a.hc_e0[blk];
    const uint32_t v = a.hub_v[hi];
    const uint32_t vbeg = a.row_off[v], vend = a.row_off[v + 1];
    const uint32_t ne = min(static_cast<uint32_t>(kTileMaxEdges), vend - e0);
    const uint32_t span = 2 * (vend - vbeg);
    const uint64_t base = a.hub_tab_off[hi];
    const LabT* __restrict__ lab = static_cast<const LabT*>(a.lab);

    uint32_t w[kEdgesPerThread];
    uint32_t l[kEdgesPerThread];
#pragma unroll
    for (int r = 0; r < kEdgesPerThread; r++) {
        const uint32_t j = tid + r * kBlock;
        if (j < ne) {
            w[r] = a.tgt[e0 + j];
            l[r] = static_cast<uint32_t>(lab[e0 + j]);
        }
    }
    uint64_t hv[kEdgesPerThread];
#pragma unroll
    for (int r = 0; r < kEdgesPerThread; r++) {
        const uint32_t j = tid + r * kBlock;
        if (j < ne) hv[r] = a.h_prev[w[r]] ^ a.salt[l[r]];
    }
    uint64_t sum = 0;
#pragma unroll
    for (int r = 0; r < kEdgesPerThread; r++) {
        const uint32_t j = tid + r * kBlock;
        if (j < ne) {
            const uint64_t f = mix64(hv[r] ^ kCE);
            if (f != 0 && global_region_insert(a.hub_tab, base, span, f)) sum += f;
        }
    }
    const uint64_t bsum = block_sum_u64(sum, S.red64);
    if (tid == 0) {
        __hip_atomic_fetch_add(&a.hub_acc[hi], bsum, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        const uint32_t prev =
            __hip_atomic_fetch_add(&a.hub_done[hi], 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
        const uint32_t last = (prev + 1 == a.hub_nchunks[hi]) ? 1u : 0u;
        S.ctl[3] = last;
        if (last) {
            const uint64_t acc = __hip_atomic_load(&a.hub_acc[hi], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
            const uint64_t h = mix64(a.t[v] ^ mix64(kCS + acc));
            a.h_next[v] = h;
            add_block_count(a.stripes, a.k, count_insert(a.tab_ins, a.tab_mask, a.zflag_ins, h));
            a.hub_acc[hi] = 0;
            a.hub_done[hi] = 0;
        }
    }
    __syncthreads();
    if (S.ctl[3]) {
        // every chunk of this hub has inserted: clear its region for the next launch
        for (uint32_t j = tid; j < span; j += kBlock) a.hub_tab[base + j] = 0;
    }
}

template <typename LabT>
__global__ void __launch_bounds__(kBlock) k_iterate(IterArgs a) {
    __shared__ IterShared S;
    const uint32_t tid = threadIdx.x;
    // ---- stop test on the previous launch's block count
    if (tid < 64) {
        uint32_t c = a.stripes[((a.k - 1) & (kStripeRing - 1)) * kStripes + tid];
        c = wave_sum_u32(c);
        if (tid == 0) {
            uint32_t ex = *reinterpret_cast<volatile uint32_t*>(&a.status->done);
            if (!ex) {
                if (blockIdx.x == 0) a.totals[a.k - 1] = c;
                const uint32_t fix = (a.k >= 2 && c == a.totals[a.k - 2]) ? 1u : 0u;
                if ((a.stop && fix) || a.k > a.k_max) {
                    ex = 1;
                    if (blockIdx.x == 0) {
                        a.status->k_done = a.k - 1;
                        a.status->fixpoint = fix;
                        a.status->done = 1;
                    }
                }
            }
            S.ctl[0] = ex;
        }
    }
    __syncthreads();
    if (S.ctl[0]) return;

    // ---- recycle the counters and the count table of iteration k+1
    if (blockIdx.x == 0) {
        if (tid < kStripes) a.stripes[((a.k + 1) & (kStripeRing - 1)) * kStripes + tid] = 0;
        if (tid == 0) *a.zflag_clr = 0;
    }
    {
        const uint64_t cap = static_cast<uint64_t>(a.tab_mask) + 1;
        const uint64_t per = (cap + gridDim.x - 1) / gridDim.x;
        const uint64_t lo = per * blockIdx.x;
        const uint64_t hi = min(cap, lo + per);
        for (uint64_t j = lo + tid; j < hi; j += kBlock) a.tab_clr[j] = 0;
    }

    if (blockIdx.x < a.n_hub_chunks)
        hub_chunk_block<LabT>(a, blockIdx.x, S);
    else if (blockIdx.x - a.n_hub_chunks < a.n_tiles)
        tile_block<LabT>(a, blockIdx.x - a.n_hub_chunks, S);
}

}  // namespace

void alloc_run_buffers(const Staged& g, uint32_t k_max, bool stop, RunBuffers& rb, Arena& arena,
                       hipStream_t s) {
    const uint32_t n = g.n;
    rb.t = arena.alloc<uint64_t>(n);
    rb.h[0] = arena.alloc<uint64_t>(n);
    rb.h[1] = arena.alloc<uint64_t>(n);
    const uint32_t cap = std::max<uint32_t>(next_pow2(static_cast<uint64_t>(n) + n / 2 + 1), 64);
    rb.tab_mask = cap - 1;
    // one allocation of 2*cap keys; finalize reuses it as cap 16-byte slots
    rb.tab[0] = arena.alloc<uint64_t>(2 * static_cast<size_t>(cap) + 2);
    rb.tab[1] = rb.tab[0] + cap;
    rb.zflag = arena.alloc<uint32_t>(2);
    rb.stripes = arena.alloc<uint32_t>(kStripeRing * kStripes);
    // k_done <= max(n, 1) when stopping at the fixpoint; the launch after
    // k_done writes totals[k_done]
    const uint64_t kc = stop ? std::min<uint64_t>(k_max, static_cast<uint64_t>(n) + 1) : k_max;
    rb.k_cap = static_cast<uint32_t>(kc) + 2;
    rb.totals = arena.alloc<uint32_t>(rb.k_cap);
    rb.hub_acc = arena.alloc<uint64_t>(g.n_hubs + 1);
    rb.hub_done = arena.alloc<uint32_t>(g.n_hubs + 1);
    rb.hub_tab = arena.alloc<uint64_t>(g.hub_tab_slots + 1);
    rb.status = arena.alloc<RunStatus>(1);
    hip_check(hipMemsetAsync(rb.tab[0], 0, (2 * static_cast<size_t>(cap) + 2) * 8, s), "clear tables");
    hip_check(hipMemsetAsync(rb.zflag, 0, 2 * 4, s), "clear flags");
    hip_check(hipMemsetAsync(rb.stripes, 0, kStripeRing * kStripes * 4, s), "clear stripes");
    hip_check(hipMemsetAsync(rb.totals, 0, rb.k_cap * 4, s), "clear totals");
    hip_check(hipMemsetAsync(rb.hub_acc, 0, (g.n_hubs + 1) * 8, s), "clear hub acc");
    hip_check(hipMemsetAsync(rb.hub_done, 0, (g.n_hubs + 1) * 4, s), "clear hub done");
    hip_check(hipMemsetAsync(rb.hub_tab, 0, (g.hub_tab_slots + 1) * 8, s), "clear hub table");
    hip_check(hipMemsetAsync(rb.status, 0, sizeof(RunStatus), s), "clear status");
}

void launch_type_hash(const Staged& g, const RunBuffers& rb, bool untyped, hipStream_t s) {
    const uint32_t n = g.n;
    k_type_hash<<<std::max<uint32_t>(ceil_div(n, kBlock), 1), kBlock, 0, s>>>(
        g.type_off, g.type_ids, g.alive, n, untyped ? 1 : 0, rb.t, rb.h[0], rb.tab[0], rb.tab_mask,
        rb.zflag + 0, rb.stripes);
    hip_check(hipGetLastError(), "type hash launch");
}

void launch_iteration(const Staged& g, const RunBuffers& rb, uint32_t k, uint32_t k_max,
                      bool stop, hipStream_t s) {
    IterArgs a;
    a.row_off = g.row_off;
    a.tgt = g.tgt;
    a.lab = g.lab;
    a.t = rb.t;
    a.salt = g.salt;
    a.h_prev = rb.h[(k - 1) & 1];
    a.h_next = rb.h[k & 1];
    a.alive = g.alive;
    a.tile_v0 = g.tile_v0;
    a.tile_v1 = g.tile_v1;
    a.hc_hub = g.hc_hub;
    a.hc_e0 = g.hc_e0;
    a.hub_v = g.hub_v;
    a.hub_nchunks = g.hub_nchunks;
    a.hub_tab_off = g.hub_tab_off;
    a.hub_tab = rb.hub_tab;
    a.hub_acc = rb.hub_acc;
    a.hub_done = rb.hub_done;
    a.tab_ins = rb.tab[k & 1];
    a.tab_clr = rb.tab[(k + 1) & 1];
    a.zflag_ins = rb.zflag + (k & 1);
    a.zflag_clr = rb.zflag + ((k + 1) & 1);
    a.stripes = rb.stripes;
    a.totals = rb.totals;
    a.status = rb.status;
    a.n_tiles = g.n_tiles;
    a.n_hub_chunks = g.n_hub_chunks;
    a.tab_mask = rb.tab_mask;
    a.k = k;
    a.k_max = k_max;
    a.stop = stop ? 1u : 0u;
    const uint32_t grid = std::max<uint32_t>(g.n_hub_chunks + g.n_tiles, 1);
    if (g.label_bytes == 2)
        k_iterate<uint16_t><<<grid, kBlock, 0, s>>>(a);
    else
        k_iterate<uint32_t><<<grid, kBlock, 0, s>>>(a);
    hip_check(hipGetLastError(), "iteration launch");
}

}  // namespace bsim
