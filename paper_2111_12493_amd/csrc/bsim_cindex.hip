// bsim_cindex.hip -- the class index of a resident state (a9): per level j,
// the classes of the level as a hash table keyed by (class at level j-1,
// h^j), each with its member count, and the class of every vertex.
//
// Sec. 3.2 keeps summaries up to date through a vertex hash index whose
// entries link vertices to the summary elements that describe them, with
// a summary element removed once no vertex links to it; this is that index
// for the refinement's classes.  The classes of level j refine those of
// level j-1 by h^j (the pair rule of Sec. 2.5), so a class is identified
// by (its level j-1 class, h^j), and n_j is the number of keys with at
// least one member.  An update re-keys only the vertices whose h^j or
// level j-1 class changed: each leaves its old class (count - 1; a count
// reaching 0 is a class gone) and joins the class of its new key (found,
// or claimed; a count leaving 0 is a class (re)born).  Keys are never
// removed, so probe chains stay intact; a table whose claimed slots pass a
// load limit is rebuilt from scratch.
//
// Table layout: slot s is the pair (word, key) at slot[2 s], slot[2 s + 1]:
// word = 0 (empty) or (pc << 32) | owner, pc = level j-1 class + 1 (1 at
// level 0), key = the key's hash, so one probe reads one 16-byte line;
// cnt[s] = members.  A vertex's class id at level j is the slot of its key.
//
// Rebuild (all vertices): one insertion pass over a cleared table; the
// member counts are left to k_ci_count, run when an update first needs them.  The
// vertex that claims a slot writes the key after its CAS on the word; a
// prober that finds the word already set but the key still 0 compares
// against the owner's hash in the level array instead (immutable during
// the pass, and the key's source).  Incremental update (a list
// of vertices): a read-only probe; the misses are de-duplicated in a small
// temporary table; one representative per new key claims an empty slot in
// a later kernel (no reader probes concurrently, and the keys are distinct
// and absent, so a claim never needs to match); then every vertex moves.
#include "bsim_append.h"

namespace bsim {

namespace {

__device__ __forceinline__ uint64_t ci_shfl_u64(uint64_t x, uint32_t src) {
    const uint32_t lo = static_cast<uint32_t>(__shfl(static_cast<int>(static_cast<uint32_t>(x)), static_cast<int>(src), 64));
    const uint32_t hi = static_cast<uint32_t>(__shfl(static_cast<int>(static_cast<uint32_t>(x >> 32)), static_cast<int>(src), 64));
    return (static_cast<uint64_t>(hi) << 32) | lo;
}

__device__ __forceinline__ uint32_t ci_home(uint32_t pc, uint64_t h, uint32_t mask) {
    return (static_cast<uint32_t>(h) ^ static_cast<uint32_t>(mix64(pc) >> 32)) & mask;
}

// Class slot of key (pc, h) in a table whose keys are checked against
// keys[owner] (the rebuild's level array, or the temporary table's own key
// array), claiming an empty slot for it when absent (*founded = 1).
__device__ uint32_t ci_join_owner(uint64_t* word, uint32_t mask, const uint64_t* __restrict__ keys, uint32_t pc,
                                  uint64_t h, uint32_t owner, uint32_t* founded) {
    const uint64_t mine = (static_cast<uint64_t>(pc) << 32) | owner;
    uint32_t slot = ci_home(pc, h, mask);
    *founded = 0;
    for (;;) {
        uint64_t cur = word[slot];  // a stale 0 only costs the CAS
        if (cur == 0) {
            cur = atomicCAS(reinterpret_cast<unsigned long long*>(&word[slot]), 0ull,
                            static_cast<unsigned long long>(mine));
            if (cur == 0) {
                *founded = 1;
                return slot;
            }
        }
        if ((cur >> 32) == pc && keys[static_cast<uint32_t>(cur)] == h) return slot;
        slot = (slot + 1) & mask;
    }
}

// The slot of key (pc, h) in a level table during a rebuild, claiming an
// empty one for it when absent (*founded = 1); keys[owner] is the owner's
// hash for a slot whose key is not written yet (see above).
__device__ uint32_t ci_join_level(const CiLevel& L, const uint64_t* __restrict__ keys, uint32_t pc, uint64_t h,
                                  uint32_t owner, uint32_t* founded) {
    const uint64_t mine = (static_cast<uint64_t>(pc) << 32) | owner;
    uint32_t slot = ci_home(pc, h, L.mask);
    *founded = 0;
    for (;;) {
        const ulonglong2 sk = *reinterpret_cast<const ulonglong2*>(&L.slot[2ull * slot]);  // a stale pair only costs the CAS
        uint64_t cur = sk.x;
        uint64_t key = sk.y;
        if (cur == 0) {
            cur = atomicCAS(reinterpret_cast<unsigned long long*>(&L.slot[2ull * slot]), 0ull,
                            static_cast<unsigned long long>(mine));
            if (cur == 0) {
                L.slot[2ull * slot + 1] = h;
                *founded = 1;
                return slot;
            }
            key = 0;  // claimed meanwhile: its key may not be written yet
        }
        if ((cur >> 32) == pc) {
            if (key == 0) key = keys[static_cast<uint32_t>(cur)];
            if (key == h) return slot;
        }
        slot = (slot + 1) & L.mask;
    }
}

// Rebuild: every alive vertex joins the class of (its level j-1 class, h^j).
// Lanes of a wave with one key (every vertex without out-edges of one type
// set and class, say) reach the table once.
__global__ void __launch_bounds__(kBlock) k_ci_build(CiLevel L, const uint32_t* __restrict__ cid_prev,
                                                     const uint64_t* __restrict__ h,
                                                     const uint8_t* __restrict__ alive, uint32_t n,
                                                     uint64_t* __restrict__ ctr) {
    __shared__ uint32_t s_red[kBlock / 64];
    const uint32_t v = blockIdx.x * kBlock + threadIdx.x;
    const uint32_t lane = lane_id();
    bool part = false;
    uint32_t pc = 0;
    uint64_t hv = 0;
    if (v < n) {
        if (alive && !alive[v]) {
            L.cid[v] = kNoClass;
        } else {
            part = true;
            pc = cid_prev ? cid_prev[v] + 1 : 1u;
            hv = h[v];
        }
    }
    // group the lanes by key, one insertion per group
    uint32_t leader_of = lane;
    bool pending = part;
    for (;;) {
        const uint64_t ball = __ballot(pending);
        if (!ball) break;
        const uint32_t leader = static_cast<uint32_t>(__ffsll(static_cast<long long>(ball)) - 1);
        const uint64_t lh = ci_shfl_u64(hv, leader);
        const uint32_t lp = static_cast<uint32_t>(__shfl(static_cast<int>(pc), static_cast<int>(leader), 64));
        if (pending && hv == lh && pc == lp) {
            leader_of = leader;
            pending = false;
        }
    }
    const bool lead = part && leader_of == lane;
    uint32_t slot = 0, founded = 0;
    if (lead) slot = ci_join_level(L, h, pc, hv, v, &founded);
    slot = static_cast<uint32_t>(__shfl(static_cast<int>(slot), static_cast<int>(leader_of), 64));
    if (part) L.cid[v] = slot;
    const uint32_t c = block_sum_u32(founded, s_red);
    if (threadIdx.x == 0 && c) {
        atomicAdd(reinterpret_cast<unsigned long long*>(&ctr[0]), static_cast<unsigned long long>(c));
        atomicAdd(reinterpret_cast<unsigned long long*>(&ctr[1]), static_cast<unsigned long long>(c));
    }
}

// Member counts of a rebuilt level, from the class ids (cnt cleared since
// the rebuild): every vertex with a class counts, lanes of a wave with one
// class add once.
__global__ void __launch_bounds__(kBlock) k_ci_count(CiLevel L, uint32_t n) {
    const uint32_t v = blockIdx.x * kBlock + threadIdx.x;
    const uint32_t lane = lane_id();
    const uint32_t c = v < n ? L.cid[v] : kNoClass;
    const bool part = c != kNoClass;
    bool pending = part;
    for (;;) {
        const uint64_t ball = __ballot(pending);
        if (!ball) break;
        const uint32_t leader = static_cast<uint32_t>(__ffsll(static_cast<long long>(ball)) - 1);
        const uint32_t lc = static_cast<uint32_t>(__shfl(static_cast<int>(c), static_cast<int>(leader), 64));
        const uint64_t same = __ballot(pending && c == lc);
        if (lane == leader) atomicAdd(&L.cnt[lc], static_cast<uint32_t>(__popcll(same)));
        if (c == lc) pending = false;
    }
}

// The update's vertex list: candidates of list a (those with flag[v] ==
// ftag when flag is given) and every vertex of list b, each once (dmark[v]
// takes dtag).  Counts na / nb are read from device memory when na_dev /
// nb_dev are given.
__global__ void __launch_bounds__(kBlock) k_ci_dlist(const uint32_t* __restrict__ a, uint32_t na,
                                                     const uint32_t* __restrict__ na_dev,
                                                     const uint32_t* __restrict__ flag, uint32_t ftag,
                                                     const uint32_t* __restrict__ b, uint32_t nb,
                                                     const uint32_t* __restrict__ nb_dev, uint32_t* __restrict__ dmark,
                                                     uint32_t dtag, uint32_t* __restrict__ d, uint32_t* __restrict__ nd) {
    __shared__ uint32_t s_wave[kBlock / 64 + 1];
    const uint32_t ca = na_dev ? *na_dev : na, cb = nb_dev ? *nb_dev : nb;
    const uint64_t total = static_cast<uint64_t>(ca) + cb;
    for (uint64_t base = static_cast<uint64_t>(blockIdx.x) * kBlock; base < total;
         base += static_cast<uint64_t>(gridDim.x) * kBlock) {  // the same trip count in every thread of a block
        const uint64_t i = base + threadIdx.x;
        bool take = false;
        uint32_t v = 0;
        if (i < total) {
            v = i < ca ? a[i] : b[i - ca];
            const bool cand = i >= ca || !flag || flag[v] == ftag;
            take = cand && atomicExch(&dmark[v], dtag) != dtag;
        }
        const uint32_t pos = block_reserve(take, nd, s_wave);
        if (take) d[pos] = v;
    }
}

// Probe: the class slot of every listed vertex's new key, or a pending
// entry when the key is new (dead vertices: no class).
__global__ void __launch_bounds__(kBlock) k_ci_probe(CiLevel L, const uint32_t* __restrict__ cid_prev,
                                                     const uint64_t* __restrict__ h,
                                                     const uint8_t* __restrict__ alive,
                                                     const uint32_t* __restrict__ d, uint32_t nd,
                                                     uint32_t* __restrict__ ns, uint32_t* __restrict__ pend,
                                                     uint32_t* __restrict__ pend_pc, uint64_t* __restrict__ pend_h,
                                                     uint32_t* __restrict__ n_pend, uint32_t* __restrict__ err) {
    __shared__ uint32_t s_wave[kBlock / 64 + 1];
    const uint32_t i = blockIdx.x * kBlock + threadIdx.x;
    bool miss = false;
    uint32_t pc = 0;
    uint64_t hv = 0;
    if (i < nd) {
        const uint32_t v = d[i];
        if (alive && !alive[v]) {
            ns[i] = kNoClass;
        } else {
            pc = cid_prev ? cid_prev[v] + 1 : 1u;
            hv = h[v];
            // the caller keeps free slots in the table; the bound only turns
            // a full table into an error instead of an endless probe
            uint32_t slot = ci_home(pc, hv, L.mask);
            uint32_t step = 0;
            for (;; step++) {
                if (step > L.mask) {
                    atomicOr(err, 1u);
                    ns[i] = kNoClass;
                    break;
                }
                const ulonglong2 sk = *reinterpret_cast<const ulonglong2*>(&L.slot[2ull * slot]);
                if (sk.x == 0) {
                    miss = true;
                    break;
                }
                if ((sk.x >> 32) == pc && sk.y == hv) {
                    ns[i] = slot;
                    break;
                }
                slot = (slot + 1) & L.mask;
            }
        }
    }
    const uint32_t p = block_reserve(miss, n_pend, s_wave);
    if (miss) {
        pend[p] = i;
        pend_pc[p] = pc;
        pend_h[p] = hv;
    }
}

// The pending keys, de-duplicated in a temporary table: prep[p] = the
// pending entry that represents p's key.
__global__ void __launch_bounds__(kBlock) k_ci_dedupe(uint64_t* tmp, uint32_t tmask,
                                                      const uint32_t* __restrict__ pend_pc,
                                                      const uint64_t* __restrict__ pend_h, uint32_t np,
                                                      uint32_t* __restrict__ prep) {
    const uint32_t p = blockIdx.x * kBlock + threadIdx.x;
    if (p >= np) return;
    uint32_t founded = 0;
    const uint32_t slot = ci_join_owner(tmp, tmask, pend_h, pend_pc[p], pend_h[p], p, &founded);
    prep[p] = founded ? p : static_cast<uint32_t>(tmp[slot]);
}

// One claim per new key: an empty slot of the level's table.  The keys are
// distinct and absent, so every occupied slot on the way belongs to
// another key.
__global__ void __launch_bounds__(kBlock) k_ci_claim(CiLevel L, const uint32_t* __restrict__ pend_pc,
                                                     const uint64_t* __restrict__ pend_h,
                                                     const uint32_t* __restrict__ prep, uint32_t np,
                                                     uint32_t* __restrict__ rslot, uint64_t* __restrict__ ctr,
                                                     uint32_t* __restrict__ err) {
    __shared__ uint32_t s_red[kBlock / 64];
    const uint32_t p = blockIdx.x * kBlock + threadIdx.x;
    uint32_t claimed = 0;
    if (p < np && prep[p] == p) {
        const uint32_t pc = pend_pc[p];
        const uint64_t hv = pend_h[p];
        const uint64_t mine = (static_cast<uint64_t>(pc) << 32) | 0xFFFFFFFFu;
        uint32_t slot = ci_home(pc, hv, L.mask);
        uint32_t step = 0;
        for (;; step++) {
            if (step > L.mask) {  // full: an error, see k_ci_probe
                atomicOr(err, 1u);
                slot = kNoClass;
                break;
            }
            if (L.slot[2ull * slot] == 0 &&
                atomicCAS(reinterpret_cast<unsigned long long*>(&L.slot[2ull * slot]), 0ull,
                          static_cast<unsigned long long>(mine)) == 0ull)
                break;
            slot = (slot + 1) & L.mask;
        }
        if (slot != kNoClass) {
            L.slot[2ull * slot + 1] = hv;
            claimed = 1;
        }
        rslot[p] = slot;
    }
    const uint32_t c = block_sum_u32(claimed, s_red);
    if (threadIdx.x == 0 && c) atomicAdd(reinterpret_cast<unsigned long long*>(&ctr[1]), static_cast<unsigned long long>(c));
}

__global__ void __launch_bounds__(kBlock) k_ci_assign(const uint32_t* __restrict__ pend,
                                                      const uint32_t* __restrict__ prep,
                                                      const uint32_t* __restrict__ rslot, uint32_t np,
                                                      uint32_t* __restrict__ ns) {
    const uint32_t p = blockIdx.x * kBlock + threadIdx.x;
    if (p < np) ns[pend[p]] = rslot[prep[p]];
}

// Move every listed vertex to its new class; the vertices whose class
// changed go to list q (they re-key at the next level).
__global__ void __launch_bounds__(kBlock) k_ci_move(CiLevel L, const uint32_t* __restrict__ d, uint32_t nd,
                                                    const uint32_t* __restrict__ ns, uint64_t* __restrict__ ctr,
                                                    uint32_t* __restrict__ q, uint32_t* __restrict__ nq) {
    __shared__ int32_t s_red[kBlock / 64];
    __shared__ uint32_t s_wave[kBlock / 64 + 1];
    const uint32_t i = blockIdx.x * kBlock + threadIdx.x;
    const uint32_t lane = lane_id();
    int32_t delta = 0;
    bool moved = false;
    uint32_t v = 0;
    if (i < nd) {
        v = d[i];
        const uint32_t old = L.cid[v], nw = ns[i];
        if (old != nw) {
            if (old != kNoClass && atomicSub(&L.cnt[old], 1u) == 1u) delta--;
            if (nw != kNoClass && atomicAdd(&L.cnt[nw], 1u) == 0u) delta++;
            L.cid[v] = nw;
            moved = true;
        }
    }
    const uint32_t pos = block_reserve(moved, nq, s_wave);
    if (moved) q[pos] = v;
    // block sum of the signed class-count changes
    int32_t x = delta;
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) x += __shfl_xor(x, o, 64);
    if (lane == 0) s_red[threadIdx.x >> 6] = x;
    __syncthreads();
    if (threadIdx.x == 0) {
        int32_t t = 0;
        for (int w = 0; w < kBlock / 64; w++) t += s_red[w];
        if (t) atomicAdd(reinterpret_cast<unsigned long long*>(&ctr[0]),
                         static_cast<unsigned long long>(static_cast<int64_t>(t)));
    }
}

}  // namespace

void ci_rebuild(const CiLevel& L, uint64_t cap, const uint32_t* cid_prev, const uint64_t* h, const uint8_t* alive,
                uint32_t n, uint64_t* ctr, hipStream_t s) {
    hip_check(hipMemsetAsync(L.slot, 0, 2 * cap * sizeof(uint64_t), s), "class index clear");
    hip_check(hipMemsetAsync(L.cnt, 0, cap * sizeof(uint32_t), s), "class index counts");
    hip_check(hipMemsetAsync(ctr, 0, 2 * sizeof(uint64_t), s), "class index counters");
    if (n) k_ci_build<<<ceil_div(n, kBlock), kBlock, 0, s>>>(L, cid_prev, h, alive, n, ctr);
    hip_check(hipGetLastError(), "class index rebuild");
}

void ci_count(const CiLevel& L, uint32_t n, hipStream_t s) {
    if (n) k_ci_count<<<ceil_div(n, kBlock), kBlock, 0, s>>>(L, n);
    hip_check(hipGetLastError(), "class index counts");
}

void ci_list(const uint32_t* a, uint32_t na, const uint32_t* na_dev, const uint32_t* flag, uint32_t ftag,
             const uint32_t* b, uint32_t nb, const uint32_t* nb_dev, uint32_t* dmark, uint32_t dtag, uint32_t* d,
             uint32_t* nd, uint32_t grid, hipStream_t s) {
    hip_check(hipMemsetAsync(nd, 0, 4, s), "class list count");
    k_ci_dlist<<<std::max<uint32_t>(grid, 1), kBlock, 0, s>>>(a, na, na_dev, flag, ftag, b, nb, nb_dev, dmark, dtag,
                                                               d, nd);
    hip_check(hipGetLastError(), "class list");
}

void ci_update(const CiLevel& L, const uint32_t* cid_prev, const uint64_t* h, const uint8_t* alive,
               const uint32_t* d, uint32_t nd, uint64_t* ctr, uint32_t* q, uint32_t* nq, uint32_t* err,
               uint32_t* host_word, Arena& arena, hipStream_t s) {
    hip_check(hipMemsetAsync(nq, 0, 4, s), "moved count");
    if (nd == 0) return;
    uint32_t* ns = arena.alloc<uint32_t>(nd);
    uint32_t* pend = arena.alloc<uint32_t>(nd);
    uint32_t* pend_pc = arena.alloc<uint32_t>(nd);
    uint64_t* pend_h = arena.alloc<uint64_t>(nd);
    uint32_t* n_pend = arena.alloc<uint32_t>(1);
    hip_check(hipMemsetAsync(n_pend, 0, 4, s), "pending count");
    const uint32_t g = ceil_div(nd, kBlock);
    k_ci_probe<<<g, kBlock, 0, s>>>(L, cid_prev, h, alive, d, nd, ns, pend, pend_pc, pend_h, n_pend, err);
    hip_check(hipMemcpyAsync(host_word, n_pend, 4, hipMemcpyDeviceToHost, s), "pending count");
    hip_check(hipStreamSynchronize(s), "pending sync");
    const uint32_t np = *host_word;
    if (np) {
        const uint64_t tcap = split_table_slots(np);
        uint64_t* tmp = arena.alloc<uint64_t>(tcap);
        uint32_t* prep = arena.alloc<uint32_t>(np);
        uint32_t* rslot = arena.alloc<uint32_t>(np);
        hip_check(hipMemsetAsync(tmp, 0, tcap * sizeof(uint64_t), s), "pending table");
        const uint32_t gp = ceil_div(np, kBlock);
        k_ci_dedupe<<<gp, kBlock, 0, s>>>(tmp, static_cast<uint32_t>(tcap - 1), pend_pc, pend_h, np, prep);
        k_ci_claim<<<gp, kBlock, 0, s>>>(L, pend_pc, pend_h, prep, np, rslot, ctr, err);
        k_ci_assign<<<gp, kBlock, 0, s>>>(pend, prep, rslot, np, ns);
    }
    k_ci_move<<<g, kBlock, 0, s>>>(L, d, nd, ns, ctr, q, nq);
    hip_check(hipGetLastError(), "class index update");
}

}  // namespace bsim
