// bsim_device.h -- device helpers shared by the refinement and finalize
// kernels: wave64 reductions, the open-addressing count table, and the tile
// layout (which vertex of a tile owns each edge).
#pragma once

#include "bsim_internal.h"

namespace bsim {

__device__ __forceinline__ uint32_t lane_id() { return threadIdx.x & 63; }

__device__ __forceinline__ uint64_t shfl_xor_u64(uint64_t x, int d) {
    uint32_t lo = static_cast<uint32_t>(__shfl_xor(static_cast<int>(static_cast<uint32_t>(x)), d, 64));
    uint32_t hi = static_cast<uint32_t>(__shfl_xor(static_cast<int>(static_cast<uint32_t>(x >> 32)), d, 64));
    return (static_cast<uint64_t>(hi) << 32) | lo;
}

__device__ __forceinline__ uint32_t wave_sum_u32(uint32_t x) {
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) x += static_cast<uint32_t>(__shfl_xor(static_cast<int>(x), d, 64));
    return x;
}

__device__ __forceinline__ uint64_t wave_sum_u64(uint64_t x) {
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) x += shfl_xor_u64(x, d);
    return x;
}

// Sum over the block; valid in thread 0.  `red` needs kBlock/64 entries.
__device__ __forceinline__ uint32_t block_sum_u32(uint32_t x, uint32_t* red) {
    x = wave_sum_u32(x);
    if (lane_id() == 0) red[threadIdx.x >> 6] = x;
    __syncthreads();
    uint32_t t = 0;
    if (threadIdx.x == 0)
        for (int i = 0; i < kBlock / 64; i++) t += red[i];
    __syncthreads();
    return t;
}

__device__ __forceinline__ uint64_t block_sum_u64(uint64_t x, uint64_t* red) {
    x = wave_sum_u64(x);
    if (lane_id() == 0) red[threadIdx.x >> 6] = x;
    __syncthreads();
    uint64_t t = 0;
    if (threadIdx.x == 0)
        for (int i = 0; i < kBlock / 64; i++) t += red[i];
    __syncthreads();
    return t;
}

// Insert hash h into a key-only open-addressing table (0 = empty slot,
// capacity mask+1 > number of keys).  The hash 0 itself is tracked by a flag.
// Returns 1 if h was not present before.
//
// Many vertices share a hash (e.g. every isolated vertex with the same type
// set), so a slot is read before it is CASed: within one launch a slot only
// changes from 0 to a key, so a plain read either sees the final key (no
// atomic needed) or a possibly stale 0 that the CAS then resolves.  Without
// this, all vertices of a large block serialize on one address.
__device__ __forceinline__ uint32_t count_insert(uint64_t* tab, uint32_t mask, uint32_t* zflag,
                                                 uint64_t h) {
    if (h == 0) {
        if (*reinterpret_cast<volatile uint32_t*>(zflag)) return 0u;
        return atomicExch(zflag, 1u) == 0u ? 1u : 0u;
    }
    uint32_t slot = static_cast<uint32_t>(h) & mask;
    for (;;) {
        uint64_t cur = tab[slot];
        if (cur == h) return 0u;
        if (cur == 0) {
            unsigned long long old = atomicCAS(reinterpret_cast<unsigned long long*>(tab + slot), 0ull,
                                               static_cast<unsigned long long>(h));
            if (old == 0ull) return 1u;
            if (old == h) return 0u;
        }
        slot = (slot + 1) & mask;
    }
}

// Insert a nonzero key into an LDS open-addressing region; returns 1 if it
// was not present.  Same read-before-CAS rule as count_insert.
// Current value of an LDS table slot other lanes may be writing.  A relaxed
// atomic load (a volatile one would keep the generic address space and
// compile to a flat load, which also waits on every global load in flight).
__device__ __forceinline__ uint64_t lds_peek(uint64_t* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

__device__ __forceinline__ uint32_t lds_insert(uint64_t* tab, uint32_t slot, uint32_t base,
                                               uint32_t end, uint64_t f) {
    for (;;) {
        uint64_t cur = lds_peek(&tab[slot]);
        if (cur == f) return 0u;
        if (cur == 0) {
            unsigned long long old = atomicCAS(reinterpret_cast<unsigned long long*>(&tab[slot]), 0ull,
                                               static_cast<unsigned long long>(f));
            if (old == 0ull) return 1u;
            if (old == f) return 0u;
        }
        if (++slot == end) slot = base;
    }
}

// Insert a nonzero key into an LDS table of `slots` slots by double hashing:
// after `slot` (already tried), probe slot + step, slot + 2 step, ... mod
// slots.  With slots prime and 0 < step < slots the sequence visits every
// slot, so a table with a free slot always ends the loop: 1 = inserted,
// 0 = already present.
__device__ __forceinline__ uint32_t lds_insert_step(uint64_t* tab, uint32_t slot, uint32_t step, uint32_t slots,
                                                    uint64_t f) {
    for (;;) {
        slot += step;
        if (slot >= slots) slot -= slots;
        uint64_t cur = lds_peek(&tab[slot]);
        if (cur == f) return 0u;
        if (cur == 0) {
            unsigned long long old = atomicCAS(reinterpret_cast<unsigned long long*>(&tab[slot]), 0ull,
                                               static_cast<unsigned long long>(f));
            if (old == 0ull) return 1u;
            if (old == f) return 0u;
        }
    }
}

// Insert a nonzero key into an LDS table of `slots` slots, probing at most
// `slots` positions: 1 = inserted, 0 = already present, 2 = table full.
__device__ __forceinline__ uint32_t lds_insert_bounded(uint64_t* tab, uint32_t slot, uint32_t slots,
                                                       uint64_t f) {
    for (uint32_t step = 0; step < slots; step++) {
        uint64_t cur = lds_peek(&tab[slot]);
        if (cur == f) return 0u;
        if (cur == 0) {
            unsigned long long old = atomicCAS(reinterpret_cast<unsigned long long*>(&tab[slot]), 0ull,
                                               static_cast<unsigned long long>(f));
            if (old == 0ull) return 1u;
            if (old == f) return 0u;
        }
        if (++slot == slots) slot = 0;
    }
    return 2u;
}

__device__ __forceinline__ void add_block_count(uint32_t* stripes, uint32_t k, uint32_t c) {
    if (c) atomicAdd(&stripes[(k & (kStripeRing - 1)) * kStripes + (blockIdx.x & (kStripes - 1))], c);
}

// Tile layout in LDS: s_off[i] = first edge of local vertex i relative to
// the tile's first edge (i = 0..nv), s_seg[j] = local vertex owning edge j.
// Requires nv <= kTileMaxVerts and ne = s_off[nv] < kTileMaxEdges.
// s_seg must be 8-byte aligned.  Ends with a barrier.
__device__ inline void tile_segments(uint32_t nv, const uint32_t* s_off, uint8_t* s_seg,
                                     uint32_t* s_red) {
    constexpr uint32_t kWords = kTileMaxEdges / 8;  // owner-map words, one per thread
    const uint32_t tid = threadIdx.x;
    uint64_t* seg64 = reinterpret_cast<uint64_t*>(s_seg);
    // zero the owner map, then mark each non-empty segment start
    if (tid < kWords) seg64[tid] = 0;
    __syncthreads();
    for (uint32_t i = tid; i < nv; i += kBlock)
        if (s_off[i + 1] > s_off[i]) s_seg[s_off[i]] = static_cast<uint8_t>(i);
    __syncthreads();
    // inclusive max-scan over the owner map: thread t owns bytes 8t..8t+7
    // (threads past the map scan zeros, which leave a max unchanged)
    const uint64_t word = tid < kWords ? seg64[tid] : 0;
    uint32_t run = 0;
#pragma unroll
    for (int r = 0; r < 8; r++) run = max(run, static_cast<uint32_t>((word >> (8 * r)) & 0xFF));
    uint32_t incl = run;
    const uint32_t lane = lane_id();
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        uint32_t y = static_cast<uint32_t>(__shfl_up(static_cast<int>(incl), d, 64));
        if (lane >= static_cast<uint32_t>(d)) incl = max(incl, y);
    }
    uint32_t excl = static_cast<uint32_t>(__shfl_up(static_cast<int>(incl), 1, 64));
    if (lane == 0) excl = 0;
    if (lane == 63) s_red[tid >> 6] = incl;
    __syncthreads();
    for (uint32_t wv = 0; wv < (tid >> 6); wv++) excl = max(excl, s_red[wv]);
    uint64_t out = 0;
    uint32_t cur = excl;
#pragma unroll
    for (int r = 0; r < 8; r++) {
        cur = max(cur, static_cast<uint32_t>((word >> (8 * r)) & 0xFF));
        out |= static_cast<uint64_t>(cur) << (8 * r);
    }
    if (tid < kWords) seg64[tid] = out;
    __syncthreads();
}

static_assert(kTileMaxEdges % 8 == 0 && kTileMaxEdges / 8 <= kBlock,
              "tile_segments keeps one 8-byte owner-map word per thread");
static_assert(kTileMaxVerts <= 256, "owner map stores vertex indices in one byte");

}  // namespace bsim
