// bsim_final.hip -- finalize (a8): relabel the final hashes to dense block
// ids, count block sizes, and build the summary graph's edges.
//
// Algorithm 4 ends with FindAndMerge: vertices with equal final identifiers
// form one block.  The refinement loop already names every vertex's class
// by a representative member; block ids are numbered by first occurrence
// (the block of the smallest vertex is 0), which depends only on the
// partition:
//   1. the smallest vertex of each class (atomicMin per class);
//   2. an exclusive scan over "v is its class's smallest vertex" flags gives
//      every such vertex its block id;
//   3. every vertex takes the id of its class's smallest vertex; block sizes
//      are counted per thread block in LDS first.
// Summary edges (Sec. 2.6: edges between vertex summaries) are the distinct
// (block(v), l, block(w)) triples: packed into one 64-bit key per edge,
// sorted by an LSD radix sort over the used bits, de-duplicated and unpacked.
#include "bsim_device.h"

namespace bsim {

namespace {

// Smallest vertex of every class (classes are named by their representative).
__global__ void __launch_bounds__(kBlock) k_fin_min(const uint32_t* __restrict__ rep,
                                                    const uint8_t* __restrict__ alive, uint32_t n,
                                                    uint32_t* cmin) {
    uint32_t v = blockIdx.x * kBlock + threadIdx.x;
    if (v >= n || (alive && !alive[v])) return;
    const uint32_t r = rep[v];
    // the minimum only decreases: skip the atomic once it is below v
    if (cmin[r] > v) atomicMin(&cmin[r], v);
}

__global__ void __launch_bounds__(kBlock) k_fin_rep(const uint32_t* __restrict__ rep,
                                                    const uint8_t* __restrict__ alive, uint32_t n,
                                                    const uint32_t* __restrict__ cmin,
                                                    uint32_t* __restrict__ isrep) {
    uint32_t v = blockIdx.x * kBlock + threadIdx.x;
    if (v >= n) return;
    isrep[v] = (!alive || alive[v]) && cmin[rep[v]] == v ? 1u : 0u;
}

// Block ids, and block sizes counted in an LDS table per block of
// kIdsPerBlock vertices first, so a block holding millions of vertices
// costs one global atomic per thread block rather than one per vertex.
constexpr int kIdsPerThread = 8;
constexpr int kIdsPerBlock = kBlock * kIdsPerThread;
constexpr int kIdsSlots = 2 * kIdsPerBlock;

__global__ void __launch_bounds__(kBlock) k_fin_ids(const uint8_t* __restrict__ alive, uint32_t n,
                                                    const uint32_t* __restrict__ rep,
                                                    const uint32_t* __restrict__ cmin,
                                                    const uint32_t* __restrict__ rank,
                                                    uint32_t* __restrict__ block_ids,
                                                    uint32_t* __restrict__ sizes) {
    __shared__ uint32_t s_key[kIdsSlots];
    __shared__ uint32_t s_cnt[kIdsSlots];
    for (int i = threadIdx.x; i < kIdsSlots; i += kBlock) {
        s_key[i] = 0xFFFFFFFFu;
        s_cnt[i] = 0;
    }
    __syncthreads();
    const uint64_t base = static_cast<uint64_t>(blockIdx.x) * kIdsPerBlock;
    for (int r = 0; r < kIdsPerThread; r++) {
        const uint64_t vv = base + static_cast<uint64_t>(r) * kBlock + threadIdx.x;
        if (vv >= n) break;
        const uint32_t v = static_cast<uint32_t>(vv);
        uint32_t bid = 0xFFFFFFFFu;
        if (!alive || alive[v]) bid = rank[cmin[rep[v]]];
        block_ids[v] = bid;
        if (bid == 0xFFFFFFFFu) continue;
        uint32_t slot = (bid * 2654435761u) & (kIdsSlots - 1);
        for (;;) {
            uint32_t cur = s_key[slot];
            if (cur == 0xFFFFFFFFu) cur = atomicCAS(&s_key[slot], 0xFFFFFFFFu, bid);
            if (cur == 0xFFFFFFFFu || cur == bid) break;
            slot = (slot + 1) & (kIdsSlots - 1);
        }
        atomicAdd(&s_cnt[slot], 1u);
    }
    __syncthreads();
    for (int i = threadIdx.x; i < kIdsSlots; i += kBlock)
        if (s_cnt[i]) atomicAdd(&sizes[s_key[i]], s_cnt[i]);
}

// ------------------------------------------------------------ edge keys

struct KeyShared {
    uint32_t off[kTileMaxVerts + 1];
    uint32_t red[kBlock / 64];
    alignas(8) uint8_t seg[kTileMaxEdges];
};

template <typename LabT>
__global__ void __launch_bounds__(kBlock) k_edge_keys(
    const uint32_t* __restrict__ row_off, const uint32_t* __restrict__ tgt,
    const LabT* __restrict__ lab, const uint32_t* __restrict__ bid, const uint32_t* __restrict__ bid_dst,
    const uint32_t* __restrict__ tile_i0, const uint32_t* __restrict__ tile_i1,
    const uint32_t* __restrict__ tile_e0, const uint32_t* __restrict__ tile_e1,
    const uint32_t* __restrict__ act, uint32_t n_tiles,
    const uint32_t* __restrict__ hub_v, uint32_t n_hubs, int lb, int bb,
    uint64_t* __restrict__ keys) {
    __shared__ KeyShared S;
    const uint32_t tid = threadIdx.x;
    if (blockIdx.x < n_hubs) {
        const uint32_t v = hub_v[blockIdx.x];
        const uint64_t src = static_cast<uint64_t>(bid[v]) << (lb + bb);
        for (uint32_t e = row_off[v] + tid; e < row_off[v + 1]; e += kBlock)
            keys[e] = src | (static_cast<uint64_t>(lab[e]) << bb) | bid_dst[tgt[e]];
        return;
    }
    const uint32_t tile = blockIdx.x - n_hubs;
    if (tile >= n_tiles) return;
    const uint32_t i0 = tile_i0[tile], nv = tile_i1[tile] - i0;
    const uint32_t ebase = tile_e0[tile];
    const uint32_t ne = tile_e1[tile] - ebase;
    for (uint32_t i = tid; i < nv; i += kBlock) S.off[i] = row_off[act[i0 + i]] - ebase;
    if (tid == 0) S.off[nv] = ne;
    __syncthreads();
    tile_segments(nv, S.off, S.seg, S.red);
    for (uint32_t j = tid; j < ne; j += kBlock) {
        const uint32_t e = ebase + j;
        const uint32_t v = act[i0 + S.seg[j]];
        keys[e] = (static_cast<uint64_t>(bid[v]) << (lb + bb)) |
                  (static_cast<uint64_t>(lab[e]) << bb) | bid_dst[tgt[e]];
    }
}

// ------------------------------------------------------------ radix sort
//
// LSD radix sort of 64-bit keys, 8 bits per pass.  Each pass: per-block digit
// histograms (digit-major, so one exclusive scan yields every block's output
// offset per digit), then a stable scatter that ranks equal digits by wave
// ballots (8 ballots isolate the lanes with the same digit).

// 16 keys per thread: a tile of 4,096 keys leaves about 16 keys per digit
// run, so the scatter writes runs of about 128 bytes
constexpr int kSortItems = 16;
constexpr int kSortTile = kBlock * kSortItems;

// Edge keys from a COO source array (graphs without a tile schedule).
template <typename LabT>
__global__ void __launch_bounds__(kBlock) k_edge_keys_coo(const uint32_t* __restrict__ src,
                                                          const uint32_t* __restrict__ tgt,
                                                          const LabT* __restrict__ lab,
                                                          const uint32_t* __restrict__ bid,
                                                          const uint32_t* __restrict__ bid_dst, uint32_t m,
                                                          int lb, int bb, uint64_t* __restrict__ keys) {
    const uint32_t e = blockIdx.x * kBlock + threadIdx.x;
    if (e >= m) return;
    keys[e] = (static_cast<uint64_t>(bid[src[e]]) << (lb + bb)) |
              (static_cast<uint64_t>(lab[e]) << bb) | bid_dst[tgt[e]];
}

__global__ void __launch_bounds__(kBlock) k_sort_hist(const uint64_t* __restrict__ in, uint32_t m,
                                                      int shift, uint32_t nblk,
                                                      uint32_t* __restrict__ hist) {
    __shared__ uint32_t s_h[256];
    s_h[threadIdx.x] = 0;
    __syncthreads();
    const uint64_t base = static_cast<uint64_t>(blockIdx.x) * kSortTile;
#pragma unroll
    for (int r = 0; r < kSortItems; r++) {
        uint64_t j = base + static_cast<uint64_t>(r) * kBlock + threadIdx.x;
        if (j < m) atomicAdd(&s_h[(in[j] >> shift) & 0xFF], 1u);
    }
    __syncthreads();
    hist[static_cast<uint64_t>(threadIdx.x) * nblk + blockIdx.x] = s_h[threadIdx.x];
}

// Stable scatter of one tile: every key gets its rank within the tile by
// digit (wave ballots isolate the lanes with the same digit; earlier rounds
// and earlier waves come first), the tile is staged in LDS in digit order,
// and each digit's run is then written out by consecutive threads.
__global__ void __launch_bounds__(kBlock) k_sort_scatter(const uint64_t* __restrict__ in,
                                                         uint64_t* __restrict__ out, uint32_t m,
                                                         int shift, uint32_t nblk,
                                                         const uint32_t* __restrict__ offs) {
    __shared__ uint64_t s_keys[kSortTile];
    __shared__ uint32_t s_run[256];     // global position of the tile's first key of each digit
    __shared__ uint32_t s_start[256];   // LDS position of the same key
    __shared__ uint32_t s_fill[256];    // keys of each digit placed so far
    __shared__ uint32_t s_cnt[kBlock / 64][256];
    const uint32_t tid = threadIdx.x, lane = lane_id(), wid = tid >> 6;
    const uint64_t base = static_cast<uint64_t>(blockIdx.x) * kSortTile;
    const uint32_t count = static_cast<uint32_t>(min(static_cast<uint64_t>(kSortTile), m - base));
    // the tile's keys per digit, from the scanned digit-major histogram: the
    // next entry is the next block of the same digit, or the first block of
    // the next digit, and the last entry ends at m
    const uint64_t idx = static_cast<uint64_t>(tid) * nblk + blockIdx.x;
    const uint32_t run = offs[idx];
    const uint32_t next = idx + 1 < static_cast<uint64_t>(nblk) * 256 ? offs[idx + 1] : m;
    s_run[tid] = run;
    s_start[tid] = next - run;
    s_fill[tid] = 0;
    for (int w = 0; w < kBlock / 64; w++) s_cnt[w][tid] = 0;
    __syncthreads();
    // exclusive scan of the 256 digit counts (one per thread)
    for (uint32_t d = 1; d < 256; d <<= 1) {
        const uint32_t v = tid >= d ? s_start[tid - d] : 0;
        __syncthreads();
        s_start[tid] += v;
        __syncthreads();
    }
    const uint32_t incl = s_start[tid];
    __syncthreads();
    s_start[tid] = incl - (next - run);
    __syncthreads();
    for (int r = 0; r < kSortItems; r++) {
        const uint32_t jl = static_cast<uint32_t>(r) * kBlock + tid;
        const bool valid = jl < count;
        const uint64_t key = valid ? in[base + jl] : 0;
        const uint32_t dig = static_cast<uint32_t>((key >> shift) & 0xFF);
        uint64_t peers = __ballot(valid);
#pragma unroll
        for (int b = 0; b < 8; b++) {
            const uint64_t bal = __ballot((dig >> b) & 1);
            peers &= ((dig >> b) & 1) ? bal : ~bal;
        }
        const uint64_t below = peers & ((1ull << lane) - 1);
        const uint32_t rank = static_cast<uint32_t>(__popcll(below));
        if (valid && below == 0) s_cnt[wid][dig] = static_cast<uint32_t>(__popcll(peers));
        __syncthreads();
        if (valid) {
            uint32_t pos = s_start[dig] + s_fill[dig] + rank;
            for (uint32_t w = 0; w < wid; w++) pos += s_cnt[w][dig];
            if (pos < kSortTile) s_keys[pos] = key;
        }
        __syncthreads();
        uint32_t add = 0;
        for (int w = 0; w < kBlock / 64; w++) {
            add += s_cnt[w][tid];
            s_cnt[w][tid] = 0;
        }
        s_fill[tid] += add;
        __syncthreads();
    }
    for (uint32_t i = tid; i < count; i += kBlock) {
        const uint64_t key = s_keys[i];
        const uint32_t dig = static_cast<uint32_t>((key >> shift) & 0xFF);
        const uint32_t pos = s_run[dig] + (i - s_start[dig]);
        if (pos < m) out[pos] = key;
    }
}

__global__ void __launch_bounds__(kBlock) k_unique_flags(const uint64_t* __restrict__ keys, uint32_t m,
                                                         uint32_t* __restrict__ flag) {
    uint32_t i = blockIdx.x * kBlock + threadIdx.x;
    if (i < m) flag[i] = (i == 0 || keys[i] != keys[i - 1]) ? 1u : 0u;
}

__global__ void __launch_bounds__(kBlock) k_unpack(const uint64_t* __restrict__ keys, uint32_t m,
                                                   const uint32_t* __restrict__ flag,
                                                   const uint32_t* __restrict__ pos, int lb, int bb,
                                                   uint32_t* __restrict__ s, uint32_t* __restrict__ l,
                                                   uint32_t* __restrict__ d) {
    uint32_t i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= m || !flag[i]) return;
    const uint64_t k = keys[i];
    const uint32_t p = pos[i];
    s[p] = static_cast<uint32_t>(k >> (lb + bb));
    l[p] = static_cast<uint32_t>((k >> bb) & ((1ull << lb) - 1));
    d[p] = static_cast<uint32_t>(k & ((1ull << bb) - 1));
}

}  // namespace

// Sort m keys ascending on bits [0, bits); returns the buffer holding the
// result (a or b).
uint64_t* radix_sort(uint64_t* a, uint64_t* b, uint32_t m, int bits, Arena& arena, hipStream_t s) {
    if (m <= 1) return a;
    const uint32_t nblk = ceil_div(m, kSortTile);
    uint32_t* hist = arena.alloc<uint32_t>(static_cast<size_t>(nblk) * 256);
    for (int shift = 0; shift < bits; shift += 8) {
        k_sort_hist<<<nblk, kBlock, 0, s>>>(a, m, shift, nblk, hist);
        scan_exclusive(hist, hist, nblk * 256, nullptr, arena, s);
        k_sort_scatter<<<nblk, kBlock, 0, s>>>(a, b, m, shift, nblk, hist);
        std::swap(a, b);
    }
    hip_check(hipGetLastError(), "radix sort launch");
    return a;
}

namespace {

// First-occurrence block ids of the classes named by `rep` into ids[n], the
// block sizes into sizes_preset or a new array of `arena`; returns the
// block count.
uint32_t number_blocks(const Staged& g, const uint32_t* rep, uint32_t* ids, uint32_t** sizes_out, Arena& arena,
                       hipStream_t s, uint32_t* sizes_preset = nullptr, uint64_t n_ids = 0) {
    const uint32_t n = g.n;
    // class names are vertex ids, or below n_ids when given
    const uint64_t ids_cap = std::max<uint64_t>(n, n_ids);
    uint32_t* cmin = arena.alloc<uint32_t>(ids_cap + 1);
    uint32_t* isrep = arena.alloc<uint32_t>(n);
    uint32_t* rank = arena.alloc<uint32_t>(n);
    uint32_t* total = arena.alloc<uint32_t>(1);
    const uint32_t gb = std::max<uint32_t>(ceil_div(n, kBlock), 1);
    hip_check(hipMemsetAsync(cmin, 0xFF, (ids_cap + 1) * 4, s), "class minima");
    if (n) {
        k_fin_min<<<gb, kBlock, 0, s>>>(rep, g.alive, n, cmin);
        k_fin_rep<<<gb, kBlock, 0, s>>>(rep, g.alive, n, cmin, isrep);
    }
    scan_exclusive(isrep, rank, n, total, arena, s);
    uint32_t nb = 0;
    hip_check(hipMemcpyAsync(&nb, total, 4, hipMemcpyDeviceToHost, s), "block count");
    hip_check(hipStreamSynchronize(s), "block count sync");
    uint32_t* sizes = sizes_preset ? sizes_preset : arena.alloc<uint32_t>(nb + 1);
    hip_check(hipMemsetAsync(sizes, 0, (static_cast<size_t>(nb) + 1) * 4, s), "sizes");
    if (n) k_fin_ids<<<ceil_div(n, kIdsPerBlock), kBlock, 0, s>>>(g.alive, n, rep, cmin, rank, ids, sizes);
    hip_check(hipGetLastError(), "finalize launch");
    *sizes_out = sizes;
    return nb;
}

void finalize_edges(const Staged& g, const uint32_t* rep, const uint32_t* rep_prev, bool want_edges,
                    FinalOut& out, Arena& arena, Arena& keep, hipStream_t s, uint64_t n_ids);

// Block ids and sizes are numbered in the call's work memory and copied
// into the result's own arrays at the end: the kernels that count the sizes
// (atomics at random blocks) and gather the ids of the edges' targets ran
// 10-20 % slower on rmat27 when these arrays were result allocations of
// their own beside the work memory's other random-access arrays.
void finalize_impl(const Staged& g, const uint32_t* rep, const uint32_t* rep_prev, bool want_edges,
                   FinalOut& out, Arena& arena, Arena& keep, hipStream_t s, uint64_t n_ids = 0) {
    if (out.preset) {
        finalize_edges(g, rep, rep_prev, want_edges, out, arena, keep, s, n_ids);
        return;
    }
    uint32_t* ids = keep.alloc<uint32_t>(g.n);
    out.block_ids = arena.alloc<uint32_t>(g.n);
    finalize_edges(g, rep, rep_prev, want_edges, out, arena, keep, s, n_ids);
    uint32_t* sizes = keep.alloc<uint32_t>(out.n_blocks + 1ull);
    if (g.n)
        hip_check(hipMemcpyAsync(ids, out.block_ids, static_cast<size_t>(g.n) * 4, hipMemcpyDeviceToDevice, s),
                  "block ids");
    hip_check(hipMemcpyAsync(sizes, out.block_sizes, (out.n_blocks + 1ull) * 4, hipMemcpyDeviceToDevice, s),
              "block sizes");
    out.block_ids = ids;
    out.block_sizes = sizes;
}

void finalize_edges(const Staged& g, const uint32_t* rep, const uint32_t* rep_prev, bool want_edges,
                    FinalOut& out, Arena& arena, Arena& keep, hipStream_t s, uint64_t n_ids) {
    const uint32_t n = g.n;
    const uint32_t nb = number_blocks(g, rep, out.block_ids, &out.block_sizes, arena, s,
                                      out.preset ? out.block_sizes : nullptr, n_ids);
    out.n_blocks = nb;
    // the target end of a summary edge: the final blocks, or the blocks of
    // the previous level's classes
    const uint32_t* dst_ids = out.block_ids;
    uint32_t nb_dst = nb;
    if (rep_prev && want_edges && g.m) {
        uint32_t* ids = arena.alloc<uint32_t>(n);
        uint32_t* sizes = nullptr;
        nb_dst = number_blocks(g, rep_prev, ids, &sizes, arena, s);
        dst_ids = ids;
    }
    uint32_t* total = arena.alloc<uint32_t>(1);
    out.n_se = 0;
    if (!want_edges || g.m == 0) {
        if (!out.preset) {
            out.se_src = keep.alloc<uint32_t>(1);
            out.se_label = keep.alloc<uint32_t>(1);
            out.se_dst = keep.alloc<uint32_t>(1);
        }
        return;
    }
    const uint32_t nb_max = std::max(nb, nb_dst);
    const int bb = std::max(1, bit_width(nb_max ? nb_max - 1 : 0));
    const int lb = std::max(1, bit_width(g.max_label));
    if (bucketed_summary_edges_fit(g, lb, bb)) {
        bucketed_summary_edges(g, out.block_ids, nb, dst_ids, lb, bb, out, arena, keep, s);
        return;
    }
    if (2 * bb + lb > 64)
        throw DeviceError{BSIM_E_UNSUPPORTED, "summary-edge triple does not fit 64 bits"};
    const uint32_t m = static_cast<uint32_t>(g.m);
    uint64_t* ka = arena.alloc<uint64_t>(m);
    uint64_t* kb = arena.alloc<uint64_t>(m);
    const uint32_t grid = std::max<uint32_t>(g.n_hubs + g.n_tiles, 1);
    if (g.src) {
        if (g.label_bytes == 2)
            k_edge_keys_coo<uint16_t><<<ceil_div(m, kBlock), kBlock, 0, s>>>(
                g.src, g.tgt, static_cast<const uint16_t*>(g.lab), out.block_ids, dst_ids, m, lb, bb, ka);
        else
            k_edge_keys_coo<uint32_t><<<ceil_div(m, kBlock), kBlock, 0, s>>>(
                g.src, g.tgt, static_cast<const uint32_t*>(g.lab), out.block_ids, dst_ids, m, lb, bb, ka);
    } else if (g.label_bytes == 2)
        k_edge_keys<uint16_t><<<grid, kBlock, 0, s>>>(g.row_off, g.tgt,
                                                      static_cast<const uint16_t*>(g.lab), out.block_ids, dst_ids,
                                                      g.tile_i0, g.tile_i1, g.tile_e0, g.tile_e1, g.act,
                                                      g.n_tiles, g.hub_v, g.n_hubs,
                                                      lb, bb, ka);
    else
        k_edge_keys<uint32_t><<<grid, kBlock, 0, s>>>(g.row_off, g.tgt,
                                                      static_cast<const uint32_t*>(g.lab), out.block_ids, dst_ids,
                                                      g.tile_i0, g.tile_i1, g.tile_e0, g.tile_e1, g.act,
                                                      g.n_tiles, g.hub_v, g.n_hubs,
                                                      lb, bb, ka);
    hip_check(hipGetLastError(), "edge key launch");
    uint64_t* sorted = radix_sort(ka, kb, m, 2 * bb + lb, arena, s);
    uint32_t* flag = arena.alloc<uint32_t>(m);
    uint32_t* pos = arena.alloc<uint32_t>(m);
    k_unique_flags<<<ceil_div(m, kBlock), kBlock, 0, s>>>(sorted, m, flag);
    scan_exclusive(flag, pos, m, total, arena, s);
    uint32_t nse = 0;
    hip_check(hipMemcpyAsync(&nse, total, 4, hipMemcpyDeviceToHost, s), "edge count");
    hip_check(hipStreamSynchronize(s), "edge count sync");
    out.n_se = nse;
    if (!out.preset) {
        out.se_src = keep.alloc<uint32_t>(nse);
        out.se_label = keep.alloc<uint32_t>(nse);
        out.se_dst = keep.alloc<uint32_t>(nse);
    }
    k_unpack<<<ceil_div(m, kBlock), kBlock, 0, s>>>(sorted, m, flag, pos, lb, bb, out.se_src,
                                                    out.se_label, out.se_dst);
    hip_check(hipGetLastError(), "unpack launch");
}

}  // namespace

void finalize(const Staged& g, const uint32_t* rep, bool want_edges, FinalOut& out, Arena& arena,
              Arena& keep, hipStream_t s, uint64_t n_ids) {
    finalize_impl(g, rep, nullptr, want_edges, out, arena, keep, s, n_ids);
}

void finalize_prev_level(const Staged& g, const uint32_t* rep, const uint32_t* rep_prev, bool want_edges,
                         FinalOut& out, Arena& arena, Arena& keep, hipStream_t s) {
    finalize_impl(g, rep, rep_prev, want_edges, out, arena, keep, s);
}

}  // namespace bsim
