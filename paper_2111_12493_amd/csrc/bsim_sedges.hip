// bsim_sedges.hip -- the summary graph's edges (a8), bucketed by source block.
//
// The summary edges (Sec. 2.6: edges between vertex summaries) are the
// distinct triples (block(v), l, block(w)) over the edges (v, l, w), listed
// by source block, then label, then target block.  A global sort of all m
// triples would move every edge through eight radix passes; here the edges
// are bucketed by source block first, so only the (label, target block)
// values inside one block's segment are ever compared:
//   1. every vertex with out-edges claims a range of its block's segment
//      (one atomic per vertex); an exclusive scan over the blocks places
//      the segments;
//   2. every edge writes its value l << bb | block(w) into its vertex's range;
//   3. every segment is sorted and de-duplicated in place, by size:
//        1 value          nothing to do;
//        2..256           one wave sorts the segments starting in 256
//                         consecutive positions, LDS radix sort on
//                         (segment ordinal, value);
//        257..16,384      one workgroup per segment, LDS radix sort;
//        more             one global LSD radix sort over all such segments
//                         on (segment rank, value);
//   4. an exclusive scan of the per-block distinct counts places the output;
//      the distinct values are unpacked to (src, label, dst).
// The LDS radix sorts rank digits with wave ballots into per-wave counters
// and skip every digit on which a segment's keys agree.
#include "bsim_device.h"

namespace bsim {

namespace {

constexpr uint32_t kSegSmallMax = 256;     // tile-packed segments hold at most this many values
constexpr uint32_t kSegMedMax = 4096;      // one 256-thread workgroup per segment
constexpr uint32_t kSegBigMax = 16384;     // one 1,024-thread workgroup per segment
constexpr uint32_t kSortIpt = 16;          // values per thread in an LDS sort (at most)
constexpr uint32_t kSmallBlock = 64;       // a small tile is one wave
constexpr uint32_t kSmallRange = 256;      // segment starts per small tile
constexpr uint32_t kSmallCap = 512;        // values per small tile: kSmallRange + kSegSmallMax - 1 fit
constexpr uint32_t kSmallMaxSeg = kSmallCap / 2;             // segments of >= 2 values
constexpr int kOrdBits = 8;                                  // tile ordinals < 256
constexpr uint32_t kUnpackTile = kBlock * 16;
constexpr uint32_t kUnpackCache = 4096;    // block offsets a tile keeps in LDS
constexpr uint32_t kBigBlock = 1024;

static_assert(kSmallRange + kSegSmallMax <= kSmallCap, "a small tile must hold its segments");
static_assert(kSmallMaxSeg <= (1u << kOrdBits), "tile ordinals must fit their field");
static_assert(kSmallCap <= kSmallBlock * kSortIpt, "a small tile fits the sort's registers");
static_assert(kBigBlock * kSortIpt == kSegBigMax && kBlock * kSortIpt == kSegMedMax, "sort capacities");

__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t x) {
    const uint32_t lane = lane_id();
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const uint32_t y = static_cast<uint32_t>(__shfl_up(static_cast<int>(x), d, 64));
        if (lane >= static_cast<uint32_t>(d)) x += y;
    }
    return x;
}

// Exclusive scan over the NT threads of a block; *total gets the sum.  All
// threads must call it.  `red` needs NT / 64 entries.
template <int NT>
__device__ __forceinline__ uint32_t block_excl_scan(uint32_t x, uint32_t* red, uint32_t* total) {
    const uint32_t incl = wave_incl_scan(x);
    const uint32_t w = threadIdx.x >> 6;
    if (lane_id() == 63) red[w] = incl;
    __syncthreads();
    uint32_t base = 0, tot = 0;
    for (uint32_t i = 0; i < NT / 64; i++) {
        const uint32_t r = red[i];
        if (i < w) base += r;
        tot += r;
    }
    __syncthreads();
    *total = tot;
    return base + incl - x;
}

// Position of the last entry of off[lo, hi) that is <= x (off nondecreasing,
// off[lo] <= x).
__device__ __forceinline__ uint32_t last_le(const uint32_t* off, uint32_t lo, uint32_t hi, uint32_t x) {
    while (hi - lo > 1) {
        const uint32_t mid = lo + (hi - lo) / 2;
        if (off[mid] <= x)
            lo = mid;
        else
            hi = mid;
    }
    return lo;
}

// Shared state of one LDS sort: the keys of the tile, the per-wave digit
// counters and the segment table.
struct SortSmem {
    uint64_t* buf;       // [cap]
    uint32_t* wc;        // [NT / 64][256]
    uint32_t* red;       // [16]
    uint32_t* misc;      // [8]
    uint32_t* lofs;      // [max_seg + 1] first position of each segment in the tile
    uint32_t* blk;       // [max_seg] its block
    uint32_t* est;       // [max_seg] its first value in vals[]
    uint32_t* dbase;     // [max_seg] distinct values before it in the tile
};

template <int NT>
__device__ SortSmem carve(uint8_t* p, uint32_t cap, uint32_t max_seg) {
    SortSmem S;
    S.buf = reinterpret_cast<uint64_t*>(p);
    p += 8ull * cap;
    S.wc = reinterpret_cast<uint32_t*>(p);
    p += 4ull * (NT / 64) * 256;
    S.red = reinterpret_cast<uint32_t*>(p);
    p += 4 * 16;
    S.misc = reinterpret_cast<uint32_t*>(p);
    p += 4 * 8;
    S.lofs = reinterpret_cast<uint32_t*>(p);
    p += 4ull * (max_seg + 1);
    S.blk = reinterpret_cast<uint32_t*>(p);
    p += 4ull * max_seg;
    S.est = reinterpret_cast<uint32_t*>(p);
    p += 4ull * max_seg;
    S.dbase = reinterpret_cast<uint32_t*>(p);
    return S;
}

__host__ __device__ constexpr uint64_t sort_smem_bytes(uint32_t nt, uint32_t cap, uint32_t max_seg) {
    return 8ull * cap + 4ull * (nt / 64) * 256 + 4 * 16 + 4 * 8 + 4ull * (max_seg + 1) + 12ull * max_seg;
}

struct SegArgs {
    uint64_t* vals;             // bucketed values, sorted and compacted in place
    const uint32_t* estart;     // nb + 1 segment offsets (estart[nb] = live edges)
    uint32_t nb;
    uint32_t* uniq;             // distinct values per block
    const uint32_t* tile_first; // small tiles: first block whose segment starts in the tile
    uint32_t n_tiles;
    const uint32_t* list;       // medium segments: their blocks
    int vb;                     // value bits
};

// Sort the tile's cnt keys (ordinal << vb | value), de-duplicate, and write
// every segment's distinct values back to the front of its segment.  The
// segment table (lofs, blk, est, nseg) is set up by the caller, followed by
// a barrier.
template <int NT>
__device__ void sort_tile(const SegArgs& a, const SortSmem& S, uint32_t cnt, uint32_t nseg) {
    constexpr uint32_t W = NT / 64;
    constexpr uint32_t DPT = NT >= 256 ? 1 : 256 / NT;  // digits per thread in the prefix step
    const uint32_t tid = threadIdx.x, lane = lane_id(), w = tid >> 6;
    const uint32_t ipt = (cnt + NT - 1) / NT;  // rounds per wave; element = (w * ipt + r) * 64 + lane
    const uint64_t vmask = (1ull << a.vb) - 1;
    const uint64_t lt = (1ull << lane) - 1;
    uint64_t key[kSortIpt];
    uint64_t kor = 0, kand = ~0ull;
#pragma unroll
    for (uint32_t r = 0; r < kSortIpt; r++) {
        key[r] = ~0ull;
        const uint32_t i = (w * ipt + r) * 64 + lane;
        if (r < ipt && i < cnt) {
            const uint32_t o = nseg == 1 ? 0u : last_le(S.lofs, 0, nseg, i);
            key[r] = (static_cast<uint64_t>(o) << a.vb) | a.vals[S.est[o] + (i - S.lofs[o])];
            kor |= key[r];
            kand &= key[r];
        }
    }
    // bits on which the keys differ: only their digits need a pass
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) {
        kor |= shfl_xor_u64(kor, d);
        kand &= shfl_xor_u64(kand, d);
    }
    if (lane == 0) {
        S.buf[2 * w] = kor;
        S.buf[2 * w + 1] = kand;
    }
    __syncthreads();
    uint64_t diff = 0;
    {
        uint64_t o = 0, n = ~0ull;
        for (uint32_t i = 0; i < W; i++) {
            o |= S.buf[2 * i];
            n &= S.buf[2 * i + 1];
        }
        diff = o ^ n;
    }
    __syncthreads();
    uint32_t lr[kSortIpt];
    for (int shift = 0; shift < 64; shift += 8) {
        if (((diff >> shift) & 0xFF) == 0) continue;  // uniform over the block
        for (uint32_t d = lane; d < 256; d += 64) S.wc[w * 256 + d] = 0;
        __builtin_amdgcn_wave_barrier();
        // wave-local stable ranks per digit
#pragma unroll
        for (uint32_t r = 0; r < kSortIpt; r++) {
            if (r >= ipt) continue;
            const uint32_t i = (w * ipt + r) * 64 + lane;
            const bool valid = i < cnt;
            const uint32_t dig = static_cast<uint32_t>((key[r] >> shift) & 0xFF);
            uint64_t peers = __ballot(valid);
#pragma unroll
            for (int b = 0; b < 8; b++) {
                const uint64_t bal = __ballot((dig >> b) & 1);
                peers &= ((dig >> b) & 1) ? bal : ~bal;
            }
            const uint32_t leader = peers ? static_cast<uint32_t>(__ffsll(static_cast<long long>(peers)) - 1) : lane;
            uint32_t base = 0;
            if (valid && lane == leader) base = atomicAdd(&S.wc[w * 256 + dig], static_cast<uint32_t>(__popcll(peers)));
            base = static_cast<uint32_t>(__shfl(static_cast<int>(base), static_cast<int>(leader), 64));
            lr[r] = base + static_cast<uint32_t>(__popcll(peers & lt));
        }
        __syncthreads();
        // digit d of wave w starts at (keys of smaller digits) + (digit d in
        // earlier waves); thread t owns digits [t DPT, (t + 1) DPT)
        const bool owner = tid * DPT < 256;
        uint32_t tot = 0;
        if (owner)
            for (uint32_t c = 0; c < DPT; c++)
                for (uint32_t i = 0; i < W; i++) tot += S.wc[i * 256 + tid * DPT + c];
        uint32_t all = 0;
        uint32_t run = block_excl_scan<NT>(owner ? tot : 0u, S.red, &all);
        if (owner)
            for (uint32_t c = 0; c < DPT; c++)
                for (uint32_t i = 0; i < W; i++) {
                    const uint32_t d = tid * DPT + c;
                    const uint32_t cc = S.wc[i * 256 + d];
                    S.wc[i * 256 + d] = run;
                    run += cc;
                }
        __syncthreads();
#pragma unroll
        for (uint32_t r = 0; r < kSortIpt; r++) {
            if (r >= ipt) continue;
            const uint32_t i = (w * ipt + r) * 64 + lane;
            if (i < cnt) {
                const uint32_t dig = static_cast<uint32_t>((key[r] >> shift) & 0xFF);
                S.buf[S.wc[w * 256 + dig] + lr[r]] = key[r];
            }
        }
        __syncthreads();
#pragma unroll
        for (uint32_t r = 0; r < kSortIpt; r++) {
            if (r >= ipt) continue;
            const uint32_t i = (w * ipt + r) * 64 + lane;
            if (i < cnt) key[r] = S.buf[i];
        }
    }
    // key[r] now holds sorted element (w * ipt + r) * 64 + lane; publish the
    // order for the neighbour comparison
#pragma unroll
    for (uint32_t r = 0; r < kSortIpt; r++) {
        if (r >= ipt) continue;
        const uint32_t i = (w * ipt + r) * 64 + lane;
        if (i < cnt) S.buf[i] = key[r];
    }
    __syncthreads();
    // distinct positions: first occurrences counted in element order
    uint32_t dloc[kSortIpt];
    uint32_t firsts = 0;  // bit r: element of round r is a first occurrence
    uint32_t wrun = 0;
#pragma unroll
    for (uint32_t r = 0; r < kSortIpt; r++) {
        if (r >= ipt) continue;
        const uint32_t i = (w * ipt + r) * 64 + lane;
        const bool first = i < cnt && (i == 0 || key[r] != S.buf[i - 1]);
        const uint64_t bal = __ballot(first);
        dloc[r] = wrun + static_cast<uint32_t>(__popcll(bal & lt));
        wrun += static_cast<uint32_t>(__popcll(bal));
        if (first) firsts |= 1u << r;
    }
    if (lane == 0) S.red[w] = wrun;
    __syncthreads();
    uint32_t wbase = 0;
    for (uint32_t i = 0; i < w; i++) wbase += S.red[i];
    // every segment start is a first occurrence: it records the segment's base
#pragma unroll
    for (uint32_t r = 0; r < kSortIpt; r++) {
        if (r >= ipt) continue;
        const uint32_t i = (w * ipt + r) * 64 + lane;
        if (i < cnt) {
            const uint32_t o = static_cast<uint32_t>(key[r] >> a.vb);
            if (S.lofs[o] == i) S.dbase[o] = wbase + dloc[r];
        }
    }
    __syncthreads();
#pragma unroll
    for (uint32_t r = 0; r < kSortIpt; r++) {
        if (r >= ipt) continue;
        const uint32_t i = (w * ipt + r) * 64 + lane;
        if (i >= cnt) continue;
        const uint32_t o = static_cast<uint32_t>(key[r] >> a.vb);
        const uint32_t d = wbase + dloc[r] - S.dbase[o];
        const bool first = (firsts >> r) & 1;
        if (first) a.vals[S.est[o] + d] = key[r] & vmask;
        if (i + 1 == S.lofs[o + 1]) a.uniq[S.blk[o]] = d + (first ? 1u : 0u);
    }
}

// Small segments (2..256 values): tile t takes the small segments whose
// first value lies in [t R, (t + 1) R), R = kSmallRange, packs them back to
// back and sorts them as one key set (segment ordinal << vb | value).  A
// tile is one wave, so the sort's barriers cost next to nothing and many
// tiles share a CU.
__global__ void __launch_bounds__(kSmallBlock) k_seg_small(SegArgs a) {
    extern __shared__ uint64_t smem_small[];
    const SortSmem S = carve<kSmallBlock>(reinterpret_cast<uint8_t*>(smem_small), kSmallCap, kSmallMaxSeg);
    const uint32_t t = blockIdx.x;
    const uint32_t b_lo = a.tile_first[t];
    const uint32_t b_hi = t + 1 < a.n_tiles ? a.tile_first[t + 1] : a.nb;
    uint32_t nseg = 0, cnt = 0;
    for (uint32_t c = b_lo; c < b_hi; c += kSmallBlock) {  // uniform trip count
        const uint32_t b = c + threadIdx.x;
        uint32_t sz = 0;
        if (b < b_hi) sz = a.estart[b + 1] - a.estart[b];
        const bool small = sz >= 2 && sz <= kSegSmallMax;
        uint32_t tot = 0;
        const uint32_t packed = block_excl_scan<kSmallBlock>(small ? (1u << 20) | sz : 0u, S.red, &tot);
        if (small) {
            const uint32_t o = nseg + (packed >> 20);
            S.lofs[o] = cnt + (packed & 0xFFFFF);
            S.blk[o] = b;
            S.est[o] = a.estart[b];
        }
        nseg += tot >> 20;
        cnt += tot & 0xFFFFF;
    }
    if (nseg == 0) return;  // uniform
    if (threadIdx.x == 0) S.lofs[nseg] = cnt;
    __syncthreads();
    sort_tile<kSmallBlock>(a, S, cnt, nseg);
}

// Medium segments: one workgroup per listed block.
template <int NT>
__global__ void __launch_bounds__(NT) k_seg_medium(SegArgs a) {
    extern __shared__ uint64_t smem_med[];
    const SortSmem S = carve<NT>(reinterpret_cast<uint8_t*>(smem_med), NT * kSortIpt, 1);
    const uint32_t b = a.list[blockIdx.x];
    const uint32_t cnt = a.estart[b + 1] - a.estart[b];
    if (threadIdx.x == 0) {
        S.lofs[0] = 0;
        S.lofs[1] = cnt;
        S.blk[0] = b;
        S.est[0] = a.estart[b];
    }
    __syncthreads();
    sort_tile<NT>(a, S, cnt, 1);
}

// ------------------------------------------------------------ set-up passes

// Every vertex with out-edges claims deg(v) values of its block's segment
// (a dead vertex has no edges: staging rejects such graphs).
__global__ void __launch_bounds__(kBlock) k_seg_claim(const uint32_t* __restrict__ row_off,
                                                      const uint32_t* __restrict__ bid, uint32_t n,
                                                      uint32_t* __restrict__ ecount, uint32_t* __restrict__ voff) {
    const uint32_t v = blockIdx.x * kBlock + threadIdx.x;
    if (v >= n) return;
    const uint32_t d = row_off[v + 1] - row_off[v];
    const uint32_t b = bid[v];
    if (d && b != 0xFFFFFFFFu) voff[v] = atomicAdd(&ecount[b], d);
}

struct FillShared {
    uint32_t off[kTileMaxVerts + 1];
    uint32_t base[kTileMaxVerts];
    uint32_t red[kBlock / 64];
    alignas(8) uint8_t seg[kTileMaxEdges];
};

// Every edge (v, l, w) writes l << bb | block(w) into v's claimed range.
template <typename LabT>
__global__ void __launch_bounds__(kBlock) k_seg_fill(
    const uint32_t* __restrict__ row_off, const uint32_t* __restrict__ tgt, const LabT* __restrict__ lab,
    const uint32_t* __restrict__ bid, const uint32_t* __restrict__ bid_dst, const uint32_t* __restrict__ estart,
    const uint32_t* __restrict__ voff, const uint32_t* __restrict__ tile_i0, const uint32_t* __restrict__ tile_i1,
    const uint32_t* __restrict__ tile_e0, const uint32_t* __restrict__ tile_e1, const uint32_t* __restrict__ act,
    uint32_t n_tiles, const uint32_t* __restrict__ hub_v, uint32_t n_hubs, int bb, uint64_t* __restrict__ vals) {
    __shared__ FillShared S;
    const uint32_t tid = threadIdx.x;
    if (blockIdx.x < n_hubs) {
        const uint32_t v = hub_v[blockIdx.x];
        const uint32_t e0 = row_off[v], e1 = row_off[v + 1];
        uint64_t* out = vals + estart[bid[v]] + voff[v];
        for (uint32_t e = e0 + tid; e < e1; e += kBlock)
            out[e - e0] = (static_cast<uint64_t>(lab[e]) << bb) | bid_dst[tgt[e]];
        return;
    }
    const uint32_t tile = blockIdx.x - n_hubs;
    if (tile >= n_tiles) return;
    const uint32_t i0 = tile_i0[tile], nv = tile_i1[tile] - i0;
    const uint32_t ebase = tile_e0[tile];
    const uint32_t ne = tile_e1[tile] - ebase;
    for (uint32_t i = tid; i < nv; i += kBlock) {
        const uint32_t v = act[i0 + i];
        const uint32_t o = row_off[v] - ebase;
        S.off[i] = o;
        // the value of local edge j of this vertex goes to base + j (mod 2^32)
        S.base[i] = estart[bid[v]] + voff[v] - o;
    }
    if (tid == 0) S.off[nv] = ne;
    __syncthreads();
    tile_segments(nv, S.off, S.seg, S.red);
    for (uint32_t j = tid; j < ne; j += kBlock) {
        const uint32_t e = ebase + j;
        vals[S.base[S.seg[j]] + j] = (static_cast<uint64_t>(lab[e]) << bb) | bid_dst[tgt[e]];
    }
}

// Size classes: single values are final; medium and large segments are
// listed (wave-aggregated appends; list order is free).
__global__ void __launch_bounds__(kBlock) k_seg_class(const uint32_t* __restrict__ estart, uint32_t nb,
                                                      uint32_t* __restrict__ uniq, uint32_t* __restrict__ l_med,
                                                      uint32_t* __restrict__ l_big, uint32_t* __restrict__ l_huge,
                                                      uint32_t* __restrict__ ctr) {
    const uint32_t b = blockIdx.x * kBlock + threadIdx.x;
    const bool in = b < nb;
    const uint32_t sz = in ? estart[b + 1] - estart[b] : 0u;
    if (in && sz <= 1) uniq[b] = sz;
    const uint32_t cls = !in ? 0u : sz > kSegBigMax ? 3u : sz > kSegMedMax ? 2u : sz > kSegSmallMax ? 1u : 0u;
    const uint32_t lane = lane_id();
    const uint64_t lt = (1ull << lane) - 1;
    uint32_t* lists[3] = {l_med, l_big, l_huge};
#pragma unroll
    for (uint32_t c = 1; c <= 3; c++) {
        const uint64_t bal = __ballot(cls == c);
        if (!bal) continue;
        const uint32_t leader = static_cast<uint32_t>(__ffsll(static_cast<long long>(bal)) - 1);
        uint32_t base = 0;
        if (lane == leader) base = atomicAdd(&ctr[c - 1], static_cast<uint32_t>(__popcll(bal)));
        base = static_cast<uint32_t>(__shfl(static_cast<int>(base), static_cast<int>(leader), 64));
        if (cls == c) lists[c - 1][base + static_cast<uint32_t>(__popcll(bal & lt))] = b;
    }
    const uint32_t huge = wave_sum_u32(cls == 3 ? sz : 0u);
    if (lane == 0 && huge) atomicAdd(&ctr[3], huge);
}

// tf[t] = first b in [0, nb] with off[b] >= t * T + c, for t < n_t (off is
// nondecreasing with nb + 1 entries and every searched point is <= off[nb]).
// Thread b writes the tiles whose point falls in (off[b - 1], off[b]].
__global__ void __launch_bounds__(kBlock) k_tile_first(const uint32_t* __restrict__ off, uint32_t nb, uint32_t T,
                                                       uint32_t c, uint32_t n_t, uint32_t* __restrict__ tf) {
    const uint32_t b = blockIdx.x * kBlock + threadIdx.x;
    if (b > nb) return;
    const int64_t lo_x = b == 0 ? 0 : static_cast<int64_t>(off[b - 1]) + 1;
    const int64_t hi_x = off[b];
    int64_t t0 = lo_x - static_cast<int64_t>(c);
    t0 = t0 <= 0 ? 0 : (t0 + T - 1) / T;
    const int64_t t1x = hi_x - static_cast<int64_t>(c);
    if (t1x < 0) return;
    const int64_t t1 = t1x / T < static_cast<int64_t>(n_t) - 1 ? t1x / T : static_cast<int64_t>(n_t) - 1;
    for (int64_t t = t0; t <= t1; t++) tf[t] = b;
}

// ------------------------------------------------------------ huge segments

__global__ void __launch_bounds__(kBlock) k_huge_sizes(const uint32_t* __restrict__ list, uint32_t nh,
                                                       const uint32_t* __restrict__ estart,
                                                       uint32_t* __restrict__ sz) {
    const uint32_t o = blockIdx.x * kBlock + threadIdx.x;
    if (o < nh) sz[o] = estart[list[o] + 1] - estart[list[o]];
}

__global__ void __launch_bounds__(kBlock) k_huge_gather(const uint32_t* __restrict__ list,
                                                        const uint32_t* __restrict__ hstart,
                                                        const uint32_t* __restrict__ estart,
                                                        const uint64_t* __restrict__ vals, int vb,
                                                        uint64_t* __restrict__ keys) {
    const uint32_t o = blockIdx.x;
    const uint32_t b = list[o];
    const uint32_t e0 = estart[b], e1 = estart[b + 1];
    uint64_t* out = keys + hstart[o];
    const uint64_t tag = static_cast<uint64_t>(o) << vb;
    for (uint32_t j = e0 + threadIdx.x; j < e1; j += kBlock) out[j - e0] = tag | vals[j];
}

__global__ void __launch_bounds__(kBlock) k_huge_first(const uint64_t* __restrict__ keys, uint32_t m,
                                                       uint32_t* __restrict__ flag) {
    const uint32_t i = blockIdx.x * kBlock + threadIdx.x;
    if (i < m) flag[i] = (i == 0 || keys[i] != keys[i - 1]) ? 1u : 0u;
}

__global__ void __launch_bounds__(kBlock) k_huge_write(const uint64_t* __restrict__ keys, uint32_t m,
                                                       const uint32_t* __restrict__ flag,
                                                       const uint32_t* __restrict__ pos,
                                                       const uint32_t* __restrict__ list,
                                                       const uint32_t* __restrict__ hstart,
                                                       const uint32_t* __restrict__ estart, int vb,
                                                       uint64_t* __restrict__ vals) {
    const uint32_t i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= m || !flag[i]) return;
    const uint64_t k = keys[i];
    const uint32_t o = static_cast<uint32_t>(k >> vb);
    vals[estart[list[o]] + pos[i] - pos[hstart[o]]] = k & ((1ull << vb) - 1);
}

__global__ void __launch_bounds__(kBlock) k_huge_uniq(const uint32_t* __restrict__ list, uint32_t nh,
                                                      const uint32_t* __restrict__ hstart,
                                                      const uint32_t* __restrict__ pos,
                                                      const uint32_t* __restrict__ pos_total,
                                                      uint32_t* __restrict__ uniq) {
    const uint32_t o = blockIdx.x * kBlock + threadIdx.x;
    if (o >= nh) return;
    const uint32_t end = o + 1 < nh ? pos[hstart[o + 1]] : *pos_total;
    uniq[list[o]] = end - pos[hstart[o]];
}

// ------------------------------------------------------------ unpack

// Output positions [t U, (t + 1) U): the distinct values of block b occupy
// [ostart[b], ostart[b + 1]) and sit at the front of its segment.
__global__ void __launch_bounds__(kBlock) k_seg_unpack(const uint64_t* __restrict__ vals,
                                                       const uint32_t* __restrict__ estart,
                                                       const uint32_t* __restrict__ ostart, uint32_t nb,
                                                       const uint32_t* __restrict__ tile_first, uint32_t n_tiles,
                                                       uint32_t nse, int bb, uint32_t* __restrict__ s,
                                                       uint32_t* __restrict__ l, uint32_t* __restrict__ d) {
    __shared__ uint32_t s_off[kUnpackCache + 1];
    const uint32_t t = blockIdx.x;
    // blocks [b0, b1] hold the tile's outputs: b0 holds position t U
    const uint32_t b0 = tile_first[t] - 1;
    const uint32_t b1 = t + 1 < n_tiles ? tile_first[t + 1] - 1 : nb - 1;
    const uint32_t nbk = b1 - b0 + 1;
    const bool cached = nbk <= kUnpackCache;
    if (cached)
        for (uint32_t i = threadIdx.x; i <= nbk; i += kBlock) s_off[i] = ostart[b0 + i];
    __syncthreads();
    const uint64_t p0 = static_cast<uint64_t>(t) * kUnpackTile;
    const uint64_t p1 = min(p0 + kUnpackTile, static_cast<uint64_t>(nse));
    const uint32_t bmask = static_cast<uint32_t>((1ull << bb) - 1);
    for (uint64_t pp = p0 + threadIdx.x; pp < p1; pp += kBlock) {
        const uint32_t p = static_cast<uint32_t>(pp);
        const uint32_t b = cached ? b0 + last_le(s_off, 0, nbk, p) : last_le(ostart, b0, b1 + 1, p);
        const uint64_t v = vals[estart[b] + (p - ostart[b])];
        s[p] = b;
        l[p] = static_cast<uint32_t>(v >> bb);
        d[p] = static_cast<uint32_t>(v) & bmask;
    }
}

}  // namespace

bool bucketed_summary_edges_fit(const Staged& g, int lb, int bb) {
    const int vb = lb + bb;
    if (g.src || g.m == 0 || g.n_tiles + g.n_hubs == 0) return false;
    if (vb + kOrdBits > 64) return false;
    // huge segments are ranked: at most m / (kSegBigMax + 1) of them
    return vb + bit_width(g.m / (kSegBigMax + 1)) <= 64;
}

void bucketed_summary_edges(const Staged& g, const uint32_t* bid, uint32_t nb, const uint32_t* dst_ids, int lb,
                            int bb, FinalOut& out, Arena& arena, Arena& keep, hipStream_t s) {
    const uint32_t n = g.n;
    const uint32_t m = static_cast<uint32_t>(g.m);
    const int vb = lb + bb;
    // 1. segments: per-vertex claims, then their placement
    uint32_t* ecount = arena.alloc<uint32_t>(static_cast<size_t>(nb) + 1);
    uint32_t* voff = arena.alloc<uint32_t>(n);
    uint32_t* estart = arena.alloc<uint32_t>(static_cast<size_t>(nb) + 1);
    uint32_t* ctr = arena.alloc<uint32_t>(8);
    hip_check(hipMemsetAsync(ecount, 0, (static_cast<size_t>(nb) + 1) * 4, s), "segment counts");
    hip_check(hipMemsetAsync(ctr, 0, 8 * 4, s), "segment classes");
    k_seg_claim<<<ceil_div(n, kBlock), kBlock, 0, s>>>(g.row_off, bid, n, ecount, voff);
    scan_exclusive(ecount, estart, nb, estart + nb, arena, s);
    // 2. values
    uint64_t* vals = arena.alloc<uint64_t>(m);
    const uint32_t grid = g.n_hubs + g.n_tiles;
    if (g.label_bytes == 2)
        k_seg_fill<uint16_t><<<grid, kBlock, 0, s>>>(g.row_off, g.tgt, static_cast<const uint16_t*>(g.lab), bid,
                                                     dst_ids, estart, voff, g.tile_i0, g.tile_i1, g.tile_e0,
                                                     g.tile_e1, g.act, g.n_tiles, g.hub_v, g.n_hubs, bb, vals);
    else
        k_seg_fill<uint32_t><<<grid, kBlock, 0, s>>>(g.row_off, g.tgt, static_cast<const uint32_t*>(g.lab), bid,
                                                     dst_ids, estart, voff, g.tile_i0, g.tile_i1, g.tile_e0,
                                                     g.tile_e1, g.act, g.n_tiles, g.hub_v, g.n_hubs, bb, vals);
    // 3. size classes
    uint32_t* uniq = arena.alloc<uint32_t>(static_cast<size_t>(nb) + 1);
    auto list_cap = [&](uint32_t above) { return std::min<uint64_t>(nb, m / (above + 1ull) + 1); };
    uint32_t* l_med = arena.alloc<uint32_t>(list_cap(kSegSmallMax));
    uint32_t* l_big = arena.alloc<uint32_t>(list_cap(kSegMedMax));
    uint32_t* l_huge = arena.alloc<uint32_t>(list_cap(kSegBigMax));
    k_seg_class<<<ceil_div(nb, kBlock), kBlock, 0, s>>>(estart, nb, uniq, l_med, l_big, l_huge, ctr);
    hip_check(hipGetLastError(), "segment launch");
    uint32_t hc[5] = {};
    hip_check(hipMemcpyAsync(hc, ctr, 4 * 4, hipMemcpyDeviceToHost, s), "segment classes");
    hip_check(hipMemcpyAsync(hc + 4, estart + nb, 4, hipMemcpyDeviceToHost, s), "live edges");
    hip_check(hipStreamSynchronize(s), "segment classes sync");
    const uint32_t n_med = hc[0], n_big = hc[1], n_huge = hc[2], huge_elems = hc[3], m_live = hc[4];
    SegArgs a{};
    a.vals = vals;
    a.estart = estart;
    a.nb = nb;
    a.uniq = uniq;
    a.vb = vb;
    const uint32_t n_st = ceil_div(m_live, kSmallRange);
    if (n_st) {
        uint32_t* tf = arena.alloc<uint32_t>(n_st);
        k_tile_first<<<ceil_div(static_cast<uint64_t>(nb) + 1, kBlock), kBlock, 0, s>>>(estart, nb, kSmallRange, 0,
                                                                                       n_st, tf);
        a.tile_first = tf;
        a.n_tiles = n_st;
        k_seg_small<<<n_st, kSmallBlock, sort_smem_bytes(kSmallBlock, kSmallCap, kSmallMaxSeg), s>>>(a);
    }
    if (n_med) {
        a.list = l_med;
        const uint64_t bytes = sort_smem_bytes(kBlock, kSegMedMax, 1);
        k_seg_medium<kBlock><<<n_med, kBlock, bytes, s>>>(a);
    }
    if (n_big) {
        a.list = l_big;
        const uint64_t bytes = sort_smem_bytes(kBigBlock, kSegBigMax, 1);
        hip_check(hipFuncSetAttribute(reinterpret_cast<const void*>(k_seg_medium<kBigBlock>),
                                      hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(bytes)),
                  "large-segment LDS");
        k_seg_medium<kBigBlock><<<n_big, kBigBlock, bytes, s>>>(a);
    }
    if (n_huge) {
        uint32_t* hsz = arena.alloc<uint32_t>(static_cast<size_t>(n_huge) + 1);
        uint32_t* hstart = arena.alloc<uint32_t>(static_cast<size_t>(n_huge) + 1);
        k_huge_sizes<<<ceil_div(n_huge, kBlock), kBlock, 0, s>>>(l_huge, n_huge, estart, hsz);
        scan_exclusive(hsz, hstart, n_huge, hstart + n_huge, arena, s);
        uint64_t* ka = arena.alloc<uint64_t>(huge_elems);
        uint64_t* kb = arena.alloc<uint64_t>(huge_elems);
        k_huge_gather<<<n_huge, kBlock, 0, s>>>(l_huge, hstart, estart, vals, vb, ka);
        uint64_t* sorted = radix_sort(ka, kb, huge_elems, bit_width(n_huge - 1) + vb, arena, s);
        // the other buffer holds the first-occurrence flags and their scan
        uint32_t* flag = reinterpret_cast<uint32_t*>(sorted == ka ? kb : ka);
        uint32_t* pos = flag + huge_elems;
        uint32_t* pos_total = arena.alloc<uint32_t>(1);
        const uint32_t gh = ceil_div(huge_elems, kBlock);
        k_huge_first<<<gh, kBlock, 0, s>>>(sorted, huge_elems, flag);
        scan_exclusive(flag, pos, huge_elems, pos_total, arena, s);
        k_huge_write<<<gh, kBlock, 0, s>>>(sorted, huge_elems, flag, pos, l_huge, hstart, estart, vb, vals);
        k_huge_uniq<<<ceil_div(n_huge, kBlock), kBlock, 0, s>>>(l_huge, n_huge, hstart, pos, pos_total, uniq);
    }
    hip_check(hipGetLastError(), "segment sort launch");
    // 4. output placement and unpacking
    uint32_t* ostart = arena.alloc<uint32_t>(static_cast<size_t>(nb) + 1);
    scan_exclusive(uniq, ostart, nb, ostart + nb, arena, s);
    uint32_t nse = 0;
    hip_check(hipMemcpyAsync(&nse, ostart + nb, 4, hipMemcpyDeviceToHost, s), "edge count");
    hip_check(hipStreamSynchronize(s), "edge count sync");
    out.n_se = nse;
    if (!out.preset) {
        out.se_src = keep.alloc<uint32_t>(nse);
        out.se_label = keep.alloc<uint32_t>(nse);
        out.se_dst = keep.alloc<uint32_t>(nse);
    }
    const uint32_t n_ut = ceil_div(nse, kUnpackTile);
    if (n_ut) {
        uint32_t* tf = arena.alloc<uint32_t>(n_ut);
        k_tile_first<<<ceil_div(static_cast<uint64_t>(nb) + 1, kBlock), kBlock, 0, s>>>(ostart, nb, kUnpackTile, 1,
                                                                                       n_ut, tf);
        k_seg_unpack<<<n_ut, kBlock, 0, s>>>(vals, estart, ostart, nb, tf, n_ut, nse, bb, out.se_src, out.se_label,
                                             out.se_dst);
    }
    hip_check(hipGetLastError(), "unpack launch");
}

}  // namespace bsim
