// bsim_stage.hip -- staging of a graph for the refinement kernels (a1) and
// the device prefix sum the library uses.
//
// Staging validates the CSR (paper Sec. 3.1 Phase 0 co-locates every vertex
// with its out-edges; here that is the out-edge CSR itself), computes the
// label salts, and cuts the vertex range into tiles and hub buckets:
//   * a vertex with kHubMinDegree or more out-edges (too many for one tile)
//     is a hub;
//   * every other vertex belongs to exactly one tile, a run of consecutive
//     non-hub vertices packed greedily (within windows of kPackWindow
//     vertices, one thread per window) up to kTileMaxEdges - 1 edges and
//     kTileMaxVerts vertices; a non-hub vertex always fits an empty tile;
//   * a hub of degree d is cut into chunks of kTileMaxEdges edges that write
//     its mixed pair keys to d scratch slots, and into 2^b hash buckets that
//     each fit the LDS table of the hub-bucket launch.
#include <algorithm>

#include "bsim_resolve.h"  // host_radix_sort
#include "bsim_internal.h"

namespace bsim {

// ------------------------------------------------------------------ scan

namespace {

constexpr int kScanItems = 4;
constexpr int kScanTile = kBlock * kScanItems;  // 1024 values per block

__device__ inline uint32_t wave_incl_scan(uint32_t x) {
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        uint32_t y = __shfl_up(x, d, 64);
        if (lane >= d) x += y;
    }
    return x;
}

// Exclusive scan of one value per thread across the block; returns the
// thread's exclusive prefix and the block total in *total.
__device__ inline uint32_t block_excl_scan(uint32_t x, uint32_t* total) {
    __shared__ uint32_t s_w[kBlock / 64];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    uint32_t inc = wave_incl_scan(x);
    if (lane == 63) s_w[wid] = inc;
    __syncthreads();
    uint32_t off = 0, tot = 0;
#pragma unroll
    for (int i = 0; i < kBlock / 64; i++) {
        if (i < wid) off += s_w[i];
        tot += s_w[i];
    }
    __syncthreads();
    *total = tot;
    return off + inc - x;
}

__global__ void __launch_bounds__(kBlock) k_scan_reduce(const uint32_t* __restrict__ in, uint32_t n,
                                                        uint32_t* __restrict__ sums) {
    const uint64_t base = static_cast<uint64_t>(blockIdx.x) * kScanTile;
    uint32_t x = 0;
#pragma unroll
    for (int i = 0; i < kScanItems; i++) {
        uint64_t j = base + static_cast<uint64_t>(i) * kBlock + threadIdx.x;
        if (j < n) x += in[j];
    }
    uint32_t tot;
    (void)block_excl_scan(x, &tot);
    if (threadIdx.x == 0) sums[blockIdx.x] = tot;
}

__global__ void __launch_bounds__(1024) k_scan_spine(uint32_t* __restrict__ sums, uint32_t nb,
                                                    uint32_t* __restrict__ total) {
    __shared__ uint32_t s_w[16];
    __shared__ uint32_t s_carry;
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (threadIdx.x == 0) s_carry = 0;
    __syncthreads();
    for (uint32_t base = 0; base < nb; base += 1024) {
        uint32_t j = base + threadIdx.x;
        uint32_t x = j < nb ? sums[j] : 0;
        uint32_t inc = wave_incl_scan(x);
        if (lane == 63) s_w[wid] = inc;
        __syncthreads();
        uint32_t off = 0, tot = 0;
        for (int i = 0; i < 16; i++) {
            if (i < wid) off += s_w[i];
            tot += s_w[i];
        }
        uint32_t carry = s_carry;
        if (j < nb) sums[j] = carry + off + inc - x;
        __syncthreads();
        if (threadIdx.x == 0) s_carry = carry + tot;
        __syncthreads();
    }
    if (threadIdx.x == 0 && total) *total = s_carry;
}

__global__ void __launch_bounds__(kBlock) k_scan_down(const uint32_t* in, uint32_t* out, uint32_t n,
                                                      const uint32_t* __restrict__ sums) {
    const uint64_t base = static_cast<uint64_t>(blockIdx.x) * kScanTile +
                          static_cast<uint64_t>(threadIdx.x) * kScanItems;
    uint32_t v[kScanItems];
    uint32_t x = 0;
#pragma unroll
    for (int i = 0; i < kScanItems; i++) {
        v[i] = (base + i < n) ? in[base + i] : 0;
        x += v[i];
    }
    uint32_t tot;
    uint32_t run = block_excl_scan(x, &tot) + sums[blockIdx.x];
#pragma unroll
    for (int i = 0; i < kScanItems; i++) {
        if (base + i < n) out[base + i] = run;
        run += v[i];
    }
}

}  // namespace

void scan_exclusive(const uint32_t* in, uint32_t* out, uint32_t n, uint32_t* total_dev,
                    Arena& arena, hipStream_t s) {
    if (n == 0) {
        if (total_dev) hip_check(hipMemsetAsync(total_dev, 0, sizeof(uint32_t), s), "scan");
        return;
    }
    uint32_t nb = ceil_div(n, kScanTile);
    uint32_t* sums = arena.alloc<uint32_t>(nb);
    k_scan_reduce<<<nb, kBlock, 0, s>>>(in, n, sums);
    k_scan_spine<<<1, 1024, 0, s>>>(sums, nb, total_dev);
    k_scan_down<<<nb, kBlock, 0, s>>>(in, out, n, sums);
    hip_check(hipGetLastError(), "scan launch");
}

// --------------------------------------------------------------- staging

namespace {

__global__ void __launch_bounds__(kBlock) k_stage_vertices(
    const uint32_t* __restrict__ row_off, const uint32_t* __restrict__ type_off,
    const uint8_t* __restrict__ alive, uint32_t n, uint64_t m, uint32_t* __restrict__ hubf,
    uint32_t* __restrict__ actf, uint32_t* __restrict__ isof, RunStatus* status) {
    uint32_t v = blockIdx.x * kBlock + threadIdx.x;
    const bool in = v < n;
    if (!in) v = n - 1;  // inactive lanes mirror the last vertex and store nothing
    uint32_t a = row_off[v], b = row_off[v + 1];
    uint32_t err = 0;
    if (b < a) err |= kErrInvalid;
    if (type_off[v + 1] < type_off[v]) err |= kErrInvalid;
    if (v == 0 && (a != 0 || type_off[0] != 0)) err |= kErrInvalid;
    if (v == n - 1 && static_cast<uint64_t>(b) != m) err |= kErrInvalid;
    uint32_t d = b - a;
    if (alive && !alive[v] && (d != 0)) err |= kErrInvalid;
    uint32_t nt = type_off[v + 1] - type_off[v];
    // one atomic per block: same-address atomics from every wave would serialize
    __shared__ uint32_t s_max[kBlock / 64];
    uint32_t wmax = in ? nt : 0;
    for (int dd = 32; dd >= 1; dd >>= 1)
        wmax = max(wmax, static_cast<uint32_t>(__shfl_xor(static_cast<int>(wmax), dd, 64)));
    if ((threadIdx.x & 63) == 0) s_max[threadIdx.x >> 6] = wmax;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int i = 1; i < kBlock / 64; i++) wmax = max(wmax, s_max[i]);
        // the maximum only grows: a block that cannot raise it (nearly all
        // of them once a few have run) issues no atomic at all
        if (wmax && wmax > __hip_atomic_load(&status->max_types, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
            atomicMax(&status->max_types, wmax);
    }
    bool hub = (b >= a) && d >= kHubMinDegree;
    if (in) {
        hubf[v] = hub ? 1u : 0u;
        actf[v] = (b > a && !hub) ? 1u : 0u;
        isof[v] = (b <= a) ? 1u : 0u;
        if (err) atomicOr(&status->error, err);
    }
}

template <typename LabT>
__global__ void __launch_bounds__(kBlock) k_stage_edges(const uint32_t* __restrict__ tgt,
                                                        const LabT* __restrict__ lab,
                                                        const uint8_t* __restrict__ alive,
                                                        uint32_t n, uint64_t m, RunStatus* status) {
    uint32_t err = 0, mx = 0;
    for (uint64_t e = static_cast<uint64_t>(blockIdx.x) * kBlock + threadIdx.x; e < m;
         e += static_cast<uint64_t>(gridDim.x) * kBlock) {
        uint32_t w = tgt[e];
        if (w >= n) err |= kErrRange;
        else if (alive && !alive[w]) err |= kErrInvalid;
        mx = max(mx, static_cast<uint32_t>(lab[e]));
    }
    // reduce over the block before touching global memory
    __shared__ uint32_t s_mx[kBlock / 64], s_err[kBlock / 64];
    for (int d = 32; d >= 1; d >>= 1) {
        mx = max(mx, static_cast<uint32_t>(__shfl_xor(static_cast<int>(mx), d, 64)));
        err |= static_cast<uint32_t>(__shfl_xor(static_cast<int>(err), d, 64));
    }
    if ((threadIdx.x & 63) == 0) {
        s_mx[threadIdx.x >> 6] = mx;
        s_err[threadIdx.x >> 6] = err;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int i = 1; i < kBlock / 64; i++) {
            mx = max(mx, s_mx[i]);
            err |= s_err[i];
        }
        if (mx && mx > __hip_atomic_load(&status->max_label, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
            atomicMax(&status->max_label, mx);
        if (err) atomicOr(&status->error, err);
    }
}

__global__ void __launch_bounds__(kBlock) k_compact_flags(const uint32_t* __restrict__ flag,
                                                          const uint32_t* __restrict__ pos,
                                                          uint32_t n, uint32_t* __restrict__ out) {
    uint32_t v = blockIdx.x * kBlock + threadIdx.x;
    if (v < n && flag[v]) out[pos[v]] = v;
}

// Greedy tile packing within windows of kPackWindow consecutive entries of
// the tile-vertex list (one wave per window): a tile grows until the next
// vertex would bring it to kTileMaxEdges edges or kTileMaxVerts vertices, or
// its edges would not follow the tile's (a hub lies between).  The wave
// loads the window's edge ranges together into LDS, then one lane runs the
// greedy scan over them.  With emit == false only the tile count per window
// is written (to cnt[w]); with emit == true tiles are written from pos[w] on.
constexpr uint32_t kPackWindow = 1024;
constexpr uint32_t kPackWaves = kBlock / 64;

__global__ void __launch_bounds__(kBlock) k_pack_tiles(const uint32_t* __restrict__ row_off,
                                                       const uint32_t* __restrict__ act, uint32_t n_act,
                                                       bool emit, uint32_t* __restrict__ cnt,
                                                       const uint32_t* __restrict__ pos,
                                                       uint32_t* __restrict__ i0, uint32_t* __restrict__ i1,
                                                       uint32_t* __restrict__ e0, uint32_t* __restrict__ e1) {
    __shared__ uint32_t s_a[kPackWaves][kPackWindow];
    __shared__ uint32_t s_b[kPackWaves][kPackWindow];
    const uint32_t lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const uint32_t w = blockIdx.x * kPackWaves + wv;
    const uint64_t ib64 = static_cast<uint64_t>(w) * kPackWindow;
    if (ib64 >= n_act) return;  // whole waves only: no block barrier below
    const uint32_t ib = static_cast<uint32_t>(ib64);
    const uint32_t ie = static_cast<uint32_t>(min<uint64_t>(n_act, ib64 + kPackWindow));
    for (uint32_t i = ib + lane; i < ie; i += 64) {
        const uint32_t v = act[i];
        s_a[wv][i - ib] = row_off[v];
        s_b[wv][i - ib] = row_off[v + 1];
    }
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    if (lane != 0) return;
    const uint32_t* A = s_a[wv];
    const uint32_t* B = s_b[wv];
    uint32_t out = emit ? pos[w] : 0, made = 0;
    uint32_t start = ib, edges = 0, verts = 0, ebeg = 0, eend = 0;
    for (uint32_t i = ib; i < ie; i++) {
        const uint32_t a = A[i - ib], b = B[i - ib];
        const uint32_t d = b - a;
        if (verts && (a != eend || verts == static_cast<uint32_t>(kTileMaxVerts) ||
                      edges + d >= static_cast<uint32_t>(kTileMaxEdges))) {
            if (emit) {
                i0[out] = start;
                i1[out] = i;
                e0[out] = ebeg;
                e1[out] = eend;
                out++;
            }
            made++;
            verts = edges = 0;
        }
        if (!verts) {
            start = i;
            ebeg = a;
        }
        edges += d;
        verts++;
        eend = b;
    }
    if (verts) {
        if (emit) {
            i0[out] = start;
            i1[out] = ie;
            e0[out] = ebeg;
            e1[out] = eend;
            out++;
        }
        made++;
    }
    if (!emit) cnt[w] = made;
}

__global__ void __launch_bounds__(kBlock) k_hub_degrees(const uint32_t* __restrict__ row_off,
                                                         const uint32_t* __restrict__ hubs,
                                                         uint32_t nh, uint32_t* __restrict__ deg) {
    uint32_t i = blockIdx.x * kBlock + threadIdx.x;
    if (i < nh) deg[i] = row_off[hubs[i] + 1] - row_off[hubs[i]];
}

__global__ void __launch_bounds__(kBlock) k_hub_starts(const uint32_t* __restrict__ row_off,
                                                        const uint32_t* __restrict__ hubs,
                                                        uint32_t nh, uint32_t* __restrict__ start) {
    uint32_t i = blockIdx.x * kBlock + threadIdx.x;
    if (i < nh) start[i] = row_off[hubs[i]];
}

// salt(l) = M(C_L + l); at and past in_base (when nonzero) the salts of
// incoming edges: label in_base + l is salted as label l + 2^31
__global__ void __launch_bounds__(kBlock) k_salt(uint64_t* salt, uint32_t count, uint32_t in_base) {
    uint32_t l = blockIdx.x * kBlock + threadIdx.x;
    if (l >= count) return;
    const uint64_t x = (in_base && l >= in_base) ? 0x80000000ull + (l - in_base) : static_cast<uint64_t>(l);
    salt[l] = mix64(kCL + x);
}

}  // namespace

void stage_graph(Staged& g, RunStatus* status_dev, RunStatus* status_host, Arena& arena,
                 hipStream_t s) {
    const uint32_t n = g.n;
    hip_check(hipMemsetAsync(status_dev, 0, sizeof(RunStatus), s), "stage status");
    uint32_t* hubf = arena.alloc<uint32_t>(n + 1);
    uint32_t* actf = arena.alloc<uint32_t>(n + 1);
    uint32_t* isof = arena.alloc<uint32_t>(n + 1);
    uint32_t* counts = arena.alloc<uint32_t>(8);
    hip_check(hipMemsetAsync(counts, 0, 8 * 4, s), "stage counts");
    if (n > 0) {
        k_stage_vertices<<<ceil_div(n, kBlock), kBlock, 0, s>>>(g.row_off, g.type_off, g.alive, n,
                                                                g.m, hubf, actf, isof, status_dev);
        if (g.m > 0 && !g.trusted) {
            uint32_t nbk = std::min<uint64_t>(ceil_div(g.m, kBlock), 2048);
            if (g.label_bytes == 2)
                k_stage_edges<uint16_t><<<nbk, kBlock, 0, s>>>(
                    g.tgt, static_cast<const uint16_t*>(g.lab), g.alive, n, g.m, status_dev);
            else
                k_stage_edges<uint32_t><<<nbk, kBlock, 0, s>>>(
                    g.tgt, static_cast<const uint32_t*>(g.lab), g.alive, n, g.m, status_dev);
        }
        hip_check(hipGetLastError(), "stage launch");
    }
    // hubs -> hub list
    uint32_t* hpos = arena.alloc<uint32_t>(n + 1);
    scan_exclusive(hubf, hpos, n, counts + 1, arena, s);
    uint32_t* hubs = arena.alloc<uint32_t>(n + 1);
    if (n) k_compact_flags<<<ceil_div(n, kBlock), kBlock, 0, s>>>(hubf, hpos, n, hubs);
    // tile vertices and vertices without out-edges -> lists
    uint32_t* apos = arena.alloc<uint32_t>(n + 1);
    uint32_t* ipos = arena.alloc<uint32_t>(n + 1);
    scan_exclusive(actf, apos, n, counts + 4, arena, s);
    scan_exclusive(isof, ipos, n, counts + 5, arena, s);
    g.act = arena.alloc<uint32_t>(n + 1);
    g.iso = arena.alloc<uint32_t>(n + 1);
    if (n) {
        k_compact_flags<<<ceil_div(n, kBlock), kBlock, 0, s>>>(actf, apos, n, g.act);
        k_compact_flags<<<ceil_div(n, kBlock), kBlock, 0, s>>>(isof, ipos, n, g.iso);
    }
    hip_check(hipMemcpyAsync(status_host, status_dev, sizeof(RunStatus), hipMemcpyDeviceToHost, s),
              "stage status");
    uint32_t hc[8];
    hip_check(hipMemcpyAsync(hc, counts, 8 * sizeof(uint32_t), hipMemcpyDeviceToHost, s), "stage counts");
    hip_check(hipStreamSynchronize(s), "stage sync");
    if (status_host->error & kErrRange)
        throw DeviceError{BSIM_E_RANGE, "edge target out of range"};
    if (status_host->error & kErrInvalid)
        throw DeviceError{BSIM_E_INVALID, "malformed CSR or an edge touching a dead vertex"};
    if (status_host->max_types > 4096)
        throw DeviceError{BSIM_E_UNSUPPORTED, "more than 4096 type ids on one vertex"};
    if (status_host->max_label >= (1u << 24))
        throw DeviceError{BSIM_E_UNSUPPORTED, "edge labels must be < 2^24"};
    if (!g.trusted) g.max_label = status_host->max_label;
    g.n_hubs = hc[1];
    g.n_act = hc[4];
    g.n_iso = hc[5];

    // tiles: greedy packing per window of the tile-vertex list
    const uint32_t nwin = ceil_div(g.n_act, kPackWindow);
    uint32_t* wcnt = arena.alloc<uint32_t>(nwin + 1);
    uint32_t* wpos = arena.alloc<uint32_t>(nwin + 1);
    if (nwin) k_pack_tiles<<<ceil_div(nwin, kPackWaves), kBlock, 0, s>>>(g.row_off, g.act, g.n_act, false, wcnt,
                                                                      nullptr, nullptr, nullptr, nullptr,
                                                                      nullptr);
    scan_exclusive(wcnt, wpos, nwin, counts + 2, arena, s);
    uint32_t ntiles = 0;
    hip_check(hipMemcpyAsync(&ntiles, counts + 2, sizeof(uint32_t), hipMemcpyDeviceToHost, s), "tiles");
    hip_check(hipStreamSynchronize(s), "tiles sync");
    g.n_tiles = ntiles;
    g.tile_i0 = arena.alloc<uint32_t>(ntiles + 1);
    g.tile_i1 = arena.alloc<uint32_t>(ntiles + 1);
    g.tile_e0 = arena.alloc<uint32_t>(ntiles + 1);
    g.tile_e1 = arena.alloc<uint32_t>(ntiles + 1);
    if (nwin) k_pack_tiles<<<ceil_div(nwin, kPackWaves), kBlock, 0, s>>>(g.row_off, g.act, g.n_act, true, nullptr,
                                                                      wpos, g.tile_i0, g.tile_i1, g.tile_e0,
                                                                      g.tile_e1);
    hip_check(hipGetLastError(), "tile packing");

    // hubs: schedule on the host (few), largest first so long buckets start early
    g.host_hub_v.assign(g.n_hubs, 0);
    g.host_hub_deg.assign(g.n_hubs, 0);
    if (g.n_hubs) {
        uint32_t* hdeg = arena.alloc<uint32_t>(g.n_hubs);
        k_hub_degrees<<<ceil_div(g.n_hubs, kBlock), kBlock, 0, s>>>(g.row_off, hubs, g.n_hubs, hdeg);
        hip_check(hipMemcpyAsync(g.host_hub_v.data(), hubs, g.n_hubs * sizeof(uint32_t),
                                 hipMemcpyDeviceToHost, s), "hubs");
        hip_check(hipMemcpyAsync(g.host_hub_deg.data(), hdeg, g.n_hubs * sizeof(uint32_t),
                                 hipMemcpyDeviceToHost, s), "hub degrees");
        hip_check(hipStreamSynchronize(s), "hubs sync");
        // by degree, largest first, ties in hub order: a stable radix sort
        // on the complemented degree (a graph of 2^30 edges has some 10^5
        // hubs, which a comparison sort orders in milliseconds)
        std::vector<uint32_t> order(g.n_hubs);
        {
            std::vector<uint64_t> key(g.n_hubs), k2;
            std::vector<uint32_t> v2;
            for (uint32_t i = 0; i < g.n_hubs; i++) {
                key[i] = 0xFFFFFFFFull - g.host_hub_deg[i];
                order[i] = i;
            }
            host_radix_sort(key, order, 32, k2, v2);
        }
        // a hub of degree d > kSoloMaxEdges: ceil(d / kTileMaxEdges) chunk
        // blocks, and 2^b bucket blocks so that a bucket expects at most 3/4
        // of the LDS slots; the others are solo blocks (no chunks, no buckets)
        const uint64_t per_bucket = std::max<uint64_t>(1, uint64_t(g.hub_table_slots) * 3 / 4);
        std::vector<uint32_t> hv(g.n_hubs), hd(g.n_hubs), hl(g.n_hubs);
        std::vector<uint64_t> ho(g.n_hubs);
        std::vector<uint32_t> ch, ce, bh, bb;
        std::vector<uint32_t> hstart(g.n_hubs);
        uint64_t keys = 0;
        uint32_t n_big = 0;
        for (uint32_t i = 0; i < g.n_hubs; i++) {
            hv[i] = g.host_hub_v[order[i]];
            hd[i] = g.host_hub_deg[order[i]];
            ho[i] = keys;
            hl[i] = 0;
            if (hd[i] <= kSoloMaxEdges) continue;
            n_big = i + 1;
            keys += hd[i];
            const uint64_t want = (hd[i] + per_bucket - 1) / per_bucket;
            hl[i] = std::min<uint32_t>(static_cast<uint32_t>(bit_width(next_pow2(want)) - 1), kMaxHubLogB);
            for (uint32_t b = 0; b < (1u << hl[i]); b++) {
                bh.push_back(i);
                bb.push_back(b);
            }
        }
        g.n_solo = g.n_hubs - n_big;
        uint32_t* hv_dev = arena.alloc<uint32_t>(g.n_hubs);
        uint32_t* hs_dev = arena.alloc<uint32_t>(g.n_hubs);
        hip_check(hipMemcpyAsync(hv_dev, hv.data(), hv.size() * 4, hipMemcpyHostToDevice, s), "hub v");
        k_hub_starts<<<ceil_div(g.n_hubs, kBlock), kBlock, 0, s>>>(g.row_off, hv_dev, g.n_hubs, hs_dev);
        hip_check(hipMemcpyAsync(hstart.data(), hs_dev, g.n_hubs * 4, hipMemcpyDeviceToHost, s), "hub starts");
        hip_check(hipStreamSynchronize(s), "hub starts sync");
        std::vector<uint32_t> hc0(g.n_hubs), hnc(g.n_hubs);
        for (uint32_t i = 0; i < g.n_hubs; i++) {
            hc0[i] = static_cast<uint32_t>(ch.size());
            hnc[i] = i < n_big ? ceil_div(hd[i], kTileMaxEdges) : 0;
            for (uint32_t c = 0; c < hnc[i]; c++) {
                ch.push_back(i);
                ce.push_back(hstart[i] + c * kTileMaxEdges);
            }
        }
        g.host_hub_v = hv;
        g.host_hub_deg = hd;
        g.n_hub_chunks = static_cast<uint32_t>(ch.size());
        g.n_hub_blocks = static_cast<uint32_t>(bh.size());
        g.hub_keys_total = keys;
        g.hub_v = hv_dev;
        g.hub_deg = arena.alloc<uint32_t>(g.n_hubs);
        g.hub_logb = arena.alloc<uint32_t>(g.n_hubs);
        g.hub_key_off = arena.alloc<uint64_t>(g.n_hubs);
        g.hub_chunk0 = arena.alloc<uint32_t>(g.n_hubs);
        g.hub_nchunks = arena.alloc<uint32_t>(g.n_hubs);
        hip_check(hipMemcpyAsync(g.hub_chunk0, hc0.data(), hc0.size() * 4, hipMemcpyHostToDevice, s), "hub c0");
        hip_check(hipMemcpyAsync(g.hub_nchunks, hnc.data(), hnc.size() * 4, hipMemcpyHostToDevice, s), "hub nc");
        g.hc_hub = arena.alloc<uint32_t>(g.n_hub_chunks);
        g.hc_e0 = arena.alloc<uint32_t>(g.n_hub_chunks);
        g.hb_hub = arena.alloc<uint32_t>(g.n_hub_blocks);
        g.hb_bucket = arena.alloc<uint32_t>(g.n_hub_blocks);
        hip_check(hipMemcpyAsync(g.hub_deg, hd.data(), hd.size() * 4, hipMemcpyHostToDevice, s), "hub deg");
        hip_check(hipMemcpyAsync(g.hub_logb, hl.data(), hl.size() * 4, hipMemcpyHostToDevice, s), "hub logb");
        hip_check(hipMemcpyAsync(g.hub_key_off, ho.data(), ho.size() * 8, hipMemcpyHostToDevice, s), "hub off");
        hip_check(hipMemcpyAsync(g.hc_hub, ch.data(), ch.size() * 4, hipMemcpyHostToDevice, s), "hub chunks");
        hip_check(hipMemcpyAsync(g.hc_e0, ce.data(), ce.size() * 4, hipMemcpyHostToDevice, s), "hub chunk e0");
        hip_check(hipMemcpyAsync(g.hb_hub, bh.data(), bh.size() * 4, hipMemcpyHostToDevice, s), "hub blocks");
        hip_check(hipMemcpyAsync(g.hb_bucket, bb.data(), bb.size() * 4, hipMemcpyHostToDevice, s), "hub buckets");
        hip_check(hipStreamSynchronize(s), "hub schedule sync");
    } else {
        g.n_hub_chunks = 0;
        g.n_hub_blocks = 0;
        g.n_solo = 0;
        g.hub_keys_total = 0;
    }

    // label salts
    uint32_t nsalt = g.max_label + 1;
    g.salt = arena.alloc<uint64_t>(nsalt);
    k_salt<<<ceil_div(nsalt, kBlock), kBlock, 0, s>>>(g.salt, nsalt, g.in_label_base);
    hip_check(hipGetLastError(), "salt launch");
}

}  // namespace bsim
