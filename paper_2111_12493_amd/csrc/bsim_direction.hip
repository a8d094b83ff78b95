// Direction and label parameterizations (Sec. 2.4; backward bisimulation,
// Sec. 2.5) as graph views in front of the unchanged refinement kernels.
//
// From a staged, validated graph g the device builds
//   f  the kept edges: those whose label is in the label set P_l (all edges
//      when there is none), in their own direction, with a per-edge source;
//      the summary edges are taken from f;
//   h  the graph the signatures read: f itself (forward), f reversed
//      (backward: the pairs of w are its incoming edges (v, l, w)), or f
//      plus f reversed (both), the reversed copies on labels L + l with
//      L = max label + 1.  The salt table of h maps label L + l to
//      M(C_L + 2^31 + l), so an incoming l-edge is salted as an outgoing
//      edge of label l + 2^31 (a range input labels never reach).
// Every step is a streaming pass or a scatter over the edges; the order of
// the edges within a row of h does not matter, since a signature is a set.
#include "bsim_internal.h"

namespace bsim {
namespace {

__global__ void __launch_bounds__(kBlock) k_label_mask(const uint32_t* __restrict__ ids, uint32_t n_ids,
                                                       uint8_t* __restrict__ mask, uint32_t mask_size) {
    const uint32_t i = blockIdx.x * kBlock + threadIdx.x;
    if (i < n_ids && ids[i] < mask_size) mask[ids[i]] = 1;
}

template <typename LabT>
__global__ void __launch_bounds__(kBlock) k_keep_flags(const LabT* __restrict__ lab, uint32_t m,
                                                       const uint8_t* __restrict__ mask,
                                                       uint32_t* __restrict__ keep) {
    const uint32_t e = blockIdx.x * kBlock + threadIdx.x;
    if (e < m) keep[e] = mask[static_cast<uint32_t>(lab[e])];
}

// Row offsets of the kept edges: f_row_off[v] = kept edges before row v.
__global__ void __launch_bounds__(kBlock) k_kept_rows(const uint32_t* __restrict__ row_off, uint32_t n, uint32_t m,
                                                      const uint32_t* __restrict__ kpos,
                                                      const uint32_t* __restrict__ m_kept,
                                                      uint32_t* __restrict__ f_row_off) {
    const uint32_t v = blockIdx.x * kBlock + threadIdx.x;
    if (v > n) return;
    const uint32_t e = row_off[v];
    f_row_off[v] = e < m ? kpos[e] : *m_kept;
}

// Copy every kept edge (all edges when keep is null) to its position, with
// the row it leaves from: the largest v with row_off[v] <= e.
template <typename LabT>
__global__ void __launch_bounds__(kBlock) k_kept_edges(const uint32_t* __restrict__ row_off, uint32_t n,
                                                       const uint32_t* __restrict__ tgt,
                                                       const LabT* __restrict__ lab, uint32_t m,
                                                       const uint32_t* __restrict__ keep,
                                                       const uint32_t* __restrict__ kpos,
                                                       uint32_t* __restrict__ f_src, uint32_t* __restrict__ f_tgt,
                                                       LabT* __restrict__ f_lab) {
    const uint32_t e = blockIdx.x * kBlock + threadIdx.x;
    if (e >= m || (keep && !keep[e])) return;
    uint32_t lo = 0, hi = n;  // row_off[lo] <= e < row_off[hi]
    while (hi - lo > 1) {
        const uint32_t mid = lo + (hi - lo) / 2;
        if (row_off[mid] <= e) lo = mid; else hi = mid;
    }
    const uint32_t p = keep ? kpos[e] : e;
    f_src[p] = lo;
    f_tgt[p] = tgt[e];
    f_lab[p] = lab[e];
}

__global__ void __launch_bounds__(kBlock) k_count_targets(const uint32_t* __restrict__ tgt, uint32_t m,
                                                          uint32_t* __restrict__ indeg) {
    const uint32_t e = blockIdx.x * kBlock + threadIdx.x;
    if (e < m) atomicAdd(&indeg[tgt[e]], 1u);
}

// Both directions: a row holds the vertex's kept out-edges, then its kept
// in-edges; cursor[v] starts where the in-edges begin.
__global__ void __launch_bounds__(kBlock) k_both_degrees(const uint32_t* __restrict__ f_row_off,
                                                         const uint32_t* __restrict__ indeg, uint32_t n,
                                                         uint32_t* __restrict__ deg) {
    const uint32_t v = blockIdx.x * kBlock + threadIdx.x;
    if (v < n) deg[v] = (f_row_off[v + 1] - f_row_off[v]) + indeg[v];
}

__global__ void __launch_bounds__(kBlock) k_both_cursor(const uint32_t* __restrict__ f_row_off,
                                                        const uint32_t* __restrict__ h_row_off, uint32_t n,
                                                        uint32_t* __restrict__ cursor) {
    const uint32_t v = blockIdx.x * kBlock + threadIdx.x;
    if (v < n) cursor[v] = h_row_off[v] + (f_row_off[v + 1] - f_row_off[v]);
}

template <typename LabT>
__global__ void __launch_bounds__(kBlock) k_copy_out(const uint32_t* __restrict__ f_src,
                                                     const uint32_t* __restrict__ f_tgt,
                                                     const LabT* __restrict__ f_lab,
                                                     const uint32_t* __restrict__ f_row_off, uint32_t m,
                                                     const uint32_t* __restrict__ h_row_off,
                                                     uint32_t* __restrict__ h_tgt, uint32_t* __restrict__ h_lab) {
    const uint32_t e = blockIdx.x * kBlock + threadIdx.x;
    if (e >= m) return;
    const uint32_t v = f_src[e];
    const uint32_t p = h_row_off[v] + (e - f_row_off[v]);
    h_tgt[p] = f_tgt[e];
    h_lab[p] = static_cast<uint32_t>(f_lab[e]);
}

// Each kept edge (v, l, w) as the edge (w, l + label_add, v) of row w.
template <typename LabT>
__global__ void __launch_bounds__(kBlock) k_scatter_reverse(const uint32_t* __restrict__ f_src,
                                                            const uint32_t* __restrict__ f_tgt,
                                                            const LabT* __restrict__ f_lab, uint32_t m,
                                                            uint32_t label_add, uint32_t* __restrict__ cursor,
                                                            uint32_t* __restrict__ h_tgt,
                                                            uint32_t* __restrict__ h_lab) {
    const uint32_t e = blockIdx.x * kBlock + threadIdx.x;
    if (e >= m) return;
    const uint32_t p = atomicAdd(&cursor[f_tgt[e]], 1u);
    h_tgt[p] = f_src[e];
    h_lab[p] = static_cast<uint32_t>(f_lab[e]) + label_add;
}

template <typename LabT>
void build_view(const Staged& g, uint32_t flags, const std::vector<uint32_t>* labels, DirectedView& out,
                Arena& arena, hipStream_t s) {
    const uint32_t n = g.n, m = static_cast<uint32_t>(g.m);
    const LabT* lab = static_cast<const LabT*>(g.lab);
    Staged& f = out.f;
    f = Staged{};
    f.n = n;
    f.label_bytes = g.label_bytes;
    f.type_off = g.type_off;
    f.type_ids = g.type_ids;
    f.alive = g.alive;
    f.max_label = g.max_label;
    f.hub_table_slots = g.hub_table_slots;
    // the kept edges
    uint32_t m_f = m;
    const uint32_t* keep = nullptr;
    const uint32_t* kpos = nullptr;
    uint32_t* f_row_off = arena.alloc<uint32_t>(static_cast<size_t>(n) + 1);
    if (labels) {
        const uint32_t mask_size = g.max_label + 1;
        uint8_t* mask = arena.alloc<uint8_t>(mask_size);
        hip_check(hipMemsetAsync(mask, 0, mask_size, s), "label mask");
        if (!labels->empty()) {
            uint32_t* ids = arena.alloc<uint32_t>(labels->size());
            hip_check(hipMemcpyAsync(ids, labels->data(), labels->size() * 4, hipMemcpyHostToDevice, s),
                      "label set");
            const uint32_t ni = static_cast<uint32_t>(labels->size());
            k_label_mask<<<ceil_div(ni, kBlock), kBlock, 0, s>>>(ids, ni, mask, mask_size);
        }
        uint32_t* kf = arena.alloc<uint32_t>(static_cast<size_t>(m) + 1);
        uint32_t* kp = arena.alloc<uint32_t>(static_cast<size_t>(m) + 1);
        uint32_t* total = arena.alloc<uint32_t>(1);
        if (m) k_keep_flags<LabT><<<ceil_div(m, kBlock), kBlock, 0, s>>>(lab, m, mask, kf);
        scan_exclusive(kf, kp, m, total, arena, s);
        k_kept_rows<<<ceil_div(static_cast<uint64_t>(n) + 1, kBlock), kBlock, 0, s>>>(g.row_off, n, m, kp, total,
                                                                                      f_row_off);
        hip_check(hipMemcpyAsync(&m_f, total, 4, hipMemcpyDeviceToHost, s), "kept edge count");
        hip_check(hipStreamSynchronize(s), "kept edge count");
        keep = kf;
        kpos = kp;
    } else {
        hip_check(hipMemcpyAsync(f_row_off, g.row_off, (static_cast<size_t>(n) + 1) * 4, hipMemcpyDeviceToDevice, s),
                  "rows");
    }
    f.m = m_f;
    f.row_off = f_row_off;
    uint32_t* f_src = arena.alloc<uint32_t>(static_cast<size_t>(m_f) + 1);
    uint32_t* f_tgt = arena.alloc<uint32_t>(static_cast<size_t>(m_f) + 1);
    LabT* f_lab = arena.alloc<LabT>(static_cast<size_t>(m_f) + 1);
    if (m) k_kept_edges<LabT><<<ceil_div(m, kBlock), kBlock, 0, s>>>(g.row_off, n, g.tgt, lab, m, keep, kpos, f_src,
                                                                     f_tgt, f_lab);
    f.src = f_src;
    f.tgt = f_tgt;
    f.lab = f_lab;
    hip_check(hipGetLastError(), "kept edges");

    Staged& h = out.h;
    if (!(flags & (BSIM_BACKWARD | BSIM_BOTH_DIRECTIONS))) {
        h = f;
        h.src = nullptr;  // h gets a tile schedule of its own
        h.trusted = true;
        return;
    }
    const bool both = (flags & BSIM_BOTH_DIRECTIONS) != 0;
    const uint64_t m_h = both ? 2ull * m_f : m_f;
    if (m_h >= (1ull << 32))
        throw DeviceError{BSIM_E_UNSUPPORTED, "both edge directions together reach 2^32 edges"};
    const uint32_t L = g.max_label + 1;
    if (both && L > (1u << 24)) throw DeviceError{BSIM_E_UNSUPPORTED, "edge labels must be < 2^24"};
    uint32_t* indeg = arena.alloc<uint32_t>(static_cast<size_t>(n) + 1);
    hip_check(hipMemsetAsync(indeg, 0, (static_cast<size_t>(n) + 1) * 4, s), "in-degrees");
    if (m_f) k_count_targets<<<ceil_div(m_f, kBlock), kBlock, 0, s>>>(f_tgt, m_f, indeg);
    uint32_t* h_row_off = arena.alloc<uint32_t>(static_cast<size_t>(n) + 1);
    uint32_t* cursor = arena.alloc<uint32_t>(static_cast<size_t>(n) + 1);
    uint32_t* h_tgt = arena.alloc<uint32_t>(m_h + 1);
    uint32_t* h_lab = arena.alloc<uint32_t>(m_h + 1);
    const uint32_t gn = std::max<uint32_t>(ceil_div(n, kBlock), 1);
    if (both) {
        uint32_t* deg = arena.alloc<uint32_t>(static_cast<size_t>(n) + 1);
        if (n) k_both_degrees<<<gn, kBlock, 0, s>>>(f_row_off, indeg, n, deg);
        scan_exclusive(deg, h_row_off, n, h_row_off + n, arena, s);
        if (n) k_both_cursor<<<gn, kBlock, 0, s>>>(f_row_off, h_row_off, n, cursor);
        if (m_f) {
            k_copy_out<LabT><<<ceil_div(m_f, kBlock), kBlock, 0, s>>>(f_src, f_tgt, f_lab, f_row_off, m_f, h_row_off,
                                                                      h_tgt, h_lab);
            k_scatter_reverse<LabT><<<ceil_div(m_f, kBlock), kBlock, 0, s>>>(f_src, f_tgt, f_lab, m_f, L, cursor,
                                                                             h_tgt, h_lab);
        }
    } else {
        scan_exclusive(indeg, h_row_off, n, h_row_off + n, arena, s);
        hip_check(hipMemcpyAsync(cursor, h_row_off, static_cast<size_t>(n) * 4, hipMemcpyDeviceToDevice, s),
                  "cursors");
        if (m_f)
            k_scatter_reverse<LabT><<<ceil_div(m_f, kBlock), kBlock, 0, s>>>(f_src, f_tgt, f_lab, m_f, 0u, cursor,
                                                                             h_tgt, h_lab);
    }
    hip_check(hipGetLastError(), "direction view");
    h = Staged{};
    h.n = n;
    h.m = m_h;
    h.label_bytes = 4;
    h.row_off = h_row_off;
    h.tgt = h_tgt;
    h.lab = h_lab;
    h.type_off = g.type_off;
    h.type_ids = g.type_ids;
    h.alive = g.alive;
    h.hub_table_slots = g.hub_table_slots;
    h.max_label = both ? 2 * L - 1 : g.max_label;
    h.in_label_base = both ? L : 0;
    h.trusted = true;
}

}  // namespace

void direction_view(const Staged& g, uint32_t flags, const std::vector<uint32_t>* labels, DirectedView& out,
                    Arena& arena, hipStream_t s) {
    if (g.label_bytes == 2)
        build_view<uint16_t>(g, flags, labels, out, arena, s);
    else
        build_view<uint32_t>(g, flags, labels, out, arena, s);
}

}  // namespace bsim
