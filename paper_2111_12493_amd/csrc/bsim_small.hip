// bsim_small.hip -- persistent refinement of the small graphs of a batch.
//
// In a batched run (bsim_batch.hip) every graph is refined by the same
// launches over the disjoint union, so a launch costs the whole union's
// edges and a small graph that needs more levels than the large ones keeps
// the run going.  This launch takes the small graphs out of that loop: a
// persistent grid of workgroups pulls graph after graph from a work queue
// and refines each one to its own fixpoint (or cap) inside the workgroup's
// LDS, with no global synchronization between levels.  Per level it does
// what a refinement launch does for one graph (Algorithm 4's message phase
// and the class split of Sec. 2.5's definition):
//   - every edge (v, l, w) forms the key h^{k-1}(w) ^ salt(l) from the LDS
//     copy of the previous level; the keys of each vertex are de-duplicated
//     in its own region of an LDS hash table (two slots per edge) and the
//     mixed distinct keys summed into h^k(v) = M(t(v) ^ M(C_S + sum));
//   - a vertex whose h^k differs from its class representative's founds or
//     joins the class (representative, h^k) in an LDS table; the number of
//     classes founded is n_k - n_{k-1}, and the run stops at the first level
//     that founds none (with the fixpoint test) or at k_max.
// The launch runs after the level-0 pass of the union (type hashes, level-0
// classes and their counts) and leaves exactly what the refinement loop
// leaves for a graph that stopped at level L: h^L in the hash buffer of
// parity L, the level-L class representatives in rep (union ids), the
// per-level founded counts, the stop level and the fixpoint flag, and the
// graph counted as done.  Later launches of the loop skip these graphs.
#include "bsim_device.h"

namespace bsim {
namespace {

constexpr int kSmallBlock = 512;
constexpr uint32_t kDead = 0xFFFFFFFFu;

struct SmallArgs {
    const uint32_t* row_off;
    const uint32_t* tgt;
    const void* lab;
    const uint64_t* t;
    const uint64_t* salt;
    uint64_t* h0;
    uint64_t* h1;
    uint32_t* rep;
    const uint32_t* glist;   // small graphs, largest first
    uint32_t n_small;
    const uint64_t* voff;    // union vertex offset of every graph (G + 1 entries)
    uint32_t* queue;         // next position in glist (zero at launch)
    BatchCtl bc;
    RunStatus* status;
    uint32_t k_max;
    uint32_t stop;
    uint32_t max_v;          // LDS capacity: vertices and edges of one graph
    uint32_t max_e;
    uint32_t tab_slots;      // LDS hash-table slots: >= 2 max_e and a power of two >= 2 max_v
};

// LDS class table: slot = ((r + 1) << 32) | owner, 0 = empty; the class key
// is the owner's hash.  Returns the owner of class (r, key) and sets
// *founded when this call created it.
__device__ uint32_t small_join(uint64_t* tab, uint32_t mask, const uint64_t* h, uint32_t r, uint64_t key,
                               uint32_t v, uint32_t* founded) {
    const uint64_t mine = (static_cast<uint64_t>(r + 1) << 32) | v;
    uint32_t slot = (static_cast<uint32_t>(key) ^ (r * 0x9E3779B9u)) & mask;
    for (;;) {
        uint64_t cur = lds_peek(&tab[slot]);
        if (cur == 0) {
            cur = atomicCAS(reinterpret_cast<unsigned long long*>(&tab[slot]), 0ull,
                            static_cast<unsigned long long>(mine));
            if (cur == 0) {
                *founded = 1;
                return v;
            }
        }
        if ((cur >> 32) == static_cast<uint64_t>(r + 1) && h[static_cast<uint32_t>(cur)] == key)
            return static_cast<uint32_t>(cur);
        slot = (slot + 1) & mask;
    }
}

template <typename LabT>
__global__ void __launch_bounds__(kSmallBlock) k_small_graphs(SmallArgs a) {
    extern __shared__ uint64_t smem[];
    __shared__ uint32_t s_g, s_founded;
    const uint32_t tid = threadIdx.x;
    const uint32_t MV = a.max_v, ME = a.max_e;
    uint64_t* salt_e = smem;                 // [ME] salt of each edge's label
    uint64_t* tt = salt_e + ME;              // [MV] t(v)
    uint64_t* hA = tt + MV;                  // [MV] two level buffers
    uint64_t* hB = hA + MV;
    uint64_t* acc = hB + MV;                 // [MV] sums of distinct mixed keys
    uint64_t* tab = acc + MV;                // [tab_slots] de-dup regions, then the class table
    uint32_t* off = reinterpret_cast<uint32_t*>(tab + a.tab_slots);  // [MV + 1]
    uint32_t* tl = off + MV + 1;             // [ME] local targets
    uint32_t* rl = tl + ME;                  // [MV] local class representatives (kDead: dead)
    uint16_t* seg = reinterpret_cast<uint16_t*>(rl + MV);  // [ME] owning vertex of each edge
    const LabT* __restrict__ lab = static_cast<const LabT*>(a.lab);
    const uint32_t G = a.bc.n_graphs;
    for (;;) {
        if (tid == 0) s_g = atomicAdd(a.queue, 1u);
        __syncthreads();
        const uint32_t qi = s_g;
        if (qi >= a.n_small) return;  // uniform: every thread read the same s_g
        const uint32_t g = a.glist[qi];
        const uint32_t v0 = static_cast<uint32_t>(a.voff[g]);
        const uint32_t n = static_cast<uint32_t>(a.voff[g + 1]) - v0;
        const uint32_t e0 = a.row_off[v0];
        const uint32_t m = a.row_off[v0 + n] - e0;
        // the host lists only graphs within the capacities; a graph beyond
        // them would overrun LDS, so it is left to the refinement loop
        if (n > MV || m > ME) {
            __syncthreads();
            continue;
        }
        for (uint32_t i = tid; i <= n; i += kSmallBlock) off[i] = a.row_off[v0 + i] - e0;
        for (uint32_t j = tid; j < m; j += kSmallBlock) {
            tl[j] = a.tgt[e0 + j] - v0;
            salt_e[j] = a.salt[static_cast<uint32_t>(lab[e0 + j])];
        }
        for (uint32_t i = tid; i < n; i += kSmallBlock) {
            const uint32_t r = a.rep[v0 + i];
            rl[i] = r == kDead ? kDead : r - v0;
            tt[i] = a.t[v0 + i];
            hA[i] = tt[i];  // h^0 = t (0 for a dead vertex)
        }
        __syncthreads();
        for (uint32_t i = tid; i < n; i += kSmallBlock)
            for (uint32_t j = off[i]; j < off[i + 1]; j++) seg[j] = static_cast<uint16_t>(i);
        uint64_t* hp = hA;
        uint64_t* hn = hB;
        uint32_t k_done = 0, fix = 0;
        uint32_t mask = 1;
        while (mask < 2 * n) mask <<= 1;
        mask -= 1;
        for (uint32_t k = 1; k <= a.k_max; k++) {
            for (uint32_t j = tid; j < 2 * m; j += kSmallBlock) tab[j] = 0;
            for (uint32_t i = tid; i < n; i += kSmallBlock) acc[i] = 0;
            __syncthreads();
            // h^k: distinct keys per vertex in its region [2 off[i], 2 off[i+1])
            for (uint32_t j = tid; j < m; j += kSmallBlock) {
                const uint64_t f = mix64((hp[tl[j]] ^ salt_e[j]) ^ kCE);
                if (f == 0) continue;  // a zero term adds nothing, repeated or not
                const uint32_t i = seg[j];
                const uint32_t lo = 2 * off[i], hi = 2 * off[i + 1];
                const uint32_t slot = lo + static_cast<uint32_t>(
                                               (static_cast<uint64_t>(static_cast<uint32_t>(f)) * (hi - lo)) >> 32);
                if (lds_insert(tab, slot, lo, hi, f))
                    atomicAdd(reinterpret_cast<unsigned long long*>(&acc[i]), static_cast<unsigned long long>(f));
            }
            __syncthreads();
            for (uint32_t i = tid; i < n; i += kSmallBlock)
                hn[i] = rl[i] == kDead ? 0 : mix64(tt[i] ^ mix64(kCS + acc[i]));
            for (uint32_t j = tid; j <= mask; j += kSmallBlock) tab[j] = 0;
            if (tid == 0) s_founded = 0;
            __syncthreads();
            // classes of level k: split every class by h^k
            uint32_t mine = 0;
            for (uint32_t i = tid; i < n; i += kSmallBlock) {
                const uint32_t r = rl[i];
                if (r == kDead || r == i || hn[i] == hn[r]) continue;
                uint32_t founded = 0;
                rl[i] = small_join(tab, mask, hn, r, hn[i], i, &founded);
                mine += founded;
            }
            mine = wave_sum_u32(mine);
            if (lane_id() == 0 && mine) atomicAdd(&s_founded, mine);
            __syncthreads();
            const uint32_t founded = s_founded;
            if (tid == 0) a.bc.hist[static_cast<size_t>(k) * G + g] = founded;
            uint64_t* sw = hp;
            hp = hn;
            hn = sw;
            k_done = k;
            fix = founded == 0 ? 1u : 0u;
            __syncthreads();
            if (a.stop && fix) break;
        }
        uint64_t* hout = (k_done & 1) ? a.h1 : a.h0;
        for (uint32_t i = tid; i < n; i += kSmallBlock) {
            hout[v0 + i] = hp[i];
            a.rep[v0 + i] = rl[i] == kDead ? kDead : rl[i] + v0;
        }
        if (tid == 0) {
            a.bc.done_level[g] = k_done;
            a.bc.fix[g] = fix;
            if (atomicAdd(a.bc.n_done, 1u) + 1 == G) {
                a.status->k_done = k_done;
                a.status->fixpoint = fix;
                a.status->done = 1;
            }
        }
        __syncthreads();
    }
}

}  // namespace

uint64_t small_graph_lds_bytes(uint32_t max_v, uint32_t max_e, uint32_t* tab_slots) {
    uint32_t cls = 1;
    while (cls < 2 * max_v) cls <<= 1;
    const uint32_t slots = std::max<uint32_t>(2 * max_e, cls);
    if (tab_slots) *tab_slots = slots;
    return 8ull * (max_e + 4ull * max_v + slots) + 4ull * (max_v + 1 + max_e + max_v) + 2ull * max_e + 16;
}

void launch_small_graphs(const Staged& g, const RunBuffers& rb, const SmallPlan& sp, uint32_t k_max, bool stop,
                         hipStream_t s) {
    if (!sp.n_small) return;
    SmallArgs a{};
    a.row_off = g.row_off;
    a.tgt = g.tgt;
    a.lab = g.lab;
    a.t = rb.t;
    a.salt = g.salt;
    a.h0 = rb.h[0];
    a.h1 = rb.h[1];
    a.rep = rb.rep;
    a.glist = sp.glist;
    a.n_small = sp.n_small;
    a.voff = sp.voff;
    a.queue = sp.queue;
    a.bc = rb.bc;
    a.status = rb.status;
    a.k_max = k_max;
    a.stop = stop ? 1u : 0u;
    a.max_v = sp.max_v;
    a.max_e = sp.max_e;
    const uint64_t bytes = small_graph_lds_bytes(sp.max_v, sp.max_e, &a.tab_slots);
    hip_check(hipMemsetAsync(sp.queue, 0, 4, s), "small-graph queue");
    const uint32_t grid = std::min<uint32_t>(sp.n_small, sp.grid);
    // (the capacities were chosen below the device's per-workgroup LDS limit)
    if (g.label_bytes == 2) {
        (void)hipFuncSetAttribute(reinterpret_cast<const void*>(k_small_graphs<uint16_t>),
                                  hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(bytes));
        k_small_graphs<uint16_t><<<grid, kSmallBlock, bytes, s>>>(a);
    } else {
        (void)hipFuncSetAttribute(reinterpret_cast<const void*>(k_small_graphs<uint32_t>),
                                  hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(bytes));
        k_small_graphs<uint32_t><<<grid, kSmallBlock, bytes, s>>>(a);
    }
    hip_check(hipGetLastError(), "small-graph launch");
}

}  // namespace bsim
