// bsim_internal.h -- shared definitions of the gfx950 k-bisimulation library.
//
// Everything here is integer-only.  The hash spec (see bsim.h) is written out
// once more for the device; it follows the published SplitMix64 output
// function (Steele, Lea & Flood, OOPSLA 2014).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <atomic>
#include <string>
#include <vector>

#include "bsim.h"
#include "bsim_host.h"

namespace bsim {

// ---------------------------------------------------------------- hash spec

__host__ __device__ constexpr uint64_t mix64(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

constexpr uint64_t kCT = mix64(1);  // type-set domain
constexpr uint64_t kCL = mix64(2);  // edge-label salt domain
constexpr uint64_t kCS = mix64(3);  // signature-sum domain
constexpr uint64_t kCE = mix64(4);  // per-pair domain

// ---------------------------------------------------------- launch geometry
//
// The refinement kernel works on "tiles": runs of consecutive vertices whose
// out-edges are contiguous in the CSR.  A tile holds at most kTileMaxVerts
// vertices and fewer than kTileMaxEdges edges, so its per-vertex
// de-duplication tables (two slots per edge) fit one block's LDS.  Vertices
// with kTileMaxEdges or more out-edges ("hubs") are cut into chunks of
// kTileMaxEdges edges whose blocks write their mixed pair keys to a per-hub
// scratch area; a second launch de-duplicates each hub's keys in LDS, split
// by the top key bits into buckets that fit a large LDS table.
//
// Classes.  Every alive vertex v keeps rep[v], a member of its current
// class.  The k-class of v is (its (k-1)-class, h^k(v)) (the bisimulation
// definition: k-bisimilar requires (k-1)-bisimilar), so after h^k is known
// a vertex stays with its representative iff h^k(v) == h^k(rep[v]); the
// others "split off" and meet the other members of their new class in a
// global table keyed by (rep, h^k).  Only split-offs touch that table, so a
// late iteration of a long chain run inserts a handful of keys.

constexpr int kBlock = 256;              // threads per block (4 wave64s)
// The refinement kernel is latency bound: its speed follows the number of
// blocks resident per CU, which its LDS sets (160 KiB per CU).  Tiles of
// fewer than 1,536 edges keep a block under 32 KiB, five blocks per CU.
constexpr int kTileMaxEdges = 1536;      // a tile holds fewer edges than this
constexpr int kTileMaxVerts = 256;
constexpr int kEdgesPerThread = kTileMaxEdges / kBlock;  // 6
constexpr int kTableSlots = 2 * kTileMaxEdges;           // 3072 x 8 B = 24 KiB
constexpr uint32_t kHubMinDegree = kTileMaxEdges;  // a hub would not fit an empty tile
// A hub of at most kSoloMaxEdges edges is a "solo" block of the refinement
// launch: one block gathers all its edges and de-duplicates them in one
// table over the block's tile arrays (kSoloSlots, a prime, with double
// hashing, load <= 0.9); larger hubs take the chunk / bucket path.
constexpr uint32_t kSoloMaxEdges = 2 * kTileMaxEdges;   // 3072
constexpr uint32_t kSoloSlots = 3449;                   // prime, 27,592 B
constexpr int kSoloPerThread = (kSoloMaxEdges + kBlock - 1) / kBlock;  // 12
// Vertices without out-edges: h^k = M(t ^ M(C_S)) for every k >= 1, so they
// need no tile.  Light blocks of kIsoPerBlock of them run their split test
// and write their hash while it can still change the buffers (levels 1 and 2
// when two buffers alternate; every level when each level has its own array).
constexpr int kIsoPerThread = 4;
constexpr uint32_t kIsoPerBlock = kBlock * kIsoPerThread;
constexpr int kHubBlock = 512;           // threads per hub-bucket block
constexpr int kMaxHubLogB = 8;           // at most 256 hash buckets per hub
constexpr uint32_t kHubTableDefault = 4096;  // LDS slots per hub-bucket block (32 KiB)
constexpr int kHubOffStride = (1 << kMaxHubLogB) + 1;  // bucket offsets per hub chunk
constexpr int kStripes = 64;             // striped per-level claim counters
constexpr int kStripeRing = 4;
constexpr int kListPerStripe = 4096;     // claimed split-table slots remembered per stripe
constexpr uint32_t kNoRep = 0xFFFFFFFEu; // virtual class of every vertex before level 0

// Device-side status of a refinement run.
// Launch k normally tests level k-2, splits level k-1 and hashes level k
// (kPhaseFused).  Near a fixpoint it can run as two launches: kPhaseSplit
// (stop test of level k-2, split of level k-1, no hashes), then kPhaseHash
// (stop test of level k-1, which the split launch completed, then h^k), so
// a run that stops at level k-1 computes no h^k.
constexpr uint32_t kPhaseFused = 0;
constexpr uint32_t kPhaseSplit = 1;
constexpr uint32_t kPhaseHash = 2;

struct RunStatus {
    uint32_t done;      // sticky: set by the first launch that sees the stop condition
    uint32_t k_done;
    uint32_t fixpoint;
    uint32_t error;     // validation / capacity error bits
    uint32_t max_label;
    uint32_t max_types;
    uint32_t pad[2];
};

constexpr uint32_t kErrInvalid = 1u;
constexpr uint32_t kErrRange = 2u;
constexpr uint32_t kErrHubSplit = 8u;   // a hub bucket could not be split small enough
constexpr uint32_t kMaxHubExtraBits = 24;  // re-split depth of an overflowing hub bucket

// The split table of one level (two alternate by level parity).  A slot is
// one class's owner word ((rep + 1) << 32) | owner, 0 when empty; the class
// key is the owner's hash at that level.
struct SplitTable {
    uint64_t* slots;      // cap slots, all zero between uses
    uint32_t* list;       // kStripes * kListPerStripe claimed slot indices
    uint32_t mask;        // cap - 1
};

// Per-graph control of a batched run: many independent graphs refined as one
// disjoint union.  Level-0 classes are keyed by a virtual class per graph, so
// no class spans two graphs; every graph has its own stop test, and once a
// graph has stopped at level L its vertices keep rep (level L classes) and
// the hash buffer of parity L untouched.  gid == nullptr: not batched.
struct BatchCtl {
    const uint32_t* gid = nullptr;  // vertex -> graph
    uint32_t* done_level = nullptr; // per graph: level it stopped at, UINT32_MAX while running
    uint32_t* fix = nullptr;        // per graph: 1 if it stopped at its fixpoint
    uint32_t* hist = nullptr;       // [hist_cap][n_graphs] classes founded per level
    uint32_t* n_done = nullptr;     // graphs stopped so far
    uint32_t n_graphs = 0;
    uint32_t hist_cap = 0;
    uint32_t virt_base = 0;         // level-0 virtual class of graph g: virt_base + g
    // per graph: 1 when the persistent small-graph launch refines it (the
    // refinement launches then leave its vertices alone), nullable
    const uint8_t* ext = nullptr;
};

// The small graphs of a batched run, refined to their fixpoints inside one
// workgroup's LDS each (bsim_small.hip) instead of by the union's launches.
struct SmallPlan {
    const uint32_t* glist = nullptr;  // graph ids, largest first
    uint32_t n_small = 0;
    const uint64_t* voff = nullptr;   // union vertex offsets (G + 1)
    uint32_t* queue = nullptr;        // work-queue counter
    uint32_t max_v = 0, max_e = 0;    // capacities of one workgroup
    uint32_t max_n = 0;               // vertices of the largest listed graph
    uint32_t grid = 0;                // persistent workgroups
};

// Arguments of one refinement launch k: split test of level k-1, h^k.
struct IterArgs {
    const uint32_t* row_off;
    const uint32_t* tgt;
    const void* lab;
    const uint64_t* t;      // type hashes t(v)
    const uint64_t* salt;   // salt(l) for l <= max label
    const uint64_t* h_prev; // h^{k-1}
    uint64_t* h_next;       // h^k
    const uint8_t* alive;   // nullable
    uint32_t* rep;
    const uint32_t* tile_i0;    // tile = positions [i0, i1) of the tile-vertex list
    const uint32_t* tile_i1;
    const uint32_t* tile_e0;    // and its edges [e0, e1)
    const uint32_t* tile_e1;
    const uint32_t* act;        // tile vertices (out-degree 1..kHubMinDegree-1), ascending
    const uint32_t* iso;        // vertices without out-edges, ascending
    const uint32_t* hc_hub;     // hub chunk block -> hub index
    const uint32_t* hc_e0;      // hub chunk block -> first edge
    const uint32_t* hub_v;
    const uint32_t* hub_logb;
    const uint64_t* hub_key_off;  // first scratch key of the hub
    uint64_t* hub_keys;
    uint32_t* hub_boff;           // per hub chunk: kHubOffStride bucket offsets
    SplitTable test_tab;    // receives the split-offs of level k-1
    SplitTable clr_tab;     // filled at level k-2, cleared here
    uint32_t* lcnt;         // [kStripeRing][kStripes] claims per level
    uint32_t* totals;       // totals[j] = n_j
    RunStatus* status;
    const uint32_t* solo_v;     // solo hub vertices
    uint32_t n_tiles;
    uint32_t n_hub_chunks;
    uint32_t n_solo;
    uint32_t n_iso;
    uint32_t n_iso_blocks;
    uint32_t all_levels;    // every level has its own hash array (else two alternate)
    uint32_t k;
    uint32_t k_max;
    uint32_t stop;
    uint32_t hash_only;     // h^k only: no stop test, split test or recycling
    uint32_t phase;         // kPhaseFused, or one half of a split launch (kPhaseSplit, kPhaseHash)
    uint32_t stop_only;     // one workgroup that records the stop the host already knows of
    BatchCtl bc;
};

// Arguments of the hub-bucket launch of iteration k.
struct HubArgs {
    const uint64_t* t;
    const uint64_t* hub_keys;
    const uint64_t* hub_key_off;
    const uint32_t* hub_boff;
    const uint32_t* hub_chunk0;
    const uint32_t* hub_nchunks;
    const uint32_t* hc_e0;
    const uint32_t* hub_v;
    const uint32_t* hub_deg;
    const uint32_t* hub_logb;
    const uint32_t* hb_hub;
    const uint32_t* hb_bucket;
    uint64_t* hub_acc;
    uint64_t* h_next;
    RunStatus* status;
    uint32_t table_slots;   // LDS slots (power of two)
    uint32_t table_limit;   // re-split a bucket beyond this many keys
    uint32_t k;
    BatchCtl bc;
};

// ------------------------------------------------------------ host helpers

// Test hook for the failure paths: the N-th device allocation from the time
// it is set fails as if the device were out of memory (process-wide; 0 =
// off).  Set with the ctx option "fail_alloc_after".
extern std::atomic<int64_t> g_fail_alloc_countdown;

// Every device allocation of the library goes through here.
inline hipError_t device_alloc(void** p, size_t bytes, hipStream_t s) {
    int64_t c = g_fail_alloc_countdown.load(std::memory_order_relaxed);
    while (c > 0) {
        if (g_fail_alloc_countdown.compare_exchange_weak(c, c - 1)) {
            if (c == 1) {
                *p = nullptr;
                return hipErrorOutOfMemory;
            }
            break;
        }
    }
    return hipMallocAsync(p, bytes, s);
}

// Stream-ordered device allocations released together (error paths included).
class Arena {
  public:
    explicit Arena(hipStream_t s) : stream_(s) {}
    ~Arena() { release(); }
    Arena(const Arena&) = delete;
    Arena& operator=(const Arena&) = delete;
    // Serve allocations from [base, base + cap) first, by bumping an offset:
    // memory the caller owns, idle on the arena's stream, that outlives the
    // arena.  What does not fit comes from the stream-ordered pool.
    void back(void* base, size_t cap) {
        base_ = static_cast<char*>(base);
        cap_ = base ? cap : 0;
        used_ = 0;
    }
    // Serve every allocation from the backing memory: one that does not fit
    // throws BSIM_E_UNSUPPORTED instead of reaching the pool.
    void set_strict(bool strict) { strict_ = strict; }
    template <typename T>
    T* alloc(size_t count) {
        void* p = nullptr;
        size_t bytes = count * sizeof(T);
        if (bytes == 0) bytes = 16;
        bytes = (bytes + 255) & ~size_t(255);
        demand_ += bytes;
        if (used_ + bytes <= cap_) {
            p = base_ + used_;
            used_ += bytes;
            return static_cast<T*>(p);
        }
        if (strict_)
            throw DeviceError{BSIM_E_UNSUPPORTED, "the temporaries need more than the " + std::to_string(cap_) +
                                                      " bytes of scratch memory"};
        if (device_alloc(&p, bytes, stream_) != hipSuccess)
            throw DeviceError{BSIM_E_NOMEM, "device allocation of " + std::to_string(bytes) + " bytes failed"};
        ptrs_.push_back(p);
        return static_cast<T*>(p);
    }
    // Hand a pool allocation over to the caller (it leaves the arena).
    void detach(void* p) {
        if (cap_ && static_cast<char*>(p) >= base_ && static_cast<char*>(p) < base_ + cap_)
            throw DeviceError{BSIM_E_DEVICE, "internal: backed arena memory cannot leave the arena"};
        for (auto& q : ptrs_)
            if (q == p) q = nullptr;
    }
    void release() {
        for (void* p : ptrs_)
            if (p) (void)hipFreeAsync(p, stream_);
        ptrs_.clear();
        used_ = 0;
    }
    // Bytes asked for so far, backed or not.
    size_t demand() const { return demand_; }

  private:
    hipStream_t stream_;
    std::vector<void*> ptrs_;
    char* base_ = nullptr;
    size_t cap_ = 0, used_ = 0, demand_ = 0;
    bool strict_ = false;
};

inline void hip_check(hipError_t e, const char* what) {
    if (e != hipSuccess)
        throw DeviceError{e == hipErrorOutOfMemory ? BSIM_E_NOMEM : BSIM_E_DEVICE,
                          std::string(what) + ": " + hipGetErrorString(e)};
}

inline uint32_t ceil_div(uint64_t a, uint64_t b) { return static_cast<uint32_t>((a + b - 1) / b); }

inline uint64_t next_pow2(uint64_t x) {
    uint64_t p = 1;
    while (p < x) p <<= 1;
    return p;
}

// Largest open-addressing table the library builds: slot indices and masks
// are 32-bit.
constexpr uint64_t kMaxTableSlots = 1ull << 32;

// Slot count of a power-of-two table with at least `want` slots (and at
// least `min_slots`); BSIM_E_UNSUPPORTED when that is more than
// kMaxTableSlots, so that a 32-bit mask (slots - 1) always covers it.
inline uint64_t table_slots(uint64_t want, uint64_t min_slots, const char* what) {
    const uint64_t cap = next_pow2(want > min_slots ? want : min_slots);
    if (cap > kMaxTableSlots)
        throw DeviceError{BSIM_E_UNSUPPORTED, std::string(what) + " would need more than 2^32 table slots"};
    return cap;
}

// Split / class table of a graph with n vertices: at most n joins per level,
// load <= 2/3.
inline uint64_t split_table_slots(uint64_t n) { return table_slots(n + n / 2 + 1, 64, "the class table"); }

// ------------------------------------------------------- library internals

// Exclusive prefix sum of n uint32 values (out may alias in); the total is
// written to total_dev[0] when total_dev is non-null.
void scan_exclusive(const uint32_t* in, uint32_t* out, uint32_t n, uint32_t* total_dev,
                    Arena& arena, hipStream_t s);

// Graph after staging: device CSR plus the tile / hub schedule.
struct Staged {
    uint32_t n = 0;
    uint64_t m = 0;
    uint32_t label_bytes = 4;
    const uint32_t* row_off = nullptr;
    const uint32_t* tgt = nullptr;
    const void* lab = nullptr;
    const uint32_t* type_off = nullptr;
    const uint32_t* type_ids = nullptr;
    const uint8_t* alive = nullptr;
    const uint32_t* src = nullptr;   // per-edge source (COO), when there is no tile schedule
    uint32_t max_label = 0;
    // the edges were checked before (a resident state's own CSR, or a view
    // built from a staged graph): staging skips the per-edge pass and keeps
    // max_label (an upper bound) as given
    bool trusted = false;
    // labels >= in_label_base (when nonzero) stand for incoming edges of
    // label l - in_label_base: salted as label l - in_label_base + 2^31
    uint32_t in_label_base = 0;
    uint64_t* salt = nullptr;
    uint32_t n_tiles = 0;
    uint32_t* tile_i0 = nullptr;     // tile: positions [i0, i1) of `act`, edges [e0, e1)
    uint32_t* tile_i1 = nullptr;
    uint32_t* tile_e0 = nullptr;
    uint32_t* tile_e1 = nullptr;
    uint32_t n_act = 0;
    uint32_t* act = nullptr;         // vertices of out-degree 1..kHubMinDegree-1
    uint32_t n_iso = 0;
    uint32_t* iso = nullptr;         // vertices without out-edges (dead ones included)
    uint32_t n_hubs = 0;             // all hubs: n_hubs - n_solo chunked ones, then the solo ones
    uint32_t n_solo = 0;
    uint32_t n_hub_chunks = 0;
    uint32_t n_hub_blocks = 0;       // hub-bucket blocks of the second launch
    uint32_t* hub_v = nullptr;       // by degree, descending (solo hubs last)
    uint32_t* hub_deg = nullptr;
    uint32_t* hub_logb = nullptr;
    uint32_t* hub_chunk0 = nullptr;   // first chunk block of the hub
    uint32_t* hub_nchunks = nullptr;
    uint64_t* hub_key_off = nullptr;
    uint64_t hub_keys_total = 0;
    uint32_t* hc_hub = nullptr;
    uint32_t* hc_e0 = nullptr;
    uint32_t* hb_hub = nullptr;
    uint32_t* hb_bucket = nullptr;
    uint32_t hub_table_slots = 0;
    std::vector<uint32_t> host_hub_v;
    std::vector<uint32_t> host_hub_deg;
};

// Validate the CSR and build the tile / hub schedule (a1).  Throws
// DeviceError with BSIM_E_INVALID / BSIM_E_RANGE on malformed input.
void stage_graph(Staged& g, RunStatus* status_dev, RunStatus* status_host, Arena& arena,
                 hipStream_t s);

// The graphs of the direction and label parameterizations (Sec. 2.4), built
// on the device from a staged graph g: f = the edges whose label is in
// *labels (all edges for labels == nullptr), with per-edge sources, for the
// summary edges; h = the graph the signatures read (f, f reversed for
// BSIM_BACKWARD, f plus f reversed on labels max_label + 1 + l for
// BSIM_BOTH_DIRECTIONS), to be staged and refined.  Arrays live in arena.
struct DirectedView {
    Staged f;
    Staged h;
};
void direction_view(const Staged& g, uint32_t flags, const std::vector<uint32_t>* labels, DirectedView& out,
                    Arena& arena, hipStream_t s);

// Per-run buffers of the refinement loop.
struct RunBuffers {
    uint64_t* t = nullptr;
    uint64_t* h[2] = {nullptr, nullptr};
    uint32_t* rep = nullptr;
    SplitTable tab[2];
    uint32_t* lcnt = nullptr;      // [kStripeRing * kStripes]
    uint32_t* totals = nullptr;    // [k_cap]
    uint32_t k_cap = 0;
    uint64_t* hub_keys = nullptr;
    uint32_t* hub_boff = nullptr;
    uint64_t* hub_acc = nullptr;
    RunStatus* status = nullptr;
    BatchCtl bc;                   // batched runs only
    SmallPlan small;               // batched runs only
};

void alloc_run_buffers(const Staged& g, uint32_t k_max, bool stop, RunBuffers& rb, Arena& arena,
                       hipStream_t s);

// Level 0: type hashes, h^0 = t, the type classes (rep) and n_0.
void launch_init(const Staged& g, const RunBuffers& rb, bool untyped, hipStream_t s);

// Launch k: stop test, split test of level k-1, h^k (tiles and hub chunks),
// or one half of it (phase; see kPhaseFused).  stop_only: the hash half of a
// launch whose split half ended the run (the host has read the founded
// count): a single workgroup takes the stop decision and records it, where
// the whole grid would only dispatch and exit.
void launch_iteration(const Staged& g, const RunBuffers& rb, uint32_t k, uint32_t k_max,
                      bool stop, bool all_levels, hipStream_t s, uint32_t phase = kPhaseFused,
                      bool stop_only = false);

// Hub buckets of iteration k (only when the graph has hubs and k <= k_max).
void launch_hubs(const Staged& g, const RunBuffers& rb, uint32_t k, hipStream_t s);

// Scratch of hash-only launches (hub keys and per-hub sums).
struct HashScratch {
    uint64_t* hub_keys = nullptr;
    uint32_t* hub_boff = nullptr;
    uint64_t* hub_acc = nullptr;   // zero, kept zero by the launches
    RunStatus* status = nullptr;   // zero (never done)
};
void alloc_hash_scratch(const Staged& g, HashScratch& hs, Arena& arena, hipStream_t s);
// h_next = h^level from h_prev = h^{level-1} for every vertex of a staged
// graph, with the refinement kernels in hash-only mode.
void launch_hash_level(const Staged& g, const uint64_t* t, const uint64_t* h_prev, uint64_t* h_next,
                       const HashScratch& hs, uint32_t level, hipStream_t s);

// Batched runs: per-graph stop test of level k-2, before launch k.
void launch_graph_stop(const RunBuffers& rb, uint32_t k, uint32_t k_max, bool stop, hipStream_t s);

// Batched runs: LDS bytes of a small-graph workgroup with the given
// capacities (and its hash-table slots), and the launch that refines the
// graphs of `sp` to their stop levels (after launch_init).
uint64_t small_graph_lds_bytes(uint32_t max_v, uint32_t max_e, uint32_t* tab_slots);
void launch_small_graphs(const Staged& g, const RunBuffers& rb, const SmallPlan& sp, uint32_t k_max, bool stop,
                         hipStream_t s);

// LDS slots the hub-bucket launch can use on this device.
// device_max: the largest table the device allows (else the default size).
uint32_t query_hub_table_slots(int device, bool device_max = false);

// Sort m 64-bit keys ascending on bits [0, bits); returns a or b, whichever
// holds the result.
uint64_t* radix_sort(uint64_t* a, uint64_t* b, uint32_t m, int bits, Arena& arena, hipStream_t s);

// Finalize (a8): block ids, block sizes, sorted distinct quotient edges.
struct FinalOut {
    // preset: the output arrays below are already allocated by the caller
    // (block_ids and block_sizes for n + 1 entries, the summary-edge columns
    // for m + 1), and finalize allocates none of them
    bool preset = false;
    uint32_t n_blocks = 0;
    uint64_t n_se = 0;
    uint32_t* block_ids = nullptr;
    uint32_t* block_sizes = nullptr;
    uint32_t* se_src = nullptr;
    uint32_t* se_label = nullptr;
    uint32_t* se_dst = nullptr;
};

// Class index of a resident state, one per level (bsim_cindex.hip): a hash
// table of the level's classes keyed by (class at level j-1, h^j) with
// member counts, and the class (table slot) of every vertex.
constexpr uint32_t kNoClass = 0xFFFFFFFFu;
struct CiLevel {
    uint64_t* slot;   // [2 cap] pairs: slot[2 s] = 0 (empty) or (level j-1 class + 1) << 32 | owner,
                      // slot[2 s + 1] = the key's hash (one 16-byte line per probe)
    uint32_t* cnt;    // [cap] members
    uint32_t* cid;    // [vertices] class slot, kNoClass for a dead vertex
    uint32_t mask;    // cap - 1
};
// Every vertex from scratch; ctr[0] = classes, ctr[1] = claimed slots; the
// member counts are left cleared for ci_count.
void ci_rebuild(const CiLevel& L, uint64_t cap, const uint32_t* cid_prev, const uint64_t* h, const uint8_t* alive,
                uint32_t n, uint64_t* ctr, hipStream_t s);
// The member counts of a rebuilt level (vertices < n).
void ci_count(const CiLevel& L, uint32_t n, hipStream_t s);
// d = (candidates of a with flag[v] == ftag, or all of a when flag is null)
// plus b, each vertex once (dmark[v] = dtag marks it); counts from the _dev
// pointers when given; *nd = its length.
void ci_list(const uint32_t* a, uint32_t na, const uint32_t* na_dev, const uint32_t* flag, uint32_t ftag,
             const uint32_t* b, uint32_t nb, const uint32_t* nb_dev, uint32_t* dmark, uint32_t dtag, uint32_t* d,
             uint32_t* nd, uint32_t grid, hipStream_t s);
// Re-key the nd vertices of d; q / *nq = those whose class changed.
// ctr[0] changes by the classes born less those gone (mod 2^64), ctr[1] by
// the slots claimed.  The table must have at least nd free slots; a full
// one sets *err (device) instead of probing on.  host_word: pinned scratch
// for one count.
void ci_update(const CiLevel& L, const uint32_t* cid_prev, const uint64_t* h, const uint8_t* alive,
               const uint32_t* d, uint32_t nd, uint64_t* ctr, uint32_t* q, uint32_t* nq, uint32_t* err,
               uint32_t* host_word, Arena& arena, hipStream_t s);

// Summary edges of a CSR graph with a tile schedule, bucketed by source
// block (bid, nb blocks) and sorted within each block; false from the fit
// test means the keys or the layout need the global sort instead.
bool bucketed_summary_edges_fit(const Staged& g, int lb, int bb);
void bucketed_summary_edges(const Staged& g, const uint32_t* bid, uint32_t nb, const uint32_t* dst_ids, int lb,
                            int bb, FinalOut& out, Arena& arena, Arena& keep, hipStream_t s);

// Blocks are the classes given by rep[] (first-occurrence numbering).
void finalize(const Staged& g, const uint32_t* rep, bool want_edges, FinalOut& out, Arena& arena,
              Arena& keep, hipStream_t s, uint64_t n_ids = 0);

}  // namespace bsim
