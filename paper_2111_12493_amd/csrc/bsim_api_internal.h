// bsim_api_internal.h -- host-side objects behind the opaque ABI handles.
#pragma once

#include <map>
#include <memory>
#include <string>
#include <vector>

#include "bsim_internal.h"

struct bsim_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    std::string err;
    bsim::RunStatus* status_host = nullptr;  // pinned, 4 entries
    hipEvent_t loop_ev[2] = {nullptr, nullptr};  // status-copy events of the refinement loop
    uint32_t chunk_max = 32;
    uint32_t time_launches = 0;
    uint32_t hub_table_slots = 8192;  // LDS slots per hub-bucket block on this device
    uint32_t frontier_limit_pct = 10;  // incremental: larger frontiers recompute the level for all vertices
    uint32_t frontier_edge_pct = 15;   // ... and so do frontiers with more than this share of the edges
    // one launch per stop check: once a level founds at most this many
    // classes per million vertices, the next level's split runs on its own
    uint32_t tail_split_ppm = 100;
    uint32_t* count_host = nullptr;   // pinned: a level's founded counts (kStripes entries)
    // batched calls: schedules picked by the autotuner, per size class
    uint32_t autotune = 1;
    struct BatchTune {
        uint64_t small_edges;       // graphs of at most this many edges go to the small-graph launch
        uint32_t hub_table_slots;   // LDS slots of a hub-bucket block
    };
    std::map<uint64_t, BatchTune> batch_tune;
    BatchTune last_batch{0, 0};     // what the last batched call ran with
    uint64_t fixed_small_edges = ~0ull;  // the schedule when autotune is off
    // temporaries of summarize and batched calls: one device buffer, grown
    // to the largest demand of the earlier calls (keep_work = 0: every call
    // takes them from the stream-ordered pool and returns them)
    uint32_t keep_work = 1;
    void* work = nullptr;
    size_t work_cap = 0, work_want = 0;
};

namespace bsim {

// Arrays shared by several results (the per-graph results of one batched
// call are views into the batch's arrays); freed with the last holder.
struct SharedArrays {
    int device = 0;
    hipStream_t stream = nullptr;
    std::vector<void*> device_ptrs;
    std::vector<void*> host_ptrs;
    ~SharedArrays();
};

// Owner of a result's arrays.
struct ResultPriv {
    int device = 0;
    hipStream_t stream = nullptr;
    std::vector<void*> device_ptrs;
    std::vector<void*> host_ptrs;
    std::vector<uint32_t> blocks_per_iter;
    std::shared_ptr<SharedArrays> shared;
};

// Device copies of the caller's graph when it arrives in host memory, or
// the caller's device pointers as they are.
struct DeviceGraph {
    Staged g;
};

void upload_graph(const bsim_graph& in, Staged& g, Arena& arena, hipStream_t s);

// Per-level hash storage handed to the refinement loop.  With `levels`
// empty the loop double-buffers; otherwise levels[k] receives h^k.
struct LevelSink {
    std::vector<uint64_t*> levels;
};

struct LoopResult {
    uint32_t k_done = 0;
    uint32_t fixpoint = 0;
    uint32_t launches = 0;
    uint32_t split_launches = 0;  // launches run as a split half and a hash half
    float ms_kernels = 0.f;      // refinement launches that did work
    float ms_hub_kernels = 0.f;  // hub launches of those iterations
    uint32_t n_timed = 0;        // launches the two sums cover
    std::vector<uint32_t> blocks_per_iter;
    const uint64_t* h_final = nullptr;
};

// Iterations 0..k_done on a staged graph.  rep_prev (nullable, n entries)
// receives the class representatives of level k_done - 1 (of level 0 when
// k_done = 0; at a fixpoint those of level k_done, the same partition).
// use_timers: bracket launches with HIP events when the ctx option asks for
// it (the allocation-free entry point passes false).
LoopResult run_refinement(bsim_ctx* ctx, const Staged& g, const bsim_params& p, RunBuffers& rb,
                          LevelSink* sink, Arena& arena, uint32_t* rep_prev = nullptr, bool use_timers = true);

// The allocation-free entry point's scratch: its device address on the
// current device, looked up once per device (bsim_ctx_create calls it).
int noalloc_scratch_init(int device, std::string* err);

// finalize with summary edges into the classes named by rep_prev (their
// first-occurrence block ids) instead of the final blocks.
void finalize_prev_level(const Staged& g, const uint32_t* rep, const uint32_t* rep_prev, bool want_edges,
                         FinalOut& out, Arena& arena, Arena& keep, hipStream_t s);

// Assemble a bsim_result from finalize output (takes ownership of `keep`);
// hashes_preset: an array of n entries in `keep` to receive the hashes.
bsim_result* make_result(bsim_ctx* ctx, const Staged& g, const LoopResult& lr, const uint64_t* h,
                         FinalOut& fo, Arena& keep, uint32_t flags, uint64_t* hashes_preset = nullptr);

// Whole batch path for one graph; labels = the kept label set of the label
// parameterization (nullptr: every edge).
bsim_result* summarize_graph(bsim_ctx* ctx, const bsim_graph& graph, const bsim_params& p,
                             const std::vector<uint32_t>* labels);

// Many independent graphs in one refinement run (a disjoint union); graphs
// of at most small_edges edges (0: none) that fit one workgroup go to the
// persistent small-graph launch.
void batch_summarize(bsim_ctx* ctx, const bsim_graph* graphs, uint32_t n_graphs, const bsim_params& p,
                     bsim_result** outs, uint64_t small_edges);

// Batch path that also returns a resident state for incremental updates.
int summarize_with_state(bsim_ctx* ctx, const bsim_graph& graph, const bsim_params& p,
                         bsim_state** state_out, bsim_result** out);

// directions: whether the caller takes BSIM_BACKWARD / BSIM_BOTH_DIRECTIONS
// (only the single-graph summarization does).
void validate_params(const bsim_graph& graph, const bsim_params& p, bool directions = false);

// Back `arena` with the ctx's work buffer, grown first to the largest
// demand of the ctx's earlier calls and to at_least bytes (what does not
// fit comes from the pool; a failed growth leaves the arena on the pool).
// ctx_note_demand records a finished call's demand; ctx_release_work frees
// the buffer.
void ctx_back_arena(bsim_ctx* ctx, Arena& arena, size_t at_least = 0);
void ctx_note_demand(bsim_ctx* ctx, const Arena& arena);
void ctx_release_work(bsim_ctx* ctx);

// Device bytes a resident state holds.
uint64_t state_bytes(const bsim_state* st);
// The context a state runs on.
bsim_ctx* state_ctx(const bsim_state* st);

}  // namespace bsim
