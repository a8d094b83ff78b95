/*
 * bsim.h -- C ABI of the MI355X (gfx950) hash-based k-bisimulation library.
 *
 * The library computes labeled forward k-bisimulation summaries of labeled
 * directed graphs with hash messages (paper Sec. 3.3, Algorithm 4; the
 * partition it computes is the one of Sec. 2.5's forward bisimulation with
 * the typed variant, chained as in Sec. 2.4's chaining parameterization):
 *
 *   h^0(v) = t(v)                                   hash of v's type set
 *   h^k(v) = F(t(v), SET{ (l, h^{k-1}(w)) : (v, l, w) in E })
 *
 * with the 64-bit hash spec
 *   M        = SplitMix64 output function (Steele, Lea & Flood, OOPSLA 2014)
 *   C_T..C_E = M(1), M(2), M(3), M(4)
 *   t(v)     = M(C_T + sum_{distinct types tau} M(C_T ^ tau))
 *   salt(l)  = M(C_L + l)
 *   h^k(v)   = M(t(v) ^ M(C_S + sum_{distinct q} M(q ^ C_E))),
 *              q = h^{k-1}(w) ^ salt(l) over v's out-edges (v, l, w)
 * All arithmetic wraps mod 2^64.  Blocks are numbered by first occurrence
 * (the block holding the smallest vertex id is 0).  The refinement stops at
 * the first k >= 1 whose block count equals that of k-1 (the partition is
 * then stable: maximal bisimulation refining the type partition) or at k_max.
 *
 * Conventions for every call:
 *  - Plain pointers and fixed-width integers only; no exceptions cross the
 *    ABI.  Calls return BSIM_OK (0) or a negative status; on error every
 *    output pointer is set to NULL and no state is modified.
 *  - A bsim_ctx is bound to one device and one HIP stream (borrowed from
 *    the caller).  All device work of a call is ordered on that stream; a
 *    call returns after its results are complete.  A ctx is not thread safe:
 *    use one ctx per host thread.
 *  - Input arrays are borrowed for the duration of the call only.
 *  - Every object returned by the library is owned by the library and freed
 *    with the matching *_free call, before the ctx it came from.
 */
#ifndef BSIM_H
#define BSIM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ------------------------------------------------------ */
#define BSIM_OK 0
#define BSIM_E_INVALID (-1)     /* malformed input: CSR not monotone, bad sizes, edge to a dead vertex */
#define BSIM_E_RANGE (-2)       /* an id or label out of its range */
#define BSIM_E_NOMEM (-3)       /* device or host allocation failed */
#define BSIM_E_DEVICE (-4)      /* a HIP runtime error; text in bsim_last_error */
#define BSIM_E_UNSUPPORTED (-5) /* valid input outside this library's limits */
#define BSIM_E_BUSY (-6)        /* server: request does not fit the memory budget now */
#define BSIM_E_IO (-7)          /* a file could not be opened, read or written */

/* ---- where an array lives ---------------------------------------------- */
#define BSIM_MEM_HOST 0u
#define BSIM_MEM_DEVICE 1u

/* ---- bsim_params.flags ------------------------------------------------- */
#define BSIM_STOP_AT_FIXPOINT 1u   /* stop when the block count stops growing */
#define BSIM_KEEP_LEVELS 2u        /* keep h^0..h^k resident in the returned state */
#define BSIM_UNTYPED 4u            /* ignore vertex types: t(v) = M(C_T) for all v */
#define BSIM_RESULT_ON_HOST 8u     /* copy result arrays to host memory */
#define BSIM_NO_SUMMARY_EDGES 16u  /* skip the quotient-edge output */
/* Direction parameterization (Sec. 2.4; backward bisimulation, Sec. 2.5).
 * Default: a signature reads the outgoing edges (v, l, w).  BSIM_BACKWARD:
 * it reads the incoming edges (v, l, w) of w, partner v, salt(l).
 * BSIM_BOTH_DIRECTIONS: both kinds in one set, an incoming l-edge salted as
 * an outgoing edge of label l + 2^31 would be, M(C_L + 2^31 + l).  The two
 * flags exclude each other; summary edges keep the edges' own direction.
 * bsim_summarize / bsim_summarize_labels, bsim_batch_summarize and server
 * summarize requests, without a state only (a state or a keep_state request
 * with them gives BSIM_E_UNSUPPORTED). */
#define BSIM_BACKWARD 32u
#define BSIM_BOTH_DIRECTIONS 64u
/* Previous-level summary edges (Sec. 2.6, inductive definition of vertex
 * summaries: the primary vertex of v links to the class, under the object
 * relation, of each neighbour; for the k-bisimulation that relation is the
 * (k-1)-bisimulation).  The summary edges become the distinct
 * (block(v), l, prev_block(w)), where prev_block numbers the
 * (k_done-1)-classes by first occurrence -- the block ids that a run with
 * k_max = k_done - 1 returns; at k_done = 0 both ends use the 0-classes.
 * At a fixpoint the two partitions agree and so do the two edge sets.
 * Forward direction only (with BSIM_BACKWARD or BSIM_BOTH_DIRECTIONS:
 * BSIM_E_INVALID); bsim_summarize / bsim_summarize_labels and server
 * summarize requests without a state (a state, a keep_state request or
 * bsim_batch_summarize: BSIM_E_UNSUPPORTED). */
#define BSIM_PREV_LEVEL_EDGES 128u

typedef struct bsim_ctx bsim_ctx;
typedef struct bsim_state bsim_state;

/*
 * A labeled directed graph in CSR form (Sec. 2.2 labeled property graphs:
 * each vertex has a set of type ids, each edge one label).
 *   row_off[n_vertices+1]  out-edge offsets, row_off[0] = 0, monotone,
 *                          row_off[n] = n_edges (< 2^32 in this library)
 *   targets[n_edges]       edge target vertex, < n_vertices
 *   labels[n_edges]        edge label, uint16 (label_bytes 2) or uint32 (4)
 *   type_off[n_vertices+1] offsets into type_ids (monotone)
 *   type_ids[...]          vertex type ids; repeats allowed (set semantics)
 *   alive[n_vertices]      NULL = all alive; else 0 marks a deleted vertex,
 *                          which must have no incident edge
 * Multi-edges and repeated triples are allowed and never change results.
 * mem_kind says whether all arrays are host or device pointers.
 *
 * Limits of this library (valid input beyond them gives BSIM_E_UNSUPPORTED,
 * never a truncated table): offsets and type ids are 32-bit (the paper's
 * workloads all have fewer than 2^32 edges, so one offset segment covers
 * them; there is no 8-byte offset or 2-byte type-id variant); labels < 2^24;
 * a class table of next_pow2(1.5 n + 1) slots must fit 2^32 slots (n below
 * about 2.86 * 10^9); a resident state holds at most 2^30 edges; change
 * detection needs next_pow2(2 m + 2) <= 2^32 table slots per snapshot.
 */
typedef struct {
    uint32_t n_vertices;
    uint32_t label_bytes;
    uint64_t n_edges;
    const uint32_t* row_off;
    const uint32_t* targets;
    const void* labels;
    const uint32_t* type_off;
    const uint32_t* type_ids;
    const uint8_t* alive;
    uint32_t mem_kind;
    uint32_t reserved;
} bsim_graph;

typedef struct {
    uint32_t k_max; /* iteration cap; UINT32_MAX = none (run to the fixpoint) */
    uint32_t flags; /* BSIM_* flags above */
} bsim_params;

/*
 * Result of a summarization (batch or incremental).  Arrays live where
 * mem_kind says (device unless BSIM_RESULT_ON_HOST was requested), except
 * blocks_per_iter, which is always host memory.
 *   hashes[n_vertices]       h^{k_done}(v); 0 for dead vertices
 *   block_ids[n_vertices]    first-occurrence block id; UINT32_MAX if dead
 *   block_sizes[n_blocks]    vertices per block (the count payload, Sec. 3.1)
 *   blocks_per_iter[k_done+1] number of blocks after iteration 0..k_done
 *   se_src/se_label/se_dst[n_summary_edges]  distinct quotient edges
 *                            (block(v), l, block(w)), sorted ascending by
 *                            (src, label, dst) (summary graph, Sec. 2.6)
 * Timings are device milliseconds of the call's phases.
 */
typedef struct {
    uint32_t n_vertices;
    uint32_t k_done;
    uint32_t fixpoint;
    uint32_t n_blocks;
    uint64_t n_summary_edges;
    uint32_t mem_kind;
    uint32_t n_iter_launches; /* refinement-kernel launches issued */
    uint64_t* hashes;
    uint32_t* block_ids;
    uint32_t* block_sizes;
    uint32_t* blocks_per_iter;
    uint32_t* se_src;
    uint32_t* se_label;
    uint32_t* se_dst;
    float ms_stage;
    float ms_iterate;
    float ms_finalize;
    float ms_total;
    float ms_iter_kernels; /* when the ctx option "time_launches" is N > 0: summed
                              durations of every N-th refinement-kernel launch
                              among those that hashed a level (launches
                              1..k_done+1, less launch k_done+1 when it ran
                              split; later ones return at once), else 0 */
    float ms_hub_kernels;  /* the same for the hub-vertex launches */
    uint32_t n_timed_launches; /* launches those sums cover */
    uint32_t n_split_launches; /* refinement launches run as a split half and a
                                  hash half (ctx option "tail_split_ppm") */
    float ms_resolve;      /* bsim_apply_updates: host time of the batch's op
                              resolution (validation and net changes), before
                              any device work; 0 for the other calls */
    void* priv;
} bsim_result;

/* Operation codes of an update batch (the six change classes of Sec. 3.2
 * arise from these: ADD_V/ADD_E give ADD-SG/ADD-PE, MOD_* give MOD-SG/MOD-PE,
 * DEL_* give DEL-PE/DEL-SG). */
#define BSIM_OP_ADD_V 1u /* new vertex, id = current n_vertices; types given */
#define BSIM_OP_MOD_V 2u /* replace the type set of vertex u */
#define BSIM_OP_DEL_V 3u /* delete vertex u and every edge incident to it */
#define BSIM_OP_ADD_E 4u /* add edge (u, label, w); no-op if the triple exists */
#define BSIM_OP_MOD_E 5u /* relabel one (u, label, w) to (u, new_label, w) */
#define BSIM_OP_DEL_E 6u /* delete every copy of (u, label, w); no-op if absent */

typedef struct {
    uint32_t op;
    uint32_t u;
    uint32_t w;
    uint32_t label;
    uint32_t new_label;
    uint32_t n_types;
    const uint32_t* types; /* host pointer, n_types entries (ADD_V / MOD_V) */
} bsim_update;

/* ---- context ------------------------------------------------------------ */

/* Bind a context to `device` and the HIP stream `hip_stream` (a hipStream_t;
 * NULL = the device's null stream).  The stream stays owned by the caller. */
int bsim_ctx_create(int device, void* hip_stream, bsim_ctx** out);
void bsim_ctx_free(bsim_ctx* ctx);
/* Text of the last error raised on this ctx ("" if none). */
const char* bsim_last_error(const bsim_ctx* ctx);
const char* bsim_status_string(int status);
/* Run-time options (see bsim_option_names()): "chunk_max" = refinement
 * launches queued per stop-flag check (1..4096); "time_launches" = N > 0
 * to bracket every N-th refinement and hub launch (0..1 << 20) with HIP
 * events and report the summed kernel times in bsim_result.ms_iter_kernels /
 * ms_hub_kernels (events on every launch add gaps between launches, so
 * sampling keeps the timed run close to an untimed one); "hub_table_slots" = LDS hash
 * slots of a hub-bucket block (power of two from 64 to the device limit,
 * the default; smaller values force more hash buckets per hub);
 * "frontier_limit_pct" (0..100, default 10) = share of the vertices beyond
 * which an update level is recomputed for all vertices (0: always, the
 * plain form); "frontier_edge_pct" (1..100, default 15) = the same for the
 * share of the out-edges that a level's frontier reads;
 * "tail_split_ppm" (0..1000000, default 100) = when the refinement launches
 * run one per stop check (graphs whose launch takes milliseconds, or
 * chunk_max = 1), a level that founds at most this many classes per
 * million vertices has the next level's split test run as a launch of its
 * own before that level's hashes, so a run that reaches its fixpoint there
 * hashes no further level (0: off);
 * "autotune" (0/1, default 1) = batched calls pick their schedule per size
 * class by timing the candidates on the first call of the class;
 * "batch_small_edges" (N >= 0) = a fixed batched schedule instead: graphs
 * of at most N edges that fit one workgroup go to the small-graph launch
 * (0: none; turns autotune off); "batch_hub_table_slots" (read only) = the
 * hub-table size of the last batched call; "keep_work" (0/1, default 1) =
 * summarize and batched calls keep their device temporaries in one buffer
 * of the largest size an earlier call on the ctx needed, held until
 * bsim_ctx_free (0: every call takes them from the stream-ordered pool and
 * returns them, and setting 0 releases the buffer at once); "fail_alloc_after" (N, 0..2^40)
 * = for tests of the failure paths, the N-th device allocation from now in
 * this process fails as if the device were out of memory (0: off; reading
 * it gives the allocations left).  Values outside the range give
 * BSIM_E_RANGE, unknown names BSIM_E_INVALID. */
int bsim_ctx_set_option(bsim_ctx* ctx, const char* name, int64_t value);
int bsim_ctx_get_option(const bsim_ctx* ctx, const char* name, int64_t* value);
const char* bsim_option_names(void);

/* ---- batch summarization (Algorithm 4 with a fixpoint test) ------------- */

/*
 * Summarize `graph` with `params`.  On success *out holds the result; if
 * state_out is non-NULL the call also returns a resident state (graph copy,
 * per-level hashes, count tables) for bsim_apply_updates; the state then
 * always keeps every level h^0..h^k (BSIM_KEEP_LEVELS is implied) and needs
 * a finite k_max.
 */
int bsim_summarize(bsim_ctx* ctx, const bsim_graph* graph, const bsim_params* params,
                   bsim_state** state_out, bsim_result** out);

/* ---- summarization without device allocation ---------------------------- */

/*
 * For callers that cannot allocate device memory: code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation.  The same
 * batch summarization as bsim_summarize (same kernels, bit-identical
 * results), but it calls no device allocator (no hipMalloc, hipMallocAsync,
 * hipFree, no allocating library routine): every temporary array lives in
 * one static device array of bsim_noalloc_scratch_bytes() bytes (256 MiB)
 * that each device holds for the life of the process, and the results go to
 * arrays the caller owns.
 *   graph   device-resident (mem_kind BSIM_MEM_DEVICE), else BSIM_E_INVALID
 *   params  flags BSIM_STOP_AT_FIXPOINT, BSIM_UNTYPED, BSIM_NO_SUMMARY_EDGES
 *           only (others: BSIM_E_UNSUPPORTED)
 *   out     caller-owned; in: the arrays, out: the scalars
 * Limit: a graph whose temporaries exceed the scratch (about 72 n + 56 m
 * bytes plus two class tables of next_pow2(1.5 n + 1) 8-byte slots and
 * 16 MiB) gives BSIM_E_UNSUPPORTED; the caller's arrays are then untouched.
 * All calls on one device share its scratch, so calls that overlap in time
 * on one device (other host threads or streams) race and must not be made;
 * nothing of a call's scratch carries over to the next.
 */
typedef struct {
    uint64_t* hashes;              /* device [n_vertices]: h^{k_done}, 0 for dead vertices */
    uint32_t* block_ids;           /* device [n_vertices] */
    uint32_t* block_sizes;         /* device [n_vertices]: first n_blocks entries written */
    uint32_t* se_src;              /* device [n_edges] each (first n_summary_edges written), */
    uint32_t* se_label;            /*   or unused with BSIM_NO_SUMMARY_EDGES */
    uint32_t* se_dst;
    uint32_t* blocks_per_iter;     /* host [blocks_per_iter_cap] */
    uint32_t blocks_per_iter_cap;  /* >= min(k_max, n_vertices + 1) + 1 with the fixpoint test,
                                      else >= k_max + 1 */
    uint32_t k_done;               /* outputs, as in bsim_result */
    uint32_t fixpoint;
    uint32_t n_blocks;
    uint64_t n_summary_edges;
    uint64_t scratch_used;         /* bytes of scratch the call used */
} bsim_noalloc_out;

uint64_t bsim_noalloc_scratch_bytes(void);
int bsim_summarize_noalloc(bsim_ctx* ctx, const bsim_graph* graph, const bsim_params* params,
                           bsim_noalloc_out* out);

/*
 * Summarize under the label parameterization (Sec. 2.4): only the edges whose
 * label is in labels[0..n_labels) count, for the signatures and for the
 * summary edges; the others are ignored as if absent.  labels is a host
 * array owned by the caller (read during the call); repeats and labels the
 * graph never uses are allowed, and n_labels = 0 keeps no edge.  Otherwise
 * as bsim_summarize without a state, the direction flags included.  Errors
 * as bsim_summarize; labels == NULL with n_labels > 0 gives BSIM_E_INVALID.
 */
int bsim_summarize_labels(bsim_ctx* ctx, const bsim_graph* graph, const bsim_params* params,
                          const uint32_t* labels, uint32_t n_labels, bsim_result** out);
void bsim_result_free(bsim_result* result);

/*
 * Source-label payload (Sec. 3.3: a payload function may memorize the source
 * label of a vertex; merging vertices into one block joins their source
 * lists).  For result's block ids and source_labels[n_vertices] (one label
 * per vertex, any uint32 value), writes the distinct (block, source label)
 * pairs over the alive vertices, sorted by (block, label), to
 * out_block[] / out_label[] and their number to *n_pairs.  source_labels and
 * the two outputs are host or device pointers as mem_kind says; the outputs
 * must hold result->n_vertices entries (an upper bound).  Caller-owned
 * memory throughout.  BSIM_E_INVALID for a NULL pointer or an unknown
 * mem_kind.
 */
int bsim_source_payload(bsim_ctx* ctx, const bsim_result* result, const uint32_t* source_labels,
                        uint32_t mem_kind, uint32_t* out_block, uint32_t* out_label, uint64_t* n_pairs);

/* Copy one result array to caller memory (host or device pointer, as
 * dst_mem_kind says).  `field` is one of "hashes", "block_ids",
 * "block_sizes", "se_src", "se_label", "se_dst". */
int bsim_result_copy(const bsim_result* result, const char* field, void* dst,
                     uint32_t dst_mem_kind);

/* ---- incremental summarization (Sec. 3.2; Theorem 2) --------------------- */

/*
 * Apply an ordered batch of ADD/MOD/DEL operations to the resident state
 * and return the updated summary.  The batch is all-or-nothing: on error
 * the state is unchanged.  Contract: the result equals bsim_summarize of
 * the updated graph (same vertex ids, alive mask and k) bit for bit --
 * the incremental-equals-batch property of Theorem 2.
 */
int bsim_apply_updates(bsim_state* state, const bsim_update* ops, uint64_t n_ops,
                       bsim_result** out);
/* Current graph of a state as host CSR arrays (for checking); the caller
 * frees each array (row_off, targets, labels, type_off, type_ids, alive)
 * with bsim_host_free.  Rows list surviving old edges first, in their old
 * order, then the edges the batches added. */
int bsim_state_graph(const bsim_state* state, bsim_graph* out_host_graph);
/* The same graph as borrowed device pointers (mem_kind DEVICE), valid until
 * the next bsim_apply_updates or bsim_state_free on this state; it can be
 * passed to bsim_summarize (full recomputation of the updated graph). */
int bsim_state_device_graph(const bsim_state* state, bsim_graph* out_device_graph);
void bsim_host_free(void* p);
void bsim_state_free(bsim_state* state);

/*
 * Checkpoint and resume of a resident state (the incremental run of Sec. 3.2
 * starts from the summary of the previous snapshot; these keep that summary
 * across processes).
 *
 * bsim_state_save writes the state's graph (CSR, labels, type lists, alive
 * mask), its parameters (k_max, flags, label width) and every level
 * h^0..h^K to the host file `path`: first to `path`.tmp, renamed over
 * `path` once complete.  The file is in host byte order with a 64-byte
 * header and a checksum over the arrays.  It takes about
 * 8(n+1) + m(4 + label_bytes) + 4 nt + n + 8 n (k_max+1) bytes.  Errors:
 * BSIM_E_INVALID for null arguments, BSIM_E_IO when the file cannot be
 * written (no partial file is left under `path`).
 *
 * bsim_state_load reads such a file into a new state owned by ctx and
 * returns that state's summary in *out (every array of the result of the
 * state's last summarize or update call).  The graph passes the checks of
 * bsim_summarize; the levels are uploaded, not recomputed, and the classes
 * are formed from them.  Later bsim_apply_updates calls on the loaded state
 * return what they would return on the state that was saved.  Errors:
 * BSIM_E_IO (cannot open or read), BSIM_E_INVALID (not a state file, a size
 * or checksum that does not match, a hash on a deleted vertex, a malformed
 * graph), BSIM_E_UNSUPPORTED (another format version), BSIM_E_NOMEM; on
 * error *state_out and *out are null.
 */
int bsim_state_save(const bsim_state* state, const char* path);
int bsim_state_load(bsim_ctx* ctx, const char* path, bsim_state** state_out, bsim_result** out);

/*
 * Change detection from two snapshots without a change log (Sec. 3.2's
 * change classes between the graph at time t and at t+1).  The snapshots
 * share vertex ids: after has at least before's n_vertices, and the ids past
 * them are new vertices.  *ops receives the ordered batch that turns before
 * into after under bsim_apply_updates' semantics (equal alive masks, type
 * sets and sets of edge triples), *n_ops its length:
 *   ADD_V  each new id in ascending order, with after's type list;
 *   MOD_V  each vertex alive in both whose type set changed (after's list);
 *   DEL_E  each distinct triple of before that after lacks, both endpoints
 *          alive in after, in order of its first copy in before;
 *   ADD_E  each distinct triple of after that before lacks, in order of its
 *          first copy in after;
 *   DEL_V  each vertex alive in before (or new) and dead in after.
 * Edges of a vertex that dies go with its DEL_V.  The batch is host memory
 * the library allocates (the type lists live in the same block); free it
 * with bsim_updates_free.  Inputs are host or device graphs (mem_kind).
 * BSIM_E_INVALID: a malformed snapshot, fewer ids after, or a vertex dead
 * before and alive after (ids are never reused).
 */
int bsim_diff_snapshots(bsim_ctx* ctx, const bsim_graph* before, const bsim_graph* after, bsim_update** ops,
                        uint64_t* n_ops);
void bsim_updates_free(bsim_update* ops);

/* ---- measurement probes (the refinement's roofline) ---------------------- */

/*
 * bsim_probe_gather: *ms_per_pass = device time of one pass that streams
 * targets[0..m) once and gathers one 8-byte value h[targets[e]] per edge
 * (targets >= n are skipped), averaged over `reps` passes after one warm-up
 * pass; the memory pattern that bounds a refinement iteration, without its
 * labels, de-duplication or classes.  targets and h are device arrays the
 * caller owns; the pass gathers from a copy of h in the ctx's work memory
 * (option keep_work), where the refinement keeps its hash arrays, and the
 * call allocates a small sink there.  bsim_probe_copy: the same
 * for a STREAM-style copy of `bytes` bytes between two arrays the call
 * allocates (read + write).  BSIM_E_INVALID for null pointers or reps = 0.
 */
int bsim_probe_gather(bsim_ctx* ctx, const uint32_t* targets, uint64_t m, const uint64_t* h, uint32_t n,
                      uint32_t reps, float* ms_per_pass);
int bsim_probe_copy(bsim_ctx* ctx, uint64_t bytes, uint32_t reps, float* ms_per_pass);

/* ---- batched summarization (many independent graphs, one launch stream) -- */

/*
 * Summarize n_graphs independent graphs; outs[i] receives graph i's result,
 * identical to a bsim_summarize call on that graph alone.
 */
int bsim_batch_summarize(bsim_ctx* ctx, const bsim_graph* graphs, uint32_t n_graphs,
                         const bsim_params* params, bsim_result** outs);

/* ---- serving: continuous batching of summarize and update requests ------ */

/*
 * A server runs requests on a pool of worker threads, each with its own
 * context and HIP stream, so the kernels of concurrent requests overlap on
 * the device.  Admission is by memory footprint: a request starts once its
 * estimated device footprint fits the budget that running requests and
 * server-owned states leave free; until then it waits (requests start in
 * submission order among those that fit).  Updates of one state run one at
 * a time in submission order.  Every result equals what the same call made
 * alone would return.
 */
typedef struct bsim_server bsim_server;

#define BSIM_REQ_SUMMARIZE 1u /* summarize `graph` (optionally keeping a state) */
#define BSIM_REQ_UPDATE 2u    /* apply `ops` to `state` */

typedef struct {
    uint32_t kind;
    uint32_t keep_state;      /* SUMMARIZE: also create a server-owned state */
    const bsim_graph* graph;  /* SUMMARIZE: host arrays are copied at submit;
                                 device arrays are borrowed until completion */
    bsim_params params;       /* SUMMARIZE */
    bsim_state* state;        /* UPDATE: a state from this server (keep_state) or
                                 one the caller does not touch meanwhile */
    const bsim_update* ops;   /* UPDATE: copied at submit (with their type lists) */
    uint64_t n_ops;
} bsim_request;

typedef struct {
    uint64_t submitted, completed, failed;
    uint64_t bytes_in_use, bytes_budget;
    double p50_ms[3], p99_ms[3]; /* index 0 all, 1 summarize, 2 update: submit-to-done */
    double busy_ms;              /* wall time from first submit to last completion */
} bsim_server_stats;

/* n_workers concurrent requests (1..64); mem_budget_bytes 0 = 90 % of the
 * device memory free at creation. */
int bsim_server_create(int device, uint64_t mem_budget_bytes, uint32_t n_workers, bsim_server** out);
/* Queue a request.  BSIM_E_BUSY: its footprint exceeds what the server-owned
 * states leave of the budget (a queued request that comes to exceed it,
 * because a keep_state request created a state meanwhile, fails with
 * BSIM_E_BUSY instead of waiting for good); BSIM_E_INVALID / BSIM_E_RANGE:
 * malformed request, or a server being freed (nothing queued). */
int bsim_server_submit(bsim_server* srv, const bsim_request* req, uint64_t* ticket);
/* Result of a request: BSIM_OK with *out (and *state_out for keep_state)
 * once done, the request's own error status if it failed, BSIM_E_BUSY if it
 * is not done and wait == 0.  Each ticket is collected once: polling a
 * ticket again, or one never issued, gives BSIM_E_INVALID at once. */
int bsim_server_poll(bsim_server* srv, uint64_t ticket, int wait, bsim_result** out, bsim_state** state_out);
int bsim_server_stats_get(bsim_server* srv, bsim_server_stats* out);
/* Set a context option (bsim_ctx_set_option's names and ranges) on every
 * context of the server: the workers', the server-owned states' and those
 * created later.  Only while no request is queued or running
 * (BSIM_E_BUSY otherwise); errors as bsim_ctx_set_option.  "keep_work" is
 * off on a server's contexts (its memory budget counts a request's
 * temporaries while the request runs) and gives BSIM_E_UNSUPPORTED. */
int bsim_server_set_option(bsim_server* srv, const char* name, int64_t value);
/* Free a server-owned state and return its memory to the budget. */
int bsim_server_release_state(bsim_server* srv, bsim_state* state);
/* Cancels the requests that have not started, waits for the running ones,
 * then frees everything the server owns (uncollected results included). */
void bsim_server_free(bsim_server* srv);

#ifdef __cplusplus
}
#endif

#endif /* BSIM_H */
