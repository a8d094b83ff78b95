/*
 * bsim_oracle.c -- CPU reference ("oracle") for hash-based labeled forward
 * k-bisimulation.  TEST INFRASTRUCTURE ONLY: the tests, the smoke check and
 * the benchmark's CPU-baseline leg may call it; the GPU library never does,
 * and this file shares no code, header or table with it.
 *
 * Plain, single-threaded, slow on purpose: every step is written the way the
 * method states it, with qsort/unique as the only library-like steps.
 *
 * What it computes (paper Sec. 2.5, forward bisimulation with the variant
 * that requires equal vertex labels at k = 0; Sec. 2.4 chaining
 * parameterization; Sec. 3.3, Algorithm 4, hash messages in place of nested
 * vertex summaries):
 *
 *   h^0(v) = t(v)                      hash of the type set of v
 *   h^k(v) = F(t(v), SET{ (l, h^{k-1}(w)) : (v, l, w) in E })   for k >= 1
 *
 * Two vertices are in the same block of the k-partition iff their h^k agree.
 * The paper fixes no hash function; it only asks that equal content gives
 * equal identifiers and that the set hash ignores order (Sec. 3.3).  The
 * concrete 64-bit spec followed here (and, independently, by the GPU path):
 *
 *   M(z)     = SplitMix64 output function (Steele, Lea & Flood, OOPSLA 2014):
 *              z ^= z >> 30; z *= 0xBF58476D1CE4E5B9;
 *              z ^= z >> 27; z *= 0x94D049BB133111EB; z ^= z >> 31
 *   C_T, C_L, C_S, C_E = M(1), M(2), M(3), M(4)
 *   t(v)     = M(C_T + sum over the distinct types tau of v of M(C_T ^ tau))
 *              (UNTYPED flag: t(v) = M(C_T) for every v)
 *   salt(l)  = M(C_L + l)
 *   key(e)   = h^{k-1}(w) ^ salt(l)                       for e = (v, l, w)
 *   h^k(v)   = M(t(v) ^ M(C_S + sum over the distinct keys q of v of M(q ^ C_E)))
 *
 * All arithmetic is unsigned and wraps mod 2^64.
 *
 * Classes.  The bisimulation definition (Sec. 2.5) makes u, v k-bisimilar
 * iff they are (k-1)-bisimilar AND their labeled successor sets match; the
 * hash decides the second condition.  So the k-class of v is the pair
 * (its (k-1)-class, h^k(v)), with the 0-class given by h^0 = t(v).  Without
 * a 64-bit collision this is exactly "equal h^k"; with one, classes that
 * were already apart stay apart.  n_k is the number of k-classes over alive
 * vertices.
 *
 * Relabelling (Algorithm 4's final FindAndMerge): blocks are numbered by
 * first occurrence -- the block holding the smallest vertex id is block 0,
 * and so on -- which depends only on the partition.  The loop stops at the
 * first k >= 1 with n_k == n_{k-1} (the partition stopped changing; it is
 * then the maximal bisimulation refining the type partition) or at k_max.
 *
 * The summary graph's edges are the distinct triples (block(v), l, block(w))
 * over all edges, i.e. the quotient of the graph by the final partition
 * (Sec. 2.6, edges between vertex summaries), sorted by (src, label, dst).
 *
 * With BO_PREV_LEVEL_EDGES the edges are instead those of the vertex
 * summaries' top layer in Sec. 2.6's inductive definition: for a CSE whose
 * object relation is the (k-1)-bisimulation, the primary vertex of v (its
 * k_done-class) has an l-edge to the primary vertex of each neighbour's
 * (k_done-1)-class.  So the triples are (block(v), l, prev_block(w)), where
 * prev_block numbers the (k_done-1)-classes by first occurrence; at
 * k_done = 0 the 0-classes stand in for both ends.  At a fixpoint the two
 * partitions agree and so do the two edge sets.
 *
 * Dead vertices (alive[v] == 0, deletions of Algorithm 3) have hash 0, block
 * 0xFFFFFFFF and are not counted; an edge touching a dead vertex is an error.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define BO_STOP_AT_FIXPOINT 1u
#define BO_UNTYPED 4u
#define BO_PREV_LEVEL_EDGES 128u

#define BO_OK 0
#define BO_E_INVALID (-1)
#define BO_E_NOMEM (-3)

uint64_t bo_mix(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

uint64_t bo_const_t(void) { return bo_mix(1); }
uint64_t bo_const_l(void) { return bo_mix(2); }
uint64_t bo_const_s(void) { return bo_mix(3); }
uint64_t bo_const_e(void) { return bo_mix(4); }

static int cmp_u64(const void* a, const void* b) {
    uint64_t x = *(const uint64_t*)a, y = *(const uint64_t*)b;
    return (x > y) - (x < y);
}

static int cmp_u32(const void* a, const void* b) {
    uint32_t x = *(const uint32_t*)a, y = *(const uint32_t*)b;
    return (x > y) - (x < y);
}

/* Sort and drop repeats; returns the number of distinct values kept. */
static size_t unique_u64(uint64_t* a, size_t n) {
    if (n == 0) return 0;
    qsort(a, n, sizeof(uint64_t), cmp_u64);
    size_t k = 1;
    for (size_t i = 1; i < n; i++)
        if (a[i] != a[k - 1]) a[k++] = a[i];
    return k;
}

static size_t unique_u32(uint32_t* a, size_t n) {
    if (n == 0) return 0;
    qsort(a, n, sizeof(uint32_t), cmp_u32);
    size_t k = 1;
    for (size_t i = 1; i < n; i++)
        if (a[i] != a[k - 1]) a[k++] = a[i];
    return k;
}

/* t(v): hash of the *set* of type ids (the k = 0 vertex-label condition). */
uint64_t bo_type_hash(const uint32_t* types, uint32_t n_types, uint32_t untyped) {
    const uint64_t ct = bo_const_t();
    if (untyped || n_types == 0) return bo_mix(ct);
    uint32_t* tmp = (uint32_t*)malloc(sizeof(uint32_t) * n_types);
    if (!tmp) abort();
    memcpy(tmp, types, sizeof(uint32_t) * n_types);
    size_t u = unique_u32(tmp, n_types);
    uint64_t sum = 0;
    for (size_t i = 0; i < u; i++) sum += bo_mix(ct ^ (uint64_t)tmp[i]);
    free(tmp);
    return bo_mix(ct + sum);
}

uint64_t bo_label_salt(uint32_t label) { return bo_mix(bo_const_l() + (uint64_t)label); }

/* One refinement step for one vertex, given its out-edges and h^{k-1}.
 * `keys` is scratch space for at least `deg` values. */
static uint64_t vertex_step(uint64_t t_v, const uint32_t* tgt, const uint32_t* lab,
                            uint64_t deg, const uint64_t* h_prev, uint64_t* keys) {
    const uint64_t cs = bo_const_s(), ce = bo_const_e();
    for (uint64_t i = 0; i < deg; i++) keys[i] = h_prev[tgt[i]] ^ bo_label_salt(lab[i]);
    size_t u = unique_u64(keys, (size_t)deg);
    uint64_t sum = 0;
    for (size_t i = 0; i < u; i++) sum += bo_mix(keys[i] ^ ce);
    return bo_mix(t_v ^ bo_mix(cs + sum));
}

uint64_t bo_vertex_step(uint64_t t_v, const uint32_t* tgt, const uint32_t* lab,
                        uint64_t deg, const uint64_t* h_prev) {
    uint64_t* keys = (uint64_t*)malloc(sizeof(uint64_t) * (deg ? deg : 1));
    if (!keys) abort();
    uint64_t r = vertex_step(t_v, tgt, lab, deg, h_prev, keys);
    free(keys);
    return r;
}

static uint64_t max_degree(uint32_t n, const uint64_t* row_off) {
    uint64_t d = 1;
    for (uint32_t v = 0; v < n; v++)
        if (row_off[v + 1] - row_off[v] > d) d = row_off[v + 1] - row_off[v];
    return d;
}

typedef struct { uint32_t c; uint64_t h; uint32_t v; } chv_triple;

static int cmp_chv(const void* a, const void* b) {
    const chv_triple* x = (const chv_triple*)a;
    const chv_triple* y = (const chv_triple*)b;
    if (x->c != y->c) return (x->c > y->c) - (x->c < y->c);
    if (x->h != y->h) return (x->h > y->h) - (x->h < y->h);
    return (x->v > y->v) - (x->v < y->v);
}

/* Refine: the new class of an alive vertex is the pair (cls[v], h[v]).
 * Classes are renumbered by first occurrence (the class of the smallest
 * vertex is 0).  Dead vertices get 0xFFFFFFFF.  Returns the class count. */
static uint32_t refine_classes(const uint32_t* cls, const uint64_t* h, const uint8_t* alive,
                               uint32_t n, uint32_t* out) {
    chv_triple* p = (chv_triple*)malloc(sizeof(chv_triple) * (n ? n : 1));
    uint32_t* minv = (uint32_t*)malloc(sizeof(uint32_t) * (n ? n : 1));
    uint32_t* rank = (uint32_t*)malloc(sizeof(uint32_t) * (n ? n : 1));
    uint8_t* is_min = (uint8_t*)calloc(n ? n : 1, 1);
    if (!p || !minv || !rank || !is_min) abort();
    size_t k = 0;
    for (uint32_t v = 0; v < n; v++)
        if (!alive || alive[v]) { p[k].c = cls ? cls[v] : 0; p[k].h = h[v]; p[k].v = v; k++; }
    qsort(p, k, sizeof(chv_triple), cmp_chv);
    /* smallest vertex of each (class, hash) group */
    for (size_t i = 0; i < k; i++) {
        int same = i > 0 && p[i].c == p[i - 1].c && p[i].h == p[i - 1].h;
        uint32_t m = same ? minv[p[i - 1].v] : p[i].v;
        minv[p[i].v] = m;
        if (m == p[i].v) is_min[p[i].v] = 1;
    }
    /* groups numbered in order of their smallest vertex */
    uint32_t nb = 0;
    for (uint32_t v = 0; v < n; v++)
        if (is_min[v]) rank[v] = nb++;
    for (uint32_t v = 0; v < n; v++)
        out[v] = (!alive || alive[v]) ? rank[minv[v]] : 0xFFFFFFFFu;
    free(p); free(minv); free(rank); free(is_min);
    return nb;
}

typedef struct { uint32_t s, l, d; } triple;

static int cmp_triple(const void* a, const void* b) {
    const triple* x = (const triple*)a;
    const triple* y = (const triple*)b;
    if (x->s != y->s) return (x->s > y->s) - (x->s < y->s);
    if (x->l != y->l) return (x->l > y->l) - (x->l < y->l);
    return (x->d > y->d) - (x->d < y->d);
}

/* One refinement step on given classes and hashes (exported for tests). */
uint32_t bo_refine_classes(const uint32_t* cls, const uint64_t* h, const uint8_t* alive, uint32_t n,
                           uint32_t* out) {
    return refine_classes(cls, h, alive, n, out);
}

/* First-occurrence block ids of the partition induced by equal values of h
 * over alive vertices.  Returns the number of blocks. */
uint32_t bo_block_ids(const uint64_t* h, const uint8_t* alive, uint32_t n, uint32_t* block) {
    return refine_classes(NULL, h, alive, n, block);
}

/*
 * Full batch summarization.  Inputs are host CSR arrays.  Outputs are
 * caller-allocated:
 *   hashes[n]            h^{k_done}
 *   prev_hashes[n]       h^{k_done-1} (nullable; equals hashes if k_done == 0)
 *   block_ids[n]         first-occurrence block of v in the k_done-partition
 *   blocks_per_iter[k_max+1]   n_0 .. n_{k_done}
 *   block_sizes[n]       vertices per block (first n_blocks entries used)
 *   se_src/se_lab/se_dst[m]    sorted distinct quotient edges
 * Returns BO_OK or BO_E_INVALID (bad CSR, or an edge touching a dead vertex).
 */
int bo_summarize(uint32_t n, uint64_t m, const uint64_t* row_off, const uint32_t* tgt,
                 const uint32_t* lab, const uint64_t* typ_off, const uint32_t* typ,
                 const uint8_t* alive, uint32_t k_max, uint32_t flags,
                 uint64_t* hashes, uint64_t* prev_hashes, uint32_t* block_ids,
                 uint32_t* blocks_per_iter, uint32_t* k_done_out, uint32_t* fixpoint_out,
                 uint32_t* n_blocks_out, uint32_t* block_sizes, uint64_t* n_se_out,
                 uint32_t* se_src, uint32_t* se_lab, uint32_t* se_dst) {
    if (row_off[0] != 0 || row_off[n] != m) return BO_E_INVALID;
    for (uint32_t v = 0; v < n; v++) {
        if (row_off[v + 1] < row_off[v] || typ_off[v + 1] < typ_off[v]) return BO_E_INVALID;
        for (uint64_t e = row_off[v]; e < row_off[v + 1]; e++) {
            if (tgt[e] >= n) return BO_E_INVALID;
            if (alive && (!alive[v] || !alive[tgt[e]])) return BO_E_INVALID;
        }
    }
    uint64_t* t = (uint64_t*)malloc(sizeof(uint64_t) * (n ? n : 1));
    uint64_t* cur = (uint64_t*)malloc(sizeof(uint64_t) * (n ? n : 1));
    uint64_t* nxt = (uint64_t*)malloc(sizeof(uint64_t) * (n ? n : 1));
    uint32_t* cls = (uint32_t*)malloc(sizeof(uint32_t) * (n ? n : 1));
    uint32_t* ncls = (uint32_t*)malloc(sizeof(uint32_t) * (n ? n : 1));
    uint64_t* keys = (uint64_t*)malloc(sizeof(uint64_t) * max_degree(n, row_off));
    if (!t || !cur || !nxt || !cls || !ncls || !keys) return BO_E_NOMEM;

    /* k = 0: types only */
    for (uint32_t v = 0; v < n; v++) {
        int a = !alive || alive[v];
        t[v] = a ? bo_type_hash(typ + typ_off[v], (uint32_t)(typ_off[v + 1] - typ_off[v]),
                                flags & BO_UNTYPED)
                 : 0;
        cur[v] = t[v];
    }
    memcpy(nxt, cur, sizeof(uint64_t) * n);
    blocks_per_iter[0] = refine_classes(NULL, cur, alive, n, cls);
    uint32_t k_done = 0, fixpoint = 0;

    for (uint32_t k = 1; k <= k_max; k++) {
        for (uint32_t v = 0; v < n; v++) {
            if (alive && !alive[v]) { nxt[v] = 0; continue; }
            nxt[v] = vertex_step(t[v], tgt + row_off[v], lab + row_off[v],
                                 row_off[v + 1] - row_off[v], cur, keys);
        }
        blocks_per_iter[k] = refine_classes(cls, nxt, alive, n, ncls);
        uint32_t* cs = cls; cls = ncls; ncls = cs;  /* cls = k-classes */
        uint64_t* sw = cur; cur = nxt; nxt = sw;   /* cur = h^k, nxt = h^{k-1} */
        k_done = k;
        if (blocks_per_iter[k] == blocks_per_iter[k - 1]) {
            fixpoint = 1;
            if (flags & BO_STOP_AT_FIXPOINT) break;
        } else {
            fixpoint = 0;
        }
    }
    memcpy(hashes, cur, sizeof(uint64_t) * n);
    if (prev_hashes) memcpy(prev_hashes, nxt, sizeof(uint64_t) * n);

    /* the k_done-classes, numbered by first occurrence, are the blocks */
    uint32_t nb = blocks_per_iter[k_done];
    memcpy(block_ids, cls, sizeof(uint32_t) * n);
    memset(block_sizes, 0, sizeof(uint32_t) * (nb ? nb : 0));
    for (uint32_t v = 0; v < n; v++)
        if (block_ids[v] != 0xFFFFFFFFu) block_sizes[block_ids[v]]++;

    /* after the loop ncls holds the (k_done-1)-classes when k_done >= 1 */
    const uint32_t* dst_ids = ((flags & BO_PREV_LEVEL_EDGES) && k_done >= 1) ? ncls : block_ids;
    triple* tr = (triple*)malloc(sizeof(triple) * (m ? m : 1));
    if (!tr) return BO_E_NOMEM;
    uint64_t ne = 0;
    for (uint32_t v = 0; v < n; v++)
        for (uint64_t e = row_off[v]; e < row_off[v + 1]; e++) {
            tr[ne].s = block_ids[v];
            tr[ne].l = lab[e];
            tr[ne].d = dst_ids[tgt[e]];
            ne++;
        }
    qsort(tr, (size_t)ne, sizeof(triple), cmp_triple);
    uint64_t u = 0;
    for (uint64_t i = 0; i < ne; i++) {
        if (u > 0 && tr[i].s == se_src[u - 1] && tr[i].l == se_lab[u - 1] &&
            tr[i].d == se_dst[u - 1])
            continue;
        se_src[u] = tr[i].s; se_lab[u] = tr[i].l; se_dst[u] = tr[i].d;
        u++;
    }
    *n_se_out = u;
    *k_done_out = k_done;
    *fixpoint_out = fixpoint;
    *n_blocks_out = nb;
    free(tr); free(t); free(cur); free(nxt); free(cls); free(ncls); free(keys);
    return BO_OK;
}

/*
 * Run exactly `iters` refinement steps (no fixpoint test) and return h^iters.
 * Used to time a bounded prefix of a large workload.
 */
int bo_iterate(uint32_t n, const uint64_t* row_off, const uint32_t* tgt, const uint32_t* lab,
               const uint64_t* typ_off, const uint32_t* typ, uint32_t iters, uint32_t flags,
               uint64_t* out_hashes, uint32_t* counts) {
    uint64_t* t = (uint64_t*)malloc(sizeof(uint64_t) * (n ? n : 1));
    uint64_t* cur = (uint64_t*)malloc(sizeof(uint64_t) * (n ? n : 1));
    uint64_t* nxt = (uint64_t*)malloc(sizeof(uint64_t) * (n ? n : 1));
    uint32_t* cls = (uint32_t*)malloc(sizeof(uint32_t) * (n ? n : 1));
    uint32_t* ncls = (uint32_t*)malloc(sizeof(uint32_t) * (n ? n : 1));
    uint64_t* keys = (uint64_t*)malloc(sizeof(uint64_t) * max_degree(n, row_off));
    if (!t || !cur || !nxt || !cls || !ncls || !keys) return BO_E_NOMEM;
    for (uint32_t v = 0; v < n; v++) {
        t[v] = bo_type_hash(typ + typ_off[v], (uint32_t)(typ_off[v + 1] - typ_off[v]),
                            flags & BO_UNTYPED);
        cur[v] = t[v];
    }
    uint32_t c0 = refine_classes(NULL, cur, NULL, n, cls);
    if (counts) counts[0] = c0;
    for (uint32_t k = 1; k <= iters; k++) {
        for (uint32_t v = 0; v < n; v++)
            nxt[v] = vertex_step(t[v], tgt + row_off[v], lab + row_off[v],
                                 row_off[v + 1] - row_off[v], cur, keys);
        uint32_t ck = refine_classes(cls, nxt, NULL, n, ncls);
        if (counts) counts[k] = ck;
        uint32_t* cs = cls; cls = ncls; ncls = cs;
        uint64_t* sw = cur; cur = nxt; nxt = sw;
    }
    memcpy(out_hashes, cur, sizeof(uint64_t) * n);
    free(t); free(cur); free(nxt); free(cls); free(ncls); free(keys);
    return BO_OK;
}

/*
 * Timing samples of one refinement step (the benchmark's CPU baseline on a
 * graph too large to run whole): t(v) for every vertex, then the step of
 * bo_summarize for every stride-th vertex from v0 (out[i] = h^k of vertex
 * v0 + i * stride, given h_prev = h^{k-1}), and the class refinement of
 * those vertices with bo_refine_classes.  The same per-vertex code as the
 * full runs; nothing is reordered.
 */
void bo_type_hashes(uint32_t n, const uint64_t* typ_off, const uint32_t* typ, uint32_t flags, uint64_t* t) {
    for (uint32_t v = 0; v < n; v++)
        t[v] = bo_type_hash(typ + typ_off[v], (uint32_t)(typ_off[v + 1] - typ_off[v]), flags & BO_UNTYPED);
}

int bo_step_strided(uint32_t n, const uint64_t* row_off, const uint32_t* tgt, const uint32_t* lab,
                    const uint64_t* t, const uint64_t* h_prev, uint32_t v0, uint32_t stride, uint32_t count,
                    uint64_t* out) {
    if (stride == 0 || (count && (uint64_t)v0 + (uint64_t)(count - 1) * stride >= n)) return BO_E_INVALID;
    uint64_t maxd = 1;
    for (uint32_t i = 0; i < count; i++) {
        const uint32_t v = v0 + i * stride;
        if (row_off[v + 1] - row_off[v] > maxd) maxd = row_off[v + 1] - row_off[v];
    }
    uint64_t* keys = (uint64_t*)malloc(sizeof(uint64_t) * maxd);
    if (!keys) return BO_E_NOMEM;
    for (uint32_t i = 0; i < count; i++) {
        const uint32_t v = v0 + i * stride;
        out[i] = vertex_step(t[v], tgt + row_off[v], lab + row_off[v], row_off[v + 1] - row_off[v], h_prev, keys);
    }
    free(keys);
    return BO_OK;
}

/*
 * Direction and label parameterizations (Sec. 2.4: the label
 * parameterization keeps only the edges whose label is in a set P_l; the
 * direction parameterization takes outgoing edges, incoming edges or both;
 * Sec. 2.5: backward bisimulation is forward bisimulation with incoming
 * edges).  TEST INFRASTRUCTURE ONLY, like everything in this file.
 *
 *   kept edges   E' = { (v, l, w) in E : P_l absent or l in P_l }
 *   forward      the (partner, salt) pairs of v are (w, salt(l))    for (v, l, w) in E'
 *   backward     the pairs of w are (v, salt(l))                    for (v, l, w) in E'
 *   both         the forward pairs of v and the backward pairs of v, the
 *                backward ones salted by salt_in(l) = M(C_L + 2^31 + l): an
 *                incoming l-edge counts as an outgoing edge whose label is
 *                l + 2^31, a range no input label reaches (labels < 2^24),
 *                so incoming and outgoing edges never make the same pair
 *   key          h^{k-1}(partner) ^ salt
 *   h^k(v)       M(t(v) ^ M(C_S + sum over the distinct keys q of v of M(q ^ C_E)))
 *
 * The refinement, the stop rule and the block numbering are those of
 * bo_summarize; the summary edges are the distinct (block(v), l, block(w))
 * over the kept edges E', in their own direction.  With forward, no P_l the
 * result equals bo_summarize.
 */
#define BO_BACKWARD 32u
#define BO_BOTH_DIRECTIONS 64u

uint64_t bo_label_salt_in(uint32_t label) { return bo_mix(bo_const_l() + 0x80000000ull + (uint64_t)label); }

/* keep_label[l] != 0 for l in P_l, for l < n_keep; NULL keeps every edge */
static int kept(const uint8_t* keep_label, uint32_t n_keep, uint32_t l) {
    return !keep_label || (l < n_keep && keep_label[l]);
}

int bo_summarize_ext(uint32_t n, uint64_t m, const uint64_t* row_off, const uint32_t* tgt,
                     const uint32_t* lab, const uint64_t* typ_off, const uint32_t* typ,
                     const uint8_t* alive, uint32_t k_max, uint32_t flags,
                     const uint8_t* keep_label, uint32_t n_keep,
                     uint64_t* hashes, uint32_t* block_ids, uint32_t* blocks_per_iter,
                     uint32_t* k_done_out, uint32_t* fixpoint_out, uint32_t* n_blocks_out,
                     uint32_t* block_sizes, uint64_t* n_se_out,
                     uint32_t* se_src, uint32_t* se_lab, uint32_t* se_dst) {
    if ((flags & BO_BACKWARD) && (flags & BO_BOTH_DIRECTIONS)) return BO_E_INVALID;
    /* previous-level edges are defined for the forward direction only */
    if ((flags & BO_PREV_LEVEL_EDGES) && (flags & (BO_BACKWARD | BO_BOTH_DIRECTIONS))) return BO_E_INVALID;
    if (row_off[0] != 0 || row_off[n] != m) return BO_E_INVALID;
    for (uint32_t v = 0; v < n; v++) {
        if (row_off[v + 1] < row_off[v] || typ_off[v + 1] < typ_off[v]) return BO_E_INVALID;
        for (uint64_t e = row_off[v]; e < row_off[v + 1]; e++) {
            if (tgt[e] >= n) return BO_E_INVALID;
            if (alive && (!alive[v] || !alive[tgt[e]])) return BO_E_INVALID;
        }
    }
    const int fwd = !(flags & BO_BACKWARD);
    const int bwd = (flags & BO_BACKWARD) || (flags & BO_BOTH_DIRECTIONS);
    /* pair lists: pcount[v] pairs of v at pair_off[v] */
    uint64_t* pair_off = (uint64_t*)calloc((size_t)n + 1, sizeof(uint64_t));
    if (!pair_off) return BO_E_NOMEM;
    for (uint32_t v = 0; v < n; v++)
        for (uint64_t e = row_off[v]; e < row_off[v + 1]; e++) {
            if (!kept(keep_label, n_keep, lab[e])) continue;
            if (fwd) pair_off[v + 1]++;
            if (bwd) pair_off[tgt[e] + 1]++;
        }
    for (uint32_t v = 0; v < n; v++) pair_off[v + 1] += pair_off[v];
    const uint64_t np = pair_off[n];
    uint32_t* partner = (uint32_t*)malloc(sizeof(uint32_t) * (np ? np : 1));
    uint64_t* salt = (uint64_t*)malloc(sizeof(uint64_t) * (np ? np : 1));
    uint64_t* fill = (uint64_t*)malloc(sizeof(uint64_t) * ((size_t)n + 1));
    if (!partner || !salt || !fill) return BO_E_NOMEM;
    memcpy(fill, pair_off, sizeof(uint64_t) * ((size_t)n + 1));
    for (uint32_t v = 0; v < n; v++)
        for (uint64_t e = row_off[v]; e < row_off[v + 1]; e++) {
            if (!kept(keep_label, n_keep, lab[e])) continue;
            const uint32_t w = tgt[e];
            if (fwd) {
                partner[fill[v]] = w;
                salt[fill[v]++] = bo_label_salt(lab[e]);
            }
            if (bwd) {
                partner[fill[w]] = v;
                salt[fill[w]++] = (flags & BO_BOTH_DIRECTIONS) ? bo_label_salt_in(lab[e]) : bo_label_salt(lab[e]);
            }
        }
    uint64_t maxp = 1;
    for (uint32_t v = 0; v < n; v++)
        if (pair_off[v + 1] - pair_off[v] > maxp) maxp = pair_off[v + 1] - pair_off[v];
    uint64_t* t = (uint64_t*)malloc(sizeof(uint64_t) * (n ? n : 1));
    uint64_t* cur = (uint64_t*)malloc(sizeof(uint64_t) * (n ? n : 1));
    uint64_t* nxt = (uint64_t*)malloc(sizeof(uint64_t) * (n ? n : 1));
    uint32_t* cls = (uint32_t*)malloc(sizeof(uint32_t) * (n ? n : 1));
    uint32_t* ncls = (uint32_t*)malloc(sizeof(uint32_t) * (n ? n : 1));
    uint64_t* keys = (uint64_t*)malloc(sizeof(uint64_t) * maxp);
    if (!t || !cur || !nxt || !cls || !ncls || !keys) return BO_E_NOMEM;
    const uint64_t cs = bo_const_s(), ce = bo_const_e();

    for (uint32_t v = 0; v < n; v++) {
        int a = !alive || alive[v];
        t[v] = a ? bo_type_hash(typ + typ_off[v], (uint32_t)(typ_off[v + 1] - typ_off[v]),
                                flags & BO_UNTYPED)
                 : 0;
        cur[v] = t[v];
    }
    blocks_per_iter[0] = refine_classes(NULL, cur, alive, n, cls);
    uint32_t k_done = 0, fixpoint = 0;
    for (uint32_t k = 1; k <= k_max; k++) {
        for (uint32_t v = 0; v < n; v++) {
            if (alive && !alive[v]) { nxt[v] = 0; continue; }
            const uint64_t d = pair_off[v + 1] - pair_off[v];
            for (uint64_t i = 0; i < d; i++) keys[i] = cur[partner[pair_off[v] + i]] ^ salt[pair_off[v] + i];
            size_t u = unique_u64(keys, (size_t)d);
            uint64_t sum = 0;
            for (size_t i = 0; i < u; i++) sum += bo_mix(keys[i] ^ ce);
            nxt[v] = bo_mix(t[v] ^ bo_mix(cs + sum));
        }
        blocks_per_iter[k] = refine_classes(cls, nxt, alive, n, ncls);
        uint32_t* sc = cls; cls = ncls; ncls = sc;
        uint64_t* sw = cur; cur = nxt; nxt = sw;
        k_done = k;
        if (blocks_per_iter[k] == blocks_per_iter[k - 1]) {
            fixpoint = 1;
            if (flags & BO_STOP_AT_FIXPOINT) break;
        } else {
            fixpoint = 0;
        }
    }
    memcpy(hashes, cur, sizeof(uint64_t) * n);
    uint32_t nb = blocks_per_iter[k_done];
    memcpy(block_ids, cls, sizeof(uint32_t) * n);
    memset(block_sizes, 0, sizeof(uint32_t) * (nb ? nb : 0));
    for (uint32_t v = 0; v < n; v++)
        if (block_ids[v] != 0xFFFFFFFFu) block_sizes[block_ids[v]]++;

    const uint32_t* dst_ids = ((flags & BO_PREV_LEVEL_EDGES) && k_done >= 1) ? ncls : block_ids;
    triple* tr = (triple*)malloc(sizeof(triple) * (m ? m : 1));
    if (!tr) return BO_E_NOMEM;
    uint64_t ne = 0;
    for (uint32_t v = 0; v < n; v++)
        for (uint64_t e = row_off[v]; e < row_off[v + 1]; e++) {
            if (!kept(keep_label, n_keep, lab[e])) continue;
            tr[ne].s = block_ids[v];
            tr[ne].l = lab[e];
            tr[ne].d = dst_ids[tgt[e]];
            ne++;
        }
    qsort(tr, (size_t)ne, sizeof(triple), cmp_triple);
    uint64_t u = 0;
    for (uint64_t i = 0; i < ne; i++) {
        if (u > 0 && tr[i].s == se_src[u - 1] && tr[i].l == se_lab[u - 1] &&
            tr[i].d == se_dst[u - 1])
            continue;
        se_src[u] = tr[i].s; se_lab[u] = tr[i].l; se_dst[u] = tr[i].d;
        u++;
    }
    *n_se_out = u;
    *k_done_out = k_done;
    *fixpoint_out = fixpoint;
    *n_blocks_out = nb;
    free(tr); free(t); free(cur); free(nxt); free(cls); free(ncls); free(keys);
    free(pair_off); free(partner); free(salt); free(fill);
    return BO_OK;
}
