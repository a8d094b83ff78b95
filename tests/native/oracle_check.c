/*
 * Sanitizer driver for the C oracle (built by tests/test_sanitizers.py with
 * -fsanitize=address,undefined and run on the CPU).  Every entry point is
 * called on seeded random graphs -- empty ones, ones with dead vertices,
 * repeated edges and high-degree vertices -- under every flag combination,
 * and the results are checked against the definitions they must satisfy:
 *   - n_0 .. n_{k_done} never decrease, a fixpoint stop has n_k = n_{k-1};
 *   - block ids are numbered by first occurrence and the block sizes add up
 *     to the alive vertices; dead vertices have hash 0 and no block;
 *   - the summary edges are sorted, distinct, and each is the image of an
 *     edge; every edge's image is among them;
 *   - the oracle's independent code paths agree: bo_summarize with the
 *     direction/label extension in its plain setting, bo_iterate, and
 *     bo_step_strided on every vertex.
 * Prints "ok <cases>" and exits 0, or prints the failed check and exits 1.
 */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#define BO_STOP_AT_FIXPOINT 1u
#define BO_UNTYPED 4u
#define BO_BACKWARD 32u
#define BO_BOTH_DIRECTIONS 64u
#define BO_PREV_LEVEL_EDGES 128u

int bo_summarize(uint32_t n, uint64_t m, const uint64_t* row_off, const uint32_t* tgt, const uint32_t* lab,
                 const uint64_t* typ_off, const uint32_t* typ, const uint8_t* alive, uint32_t k_max,
                 uint32_t flags, uint64_t* hashes, uint64_t* prev_hashes, uint32_t* block_ids,
                 uint32_t* blocks_per_iter, uint32_t* k_done_out, uint32_t* fixpoint_out, uint32_t* n_blocks_out,
                 uint32_t* block_sizes, uint64_t* n_se_out, uint32_t* se_src, uint32_t* se_lab, uint32_t* se_dst);
int bo_summarize_ext(uint32_t n, uint64_t m, const uint64_t* row_off, const uint32_t* tgt, const uint32_t* lab,
                     const uint64_t* typ_off, const uint32_t* typ, const uint8_t* alive, uint32_t k_max,
                     uint32_t flags, const uint8_t* keep_label, uint32_t n_keep, uint64_t* hashes,
                     uint32_t* block_ids, uint32_t* blocks_per_iter, uint32_t* k_done_out, uint32_t* fixpoint_out,
                     uint32_t* n_blocks_out, uint32_t* block_sizes, uint64_t* n_se_out, uint32_t* se_src,
                     uint32_t* se_lab, uint32_t* se_dst);
int bo_iterate(uint32_t n, const uint64_t* row_off, const uint32_t* tgt, const uint32_t* lab,
               const uint64_t* typ_off, const uint32_t* typ, uint32_t iters, uint32_t flags, uint64_t* out_hashes,
               uint32_t* counts);
void bo_type_hashes(uint32_t n, const uint64_t* typ_off, const uint32_t* typ, uint32_t flags, uint64_t* t);
int bo_step_strided(uint32_t n, const uint64_t* row_off, const uint32_t* tgt, const uint32_t* lab,
                    const uint64_t* t, const uint64_t* h_prev, uint32_t v0, uint32_t stride, uint32_t count,
                    uint64_t* out);
uint32_t bo_block_ids(const uint64_t* h, const uint8_t* alive, uint32_t n, uint32_t* block);

static uint64_t rng_state;
static uint32_t rnd(uint32_t bound) {
    rng_state ^= rng_state << 13;
    rng_state ^= rng_state >> 7;
    rng_state ^= rng_state << 17;
    return bound ? (uint32_t)(rng_state % bound) : 0u;
}

#define CHECK(cond, what)                                                               \
    do {                                                                                \
        if (!(cond)) {                                                                  \
            printf("FAIL case %d: %s (%s:%d)\n", case_no, what, __FILE__, __LINE__);    \
            exit(1);                                                                    \
        }                                                                               \
    } while (0)

static int case_no = 0;

typedef struct {
    uint32_t n;
    uint64_t m;
    uint64_t* row_off;
    uint32_t* tgt;
    uint32_t* lab;
    uint64_t* typ_off;
    uint32_t* typ;
    uint8_t* alive;  /* NULL: all alive */
} graph;

static void free_graph(graph* g) {
    free(g->row_off);
    free(g->tgt);
    free(g->lab);
    free(g->typ_off);
    free(g->typ);
    free(g->alive);
}

/* n vertices, about m edges among the alive ones, n_lab labels, up to 3 types
 * of n_typ per vertex; a few hubs and repeated edges */
static graph random_graph(uint32_t n, uint32_t m_want, uint32_t n_lab, uint32_t n_typ, int with_dead) {
    graph g;
    memset(&g, 0, sizeof(g));
    g.n = n;
    g.row_off = (uint64_t*)calloc((size_t)n + 1, sizeof(uint64_t));
    g.typ_off = (uint64_t*)calloc((size_t)n + 1, sizeof(uint64_t));
    if (with_dead && n) {
        g.alive = (uint8_t*)malloc(n);
        for (uint32_t v = 0; v < n; v++) g.alive[v] = rnd(5) != 0;
    }
    uint32_t* deg = (uint32_t*)calloc((size_t)n + 1, sizeof(uint32_t));
    uint32_t n_alive = 0;
    for (uint32_t v = 0; v < n; v++) n_alive += !g.alive || g.alive[v];
    uint64_t m = 0;
    if (n_alive)
        for (uint32_t v = 0; v < n; v++) {
            if (g.alive && !g.alive[v]) continue;
            uint32_t d = rnd(2 * m_want / (n ? n : 1) + 1);
            if (rnd(40) == 0) d += rnd(4 * m_want / 10 + 1); /* a hub */
            deg[v] = d;
            m += d;
        }
    g.m = m;
    g.tgt = (uint32_t*)malloc(sizeof(uint32_t) * (m ? m : 1));
    g.lab = (uint32_t*)malloc(sizeof(uint32_t) * (m ? m : 1));
    uint64_t e = 0;
    for (uint32_t v = 0; v < n; v++) {
        g.row_off[v] = e;
        for (uint32_t j = 0; j < deg[v]; j++) {
            uint32_t w;
            do {
                w = rnd(n);
            } while (g.alive && !g.alive[w]);
            if (j && rnd(4) == 0) {
                /* repeat an earlier edge of v */
                const uint64_t f = g.row_off[v] + rnd(j);
                g.tgt[e] = g.tgt[f];
                g.lab[e] = g.lab[f];
            } else {
                g.tgt[e] = w;
                g.lab[e] = rnd(n_lab);
            }
            e++;
        }
    }
    g.row_off[n] = e;
    uint64_t nt = 0;
    for (uint32_t v = 0; v < n; v++) {
        g.typ_off[v] = nt;
        nt += (g.alive && !g.alive[v]) ? 0 : rnd(4);
    }
    g.typ_off[n] = nt;
    g.typ = (uint32_t*)malloc(sizeof(uint32_t) * (nt ? nt : 1));
    for (uint64_t i = 0; i < nt; i++) g.typ[i] = rnd(n_typ);
    free(deg);
    return g;
}

static void check_summary(const graph* g, uint32_t k_max, uint32_t flags) {
    const uint32_t n = g->n;
    const uint64_t m = g->m;
    const size_t nn = n ? n : 1, mm = m ? m : 1;
    uint64_t* h = (uint64_t*)malloc(8 * nn);
    uint64_t* hp = (uint64_t*)malloc(8 * nn);
    uint32_t* bid = (uint32_t*)malloc(4 * nn);
    uint32_t* bpi = (uint32_t*)malloc(4 * ((size_t)k_max + 1));
    uint32_t* bsz = (uint32_t*)malloc(4 * nn);
    uint32_t *ss = (uint32_t*)malloc(4 * mm), *sl = (uint32_t*)malloc(4 * mm), *sd = (uint32_t*)malloc(4 * mm);
    uint32_t kd = 0, fx = 0, nb = 0;
    uint64_t nse = 0;
    int rc = bo_summarize(n, m, g->row_off, g->tgt, g->lab, g->typ_off, g->typ, g->alive, k_max, flags, h, hp, bid,
                          bpi, &kd, &fx, &nb, bsz, &nse, ss, sl, sd);
    CHECK(rc == 0, "bo_summarize accepts a valid graph");
    CHECK(kd <= k_max, "k_done within the cap");
    uint32_t n_alive = 0;
    for (uint32_t v = 0; v < n; v++) n_alive += !g->alive || g->alive[v];
    for (uint32_t k = 1; k <= kd; k++) CHECK(bpi[k] >= bpi[k - 1], "block counts never decrease");
    CHECK(bpi[kd] <= n_alive && nb == bpi[kd], "n_blocks = n_{k_done} <= alive vertices");
    if ((flags & BO_STOP_AT_FIXPOINT) && kd < k_max) CHECK(fx && kd >= 1 && bpi[kd] == bpi[kd - 1], "fixpoint stop");
    /* first-occurrence numbering and sizes */
    uint32_t next = 0;
    uint64_t total = 0;
    for (uint32_t v = 0; v < n; v++) {
        if (g->alive && !g->alive[v]) {
            CHECK(bid[v] == 0xFFFFFFFFu && h[v] == 0, "dead vertices: no block, hash 0");
            continue;
        }
        CHECK(bid[v] <= next, "first-occurrence block ids");
        if (bid[v] == next) next++;
    }
    CHECK(next == nb, "every block id used");
    for (uint32_t b = 0; b < nb; b++) total += bsz[b];
    CHECK(total == n_alive, "block sizes add up to the alive vertices");
    /* summary edges: sorted, distinct, and exactly the images of the edges */
    for (uint64_t i = 1; i < nse; i++) {
        const int less = ss[i - 1] < ss[i] || (ss[i - 1] == ss[i] && (sl[i - 1] < sl[i] ||
                                                                      (sl[i - 1] == sl[i] && sd[i - 1] < sd[i])));
        CHECK(less, "summary edges sorted and distinct");
    }
    CHECK(nse <= m && (m == 0) == (nse == 0), "summary edge count");
    if (!(flags & BO_PREV_LEVEL_EDGES)) {
        for (uint32_t v = 0; v < n; v++)
            for (uint64_t e = g->row_off[v]; e < g->row_off[v + 1]; e++) {
                /* binary search of the image */
                uint64_t lo = 0, hi = nse;
                const uint32_t s = bid[v], l = g->lab[e], d = bid[g->tgt[e]];
                int found = 0;
                while (lo < hi) {
                    const uint64_t mid = (lo + hi) / 2;
                    const int lt = ss[mid] < s || (ss[mid] == s && (sl[mid] < l || (sl[mid] == l && sd[mid] < d)));
                    if (lt)
                        lo = mid + 1;
                    else
                        hi = mid;
                }
                found = lo < nse && ss[lo] == s && sl[lo] == l && sd[lo] == d;
                CHECK(found, "every edge's image is a summary edge");
            }
    }
    /* the extension in its plain setting is the same computation */
    if (!(flags & BO_PREV_LEVEL_EDGES)) {
        uint64_t* h2 = (uint64_t*)malloc(8 * nn);
        uint32_t* bid2 = (uint32_t*)malloc(4 * nn);
        uint32_t* bpi2 = (uint32_t*)malloc(4 * ((size_t)k_max + 1));
        uint32_t* bsz2 = (uint32_t*)malloc(4 * nn);
        uint32_t *ss2 = (uint32_t*)malloc(4 * mm), *sl2 = (uint32_t*)malloc(4 * mm), *sd2 = (uint32_t*)malloc(4 * mm);
        uint32_t kd2 = 0, fx2 = 0, nb2 = 0;
        uint64_t nse2 = 0;
        rc = bo_summarize_ext(n, m, g->row_off, g->tgt, g->lab, g->typ_off, g->typ, g->alive, k_max, flags, NULL, 0,
                              h2, bid2, bpi2, &kd2, &fx2, &nb2, bsz2, &nse2, ss2, sl2, sd2);
        CHECK(rc == 0 && kd2 == kd && fx2 == fx && nb2 == nb && nse2 == nse, "extension agrees (scalars)");
        CHECK(!memcmp(h, h2, 8 * (size_t)n) && !memcmp(bid, bid2, 4 * (size_t)n), "extension agrees (arrays)");
        CHECK(!memcmp(ss, ss2, 4 * nse) && !memcmp(sl, sl2, 4 * nse) && !memcmp(sd, sd2, 4 * nse),
              "extension agrees (summary edges)");
        /* the other directions and a label filter run cleanly */
        uint8_t keep[3] = {1, 0, 1};
        const uint32_t dirs[3] = {BO_BACKWARD, BO_BOTH_DIRECTIONS, 0};
        for (int i = 0; i < 3; i++) {
            rc = bo_summarize_ext(n, m, g->row_off, g->tgt, g->lab, g->typ_off, g->typ, g->alive, k_max,
                                  flags | dirs[i], i == 2 ? keep : NULL, 3, h2, bid2, bpi2, &kd2, &fx2, &nb2, bsz2,
                                  &nse2, ss2, sl2, sd2);
            CHECK(rc == 0 && nb2 == bpi2[kd2] && nse2 <= m, "directions and label filter");
        }
        rc = bo_summarize_ext(n, m, g->row_off, g->tgt, g->lab, g->typ_off, g->typ, g->alive, k_max,
                              flags | BO_BACKWARD | BO_BOTH_DIRECTIONS, NULL, 0, h2, bid2, bpi2, &kd2, &fx2, &nb2,
                              bsz2, &nse2, ss2, sl2, sd2);
        CHECK(rc != 0, "conflicting direction flags are refused");
        free(h2);
        free(bid2);
        free(bpi2);
        free(bsz2);
        free(ss2);
        free(sl2);
        free(sd2);
    }
    /* without dead vertices or a stop: the fixed-count iteration and the
     * strided step reproduce the hashes */
    if (!g->alive && !(flags & BO_STOP_AT_FIXPOINT) && !(flags & BO_PREV_LEVEL_EDGES)) {
        uint64_t* h3 = (uint64_t*)malloc(8 * nn);
        uint32_t* cnt = (uint32_t*)malloc(4 * ((size_t)k_max + 1));
        rc = bo_iterate(n, g->row_off, g->tgt, g->lab, g->typ_off, g->typ, kd, flags & BO_UNTYPED, h3, cnt);
        CHECK(rc == 0 && !memcmp(h3, h, 8 * (size_t)n) && !memcmp(cnt, bpi, 4 * ((size_t)kd + 1)),
              "bo_iterate agrees");
        if (kd >= 1 && n) {
            uint64_t* t = (uint64_t*)malloc(8 * nn);
            uint64_t* prev = (uint64_t*)malloc(8 * nn);
            bo_type_hashes(n, g->typ_off, g->typ, flags & BO_UNTYPED, t);
            rc = bo_iterate(n, g->row_off, g->tgt, g->lab, g->typ_off, g->typ, kd - 1, flags & BO_UNTYPED, prev, NULL);
            CHECK(rc == 0, "bo_iterate (one level less)");
            const uint32_t stride = 1 + rnd(3);
            const uint32_t count = (n - 1) / stride + 1;
            rc = bo_step_strided(n, g->row_off, g->tgt, g->lab, t, prev, 0, stride, count, h3);
            CHECK(rc == 0, "bo_step_strided");
            for (uint32_t i = 0; i < count; i++) CHECK(h3[i] == h[i * stride], "strided step agrees");
            CHECK(bo_step_strided(n, g->row_off, g->tgt, g->lab, t, prev, 0, stride, count + 1, h3) != 0,
                  "strided step refuses to run past the last vertex");
            uint32_t* b3 = (uint32_t*)malloc(4 * nn);
            const uint32_t nb3 = bo_block_ids(h, NULL, n, b3);
            CHECK(nb3 >= 1 && nb3 <= n, "bo_block_ids");
            free(b3);
            free(t);
            free(prev);
        }
        free(h3);
        free(cnt);
    }
    free(h);
    free(hp);
    free(bid);
    free(bpi);
    free(bsz);
    free(ss);
    free(sl);
    free(sd);
}

int main(int argc, char** argv) {
    rng_state = argc > 1 ? strtoull(argv[1], NULL, 10) | 1u : 0x9E3779B97F4A7C15ull;
    const uint32_t flag_sets[6] = {0, BO_STOP_AT_FIXPOINT, BO_UNTYPED, BO_STOP_AT_FIXPOINT | BO_UNTYPED,
                                   BO_PREV_LEVEL_EDGES, BO_STOP_AT_FIXPOINT | BO_PREV_LEVEL_EDGES};
    for (int round = 0; round < 60; round++) {
        const uint32_t n = round < 4 ? (uint32_t)round : 1 + rnd(round < 50 ? 120 : 2500);
        const uint32_t m = rnd(6 * n + 1);
        graph g = random_graph(n, m, 1 + rnd(6), 1 + rnd(5), round % 3 == 1);
        for (int f = 0; f < 6; f++) {
            const uint32_t k_max = (f & 1) ? n + 2 : rnd(6);
            case_no++;
            check_summary(&g, k_max, flag_sets[f]);
        }
        free_graph(&g);
    }
    /* a malformed CSR is refused, not read past its end */
    {
        uint64_t row_off[3] = {0, 2, 1};
        uint32_t tgt[2] = {0, 1}, lab[2] = {0, 0};
        uint64_t typ_off[3] = {0, 0, 0};
        uint32_t typ[1] = {0};
        uint64_t h[2], hp[2];
        uint32_t bid[2], bpi[3], bsz[2], ss[2], sl[2], sd[2], kd, fx, nb;
        uint64_t nse;
        case_no++;
        CHECK(bo_summarize(2, 1, row_off, tgt, lab, typ_off, typ, NULL, 2, 0, h, hp, bid, bpi, &kd, &fx, &nb, bsz,
                           &nse, ss, sl, sd) != 0, "decreasing row offsets are refused");
        uint64_t row_ok[3] = {0, 1, 2};
        uint32_t bad_tgt[2] = {0, 7};
        CHECK(bo_summarize(2, 2, row_ok, bad_tgt, lab, typ_off, typ, NULL, 2, 0, h, hp, bid, bpi, &kd, &fx, &nb, bsz,
                           &nse, ss, sl, sd) != 0, "out-of-range targets are refused");
        uint8_t alive[2] = {1, 0};
        CHECK(bo_summarize(2, 2, row_ok, tgt, lab, typ_off, typ, alive, 2, 0, h, hp, bid, bpi, &kd, &fx, &nb, bsz,
                           &nse, ss, sl, sd) != 0, "edges of dead vertices are refused");
    }
    printf("ok %d\n", case_no);
    return 0;
}
