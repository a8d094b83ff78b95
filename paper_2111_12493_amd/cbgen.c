/*
 * cbgen.c -- counter-based generator of large seeded input graphs (host C).
 *
 * INPUT GENERATION ONLY: this file produces graphs and holds none of the
 * summarization arithmetic.  The CPU oracle (through the Python wrapper in
 * graphgen.py) and the GPU library both consume the graphs it writes.
 *
 * Every random number is a pure function of (seed, stream, item, word): the
 * Philox4x32-10 counter-based generator of Salmon, Moraes, Dror and Shaw
 * ("Parallel random numbers: as easy as 1, 2, 3", SC 2011), written here from
 * its published description:
 *   state  (c0, c1, c2, c3), key (k0, k1)
 *   round  (hi0, lo0) = M0 * c0 and (hi1, lo1) = M1 * c2 as 64-bit products;
 *          c <- (hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0)
 *   key    k0 += W0, k1 += W1 between rounds; 10 rounds
 *   M0 = 0xD2511F53, M1 = 0xCD9E8D57, W0 = 0x9E3779B9, W1 = 0xBB67AE85
 * The key is (seed & 0xFFFFFFFF, (seed >> 32) ^ stream), so any thread can
 * draw item i, and the graph depends on neither the thread count nor the
 * machine.
 *
 * Recipes (the graph model of graphgen.py; streams are fixed per purpose):
 *   R-MAT endpoints (stream 0): edge i draws u_0..u_{scale-1} from counter
 *     (i_lo, i_hi, j, 0), u_l = word l % 4 of block j = l / 4.  Level l
 *     chooses the quadrant: u < A -> (0, 0), u < A + B -> (0, 1),
 *     u < A + B + C -> (1, 0), else (1, 1), with A = floor(a 2^32) etc.;
 *     the first level gives the most significant bit of (src, dst).
 *   edge labels (stream 1): edge i takes x = (w0 * 2^21 + (w1 >> 11)) 2^-53
 *     from words 0, 1 of counter (i_lo, i_hi, 0, 0), and the label is the
 *     first index j with cdf[j] > x, cdf the normalized cumulative sum of
 *     (j + 1)^-s (a finite Zipf law).
 *   type count (stream 2): vertex v takes lo + floor(w0 (hi - lo + 1) / 2^32)
 *     from counter (v_lo, v_hi, 0, 0).
 *   type ids (stream 3): the j-th type of v (j < 4 per block) is a Zipf draw
 *     from words 2(j % 2), 2(j % 2) + 1 of counter (v_lo, v_hi, j / 2, 0).
 * The CSR lists each vertex's out-edges in edge-index order (a stable sort
 * by source).  Self loops and repeated triples are kept.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

typedef struct { uint32_t v[4]; } cb4;

static void mulhilo(uint32_t a, uint32_t b, uint32_t* hi, uint32_t* lo) {
    const uint64_t p = (uint64_t)a * (uint64_t)b;
    *hi = (uint32_t)(p >> 32);
    *lo = (uint32_t)p;
}

/* Philox4x32-10 of counter c under key (k0, k1). */
cb4 cb_philox(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, uint32_t k0, uint32_t k1) {
    uint32_t x0 = c0, x1 = c1, x2 = c2, x3 = c3;
    for (int r = 0; r < 10; r++) {
        if (r) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        uint32_t hi0, lo0, hi1, lo1;
        mulhilo(0xD2511F53u, x0, &hi0, &lo0);
        mulhilo(0xCD9E8D57u, x2, &hi1, &lo1);
        const uint32_t y0 = hi1 ^ x1 ^ k0, y1 = lo1, y2 = hi0 ^ x3 ^ k1, y3 = lo0;
        x0 = y0;
        x1 = y1;
        x2 = y2;
        x3 = y3;
    }
    cb4 o = {{x0, x1, x2, x3}};
    return o;
}

/* Exported for the known-answer test of the generator. */
void cb_philox_out(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, uint32_t k0, uint32_t k1, uint32_t* out) {
    cb4 o = cb_philox(c0, c1, c2, c3, k0, k1);
    memcpy(out, o.v, sizeof(o.v));
}

static double unit53(uint32_t w0, uint32_t w1) {
    return ((double)w0 * 2097152.0 + (double)(w1 >> 11)) * (1.0 / 9007199254740992.0);
}

/* Normalized cumulative Zipf weights (j + 1)^-s over k ids. */
static double* zipf_cdf(uint32_t k, double s) {
    double* c = (double*)malloc(sizeof(double) * (k ? k : 1));
    if (!c) return NULL;
    double acc = 0.0;
    for (uint32_t j = 0; j < k; j++) {
        acc += pow((double)(j + 1), -s);
        c[j] = acc;
    }
    for (uint32_t j = 0; j < k; j++) c[j] /= acc;
    return c;
}

static uint32_t zipf_pick(const double* cdf, uint32_t k, double x) {
    uint32_t lo = 0, hi = k;  /* first j with cdf[j] > x */
    while (lo < hi) {
        const uint32_t mid = lo + (hi - lo) / 2;
        if (cdf[mid] > x) hi = mid; else lo = mid + 1;
    }
    return lo < k ? lo : k - 1;
}

/*
 * R-MAT edge list: src[i], dst[i], lab[i] for i in [0, m) (lab as uint16 when
 * lab_u16, else uint32).  Returns 0, or -1 when memory runs out.
 */
int cb_rmat_edges(uint64_t seed, uint32_t scale, uint64_t m, double a, double b, double c, uint32_t n_labels,
                  double s_labels, uint32_t* src, uint32_t* dst, void* lab, int lab_u16) {
    const uint64_t A = (uint64_t)floor(a * 4294967296.0);
    const uint64_t AB = (uint64_t)floor((a + b) * 4294967296.0);
    const uint64_t ABC = (uint64_t)floor((a + b + c) * 4294967296.0);
    const uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
    double* cdf = zipf_cdf(n_labels, s_labels);
    if (!cdf) return -1;
    int64_t i;
#pragma omp parallel for schedule(static, 65536)
    for (i = 0; i < (int64_t)m; i++) {
        const uint32_t lo = (uint32_t)i, hi = (uint32_t)((uint64_t)i >> 32);
        uint32_t s = 0, d = 0;
        cb4 r = {{0, 0, 0, 0}};
        for (uint32_t l = 0; l < scale; l++) {
            if ((l & 3) == 0) r = cb_philox(lo, hi, l >> 2, 0, k0, k1 ^ 0u);
            const uint64_t u = r.v[l & 3];
            const uint32_t sb = u >= AB, db = (u >= A && u < AB) || u >= ABC;
            s = (s << 1) | sb;
            d = (d << 1) | db;
        }
        src[i] = s;
        dst[i] = d;
        const cb4 q = cb_philox(lo, hi, 0, 0, k0, k1 ^ 1u);
        const uint32_t li = zipf_pick(cdf, n_labels, unit53(q.v[0], q.v[1]));
        if (lab_u16) ((uint16_t*)lab)[i] = (uint16_t)li;
        else ((uint32_t*)lab)[i] = li;
    }
    free(cdf);
    return 0;
}

/*
 * CSR from an edge list, stable in edge order: row_off[n+1] (uint64), and
 * tgt / lab (label width lab_bytes) in CSR order.  Returns 0, -1 on memory,
 * -2 on an endpoint >= n.
 *
 * A parallel counting sort in two levels that keeps edge order within a
 * source: edges go to source-range buckets (chunks of the edge list in
 * order, edges in order within a chunk), then each bucket is counted and
 * placed by exact source.  The result does not depend on the thread count.
 */
int cb_csr(uint32_t n, uint64_t m, const uint32_t* src, const uint32_t* dst, const void* lab, int lab_bytes,
           uint64_t* row_off, uint32_t* tgt, void* lab_out) {
    int bits = 0;
    while (bits < 32 && ((uint64_t)1 << bits) < (uint64_t)n) bits++;
    const int bs = bits > 12 ? bits - 12 : 0;                 /* at most 4096 buckets */
    const uint64_t B = n ? (((uint64_t)n - 1) >> bs) + 1 : 1;
    const uint64_t C = 256;                                   /* edge chunks */
    const uint64_t per = (m + C - 1) / C;
    uint64_t* hist = (uint64_t*)calloc(C * B, sizeof(uint64_t));
    uint64_t* bstart = (uint64_t*)malloc(sizeof(uint64_t) * (B + 1));
    uint32_t* ts = (uint32_t*)malloc(sizeof(uint32_t) * (m ? m : 1));
    uint32_t* td = (uint32_t*)malloc(sizeof(uint32_t) * (m ? m : 1));
    uint8_t* tl = (uint8_t*)malloc((size_t)lab_bytes * (m ? m : 1));
    if (!hist || !bstart || !ts || !td || !tl) {
        free(hist); free(bstart); free(ts); free(td); free(tl);
        return -1;
    }
    int bad = 0;
    int64_t c;
#pragma omp parallel for schedule(dynamic, 1) reduction(|: bad)
    for (c = 0; c < (int64_t)C; c++) {
        const uint64_t i0 = (uint64_t)c * per, i1 = i0 + per < m ? i0 + per : m;
        uint64_t* h = hist + (uint64_t)c * B;
        for (uint64_t i = i0; i < i1; i++) {
            if (src[i] >= n || dst[i] >= n) {
                bad = 1;
                break;
            }
            h[src[i] >> bs]++;
        }
    }
    if (bad) {
        free(hist); free(bstart); free(ts); free(td); free(tl);
        return -2;
    }
    /* bucket-major, chunk-minor exclusive prefix: hist becomes the offsets */
    uint64_t pos = 0;
    for (uint64_t b = 0; b < B; b++) {
        bstart[b] = pos;
        for (uint64_t cc = 0; cc < C; cc++) {
            const uint64_t x = hist[cc * B + b];
            hist[cc * B + b] = pos;
            pos += x;
        }
    }
    bstart[B] = pos;
#pragma omp parallel for schedule(dynamic, 1)
    for (c = 0; c < (int64_t)C; c++) {
        const uint64_t i0 = (uint64_t)c * per, i1 = i0 + per < m ? i0 + per : m;
        uint64_t* cur = hist + (uint64_t)c * B;
        for (uint64_t i = i0; i < i1; i++) {
            const uint64_t p = cur[src[i] >> bs]++;
            ts[p] = src[i];
            td[p] = dst[i];
            memcpy(tl + p * lab_bytes, (const uint8_t*)lab + i * lab_bytes, (size_t)lab_bytes);
        }
    }
    int64_t b;
    int oom = 0;
#pragma omp parallel for schedule(dynamic, 1) reduction(|: oom)
    for (b = 0; b < (int64_t)B; b++) {
        const uint64_t v0 = (uint64_t)b << bs;
        const uint64_t v1 = v0 + ((uint64_t)1 << bs) < n ? v0 + ((uint64_t)1 << bs) : n;
        uint64_t* cnt = (uint64_t*)calloc((size_t)(v1 - v0) + 1, sizeof(uint64_t));
        if (!cnt) {
            oom = 1;
            continue;
        }
        for (uint64_t p = bstart[b]; p < bstart[b + 1]; p++) cnt[ts[p] - v0]++;
        uint64_t run = bstart[b];
        for (uint64_t v = v0; v < v1; v++) {
            const uint64_t x = cnt[v - v0];
            row_off[v] = run;
            cnt[v - v0] = run;
            run += x;
        }
        for (uint64_t p = bstart[b]; p < bstart[b + 1]; p++) {
            const uint64_t q = cnt[ts[p] - v0]++;
            tgt[q] = td[p];
            memcpy((uint8_t*)lab_out + q * lab_bytes, tl + p * lab_bytes, (size_t)lab_bytes);
        }
        free(cnt);
    }
    row_off[n] = m;
    free(hist); free(bstart); free(ts); free(td); free(tl);
    return oom ? -1 : 0;
}

/* Type counts per vertex (lo..hi), written to cnt[n]. */
void cb_type_counts(uint64_t seed, uint32_t n, uint32_t lo, uint32_t hi, uint32_t* cnt) {
    const uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
    const uint64_t span = (uint64_t)hi - lo + 1;
    int64_t v;
#pragma omp parallel for schedule(static, 65536)
    for (v = 0; v < (int64_t)n; v++) {
        const cb4 q = cb_philox((uint32_t)v, 0, 0, 0, k0, k1 ^ 2u);
        cnt[v] = lo + (uint32_t)(((uint64_t)q.v[0] * span) >> 32);
    }
}

/* Type ids of every vertex at typ_off[v] (uint64 offsets, counts from
 * cb_type_counts).  Returns 0 or -1 on memory. */
int cb_type_ids(uint64_t seed, uint32_t n, uint32_t n_types, double s_types, const uint64_t* typ_off,
                uint32_t* typ) {
    const uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
    double* cdf = zipf_cdf(n_types, s_types);
    if (!cdf) return -1;
    int64_t v;
#pragma omp parallel for schedule(static, 65536)
    for (v = 0; v < (int64_t)n; v++) {
        const uint64_t a = typ_off[v], cnt = typ_off[v + 1] - a;
        cb4 q = {{0, 0, 0, 0}};
        for (uint64_t j = 0; j < cnt; j++) {
            if ((j & 1) == 0) q = cb_philox((uint32_t)v, 0, (uint32_t)(j >> 1), 0, k0, k1 ^ 3u);
            const uint32_t w = (uint32_t)(2 * (j & 1));
            typ[a + j] = zipf_pick(cdf, n_types, unit53(q.v[w], q.v[w + 1]));
        }
    }
    free(cdf);
    return 0;
}

int cb_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
