// bsim_resolve.h -- host-side resolution of an update batch (Sec. 3.2):
// the ordered operations of one bsim_apply_updates call become the net
// change of every touched (u, label, w) triple and the final type set of
// every touched vertex.  Host code only (no HIP), so it also builds into
// the CPU tests, under the address and undefined-behaviour sanitizers.
#pragma once

#include <algorithm>
#include <cstdint>
#include <thread>
#include <utility>
#include <vector>

#include "bsim.h"
#include "bsim_host.h"

namespace bsim {

constexpr uint32_t kChgDeleted = 1u;  // change flags: the triple's old copies go
constexpr uint32_t kChgPresent = 2u;  // ... and it exists after the batch
constexpr uint32_t kMaxStateTypes = 4096;

// Net effect of one update batch, resolved on the host.
struct HostBatch {
    uint32_t n_new = 0;
    std::vector<uint32_t> cu, cw, cl, cf;      // changed triples, sorted by (u, w, l)
    std::vector<uint32_t> gsrc, gbeg, gend;    // change range of every source
    std::vector<uint32_t> rw, ru;              // reverse-list additions, sorted by (w, u)
    std::vector<uint32_t> rgw, rgbeg, rgend;
    std::vector<uint32_t> tl, tl_off, tl_ids;  // vertices with a new type set (sorted) and the sets
    std::vector<uint32_t> dead;                // vertices deleted by the batch
    uint32_t max_label = 0;
    uint64_t n_present = 0;                    // changes that end present (upper bound of appends)
};

// One edge operation's record: (u, w, l) and whether it adds the triple.
struct ResolveRec {
    uint32_t u, w, l, add;
};

// Per-vertex marks of the resolution, kept between calls so a batch costs
// O(batch) rather than O(n): vmark[v] = 0 untouched, 1 alive with a vertex
// op, 2 deleted; vtype[v] = 1 + index of v's new type list (0: none).  The
// other members are buffers reused from batch to batch: a large batch
// spends much of its host time on first touches of freshly allocated
// memory otherwise.
struct ResolveScratch {
    std::vector<uint8_t> vmark;
    std::vector<uint32_t> vtype;
    std::vector<std::vector<ResolveRec>> part;  // edge records per thread
    std::vector<ResolveRec> recs;
    std::vector<uint64_t> key, key2;
    std::vector<uint32_t> val, val2;
    std::vector<uint64_t> vpos;   // positions of the vertex operations
    std::vector<uint64_t> dbits;  // deleted vertices
    HostBatch hb;  // the result of resolve_ops_into
};

// Stable LSD radix sort of (key, val) pairs on the low `bits` bits of key.
// Large inputs are split over host threads: per pass, every thread counts
// the digits of its share, one prefix over (digit, thread) places them, and
// every thread scatters its share (so equal digits keep their order).
// k2 and v2 are buffers of the caller (resized to n; their contents are
// lost).
inline void host_radix_sort(std::vector<uint64_t>& key, std::vector<uint32_t>& val, int bits,
                            std::vector<uint64_t>& k2, std::vector<uint32_t>& v2) {
    constexpr int kDigit = 11;
    constexpr uint32_t kBuckets = 1u << kDigit;
    const size_t n = key.size();
    if (n < 2) return;
    const unsigned hw = std::thread::hardware_concurrency();
    const size_t T = std::max<size_t>(1, std::min<size_t>({static_cast<size_t>(hw ? hw : 1), 8, n / 65536}));
    k2.resize(n);
    v2.resize(n);
    std::vector<uint32_t> cnt(kBuckets * T);
    auto par = [&](auto f) {
        std::vector<std::thread> th;
        size_t t = 1;
        try {
            for (; t < T; t++) th.emplace_back(f, t);
        } catch (...) {
        }
        for (size_t u = t; u < T; u++) f(u);  // shares no thread could take
        f(0);
        for (auto& x : th) x.join();
    };
    for (int sh = 0; sh < bits; sh += kDigit) {
        par([&](size_t t) {
            uint32_t* c = &cnt[t * kBuckets];
            std::fill(c, c + kBuckets, 0u);
            for (size_t i = n * t / T, e = n * (t + 1) / T; i < e; i++) c[(key[i] >> sh) & (kBuckets - 1)]++;
        });
        uint32_t run = 0;
        for (uint32_t d = 0; d < kBuckets; d++)
            for (size_t t = 0; t < T; t++) {
                uint32_t& c = cnt[t * kBuckets + d];
                const uint32_t x = c;
                c = run;
                run += x;
            }
        par([&](size_t t) {
            uint32_t* c = &cnt[t * kBuckets];
            for (size_t i = n * t / T, e = n * (t + 1) / T; i < e; i++) {
                const uint32_t p = c[(key[i] >> sh) & (kBuckets - 1)]++;
                k2[p] = key[i];
                v2[p] = val[i];
            }
        });
        key.swap(k2);
        val.swap(v2);
    }
}

// The batch's net effect, by the sequential semantics of the operations:
// every (u, l, w) the batch touches ends deleted and/or present, every
// touched vertex ends alive with a type set or deleted.  n0 is the state's
// vertex count, alive its alive mask (n0 entries), label_bytes its label
// width.  Per-vertex marks live in the caller's scratch (all zero on entry
// and again on every return or throw), and the edge records are radix
// sorted, so a batch of 10^6 operations resolves in tens of milliseconds.
// Throws DeviceError for an invalid batch (out-of-range ids or labels,
// deleted vertices named, too many types, unknown op codes).
// The same into hb (its vectors are cleared first; their capacity is kept).
inline HostBatch& resolve_ops_into(HostBatch& hb, uint32_t n0, uint32_t label_bytes,
                                   const std::vector<uint8_t>& alive, ResolveScratch& rs, const bsim_update* ops,
                                   uint64_t n_ops) {
    for (std::vector<uint32_t>* v : {&hb.cu, &hb.cw, &hb.cl, &hb.cf, &hb.gsrc, &hb.gbeg, &hb.gend, &hb.rw, &hb.ru,
                                     &hb.rgw, &hb.rgbeg, &hb.rgend, &hb.tl, &hb.tl_off, &hb.tl_ids, &hb.dead})
        v->clear();
    hb.n_new = 0;
    hb.max_label = 0;
    hb.n_present = 0;
    uint32_t n_cur = n0;
    std::vector<uint8_t>& vmark = rs.vmark;
    std::vector<uint32_t>& vtype = rs.vtype;
    std::vector<uint32_t> touched;   // vertices with a vertex op, first touch order
    std::vector<uint32_t> ty_pool;   // type lists of the vertex ops
    std::vector<std::pair<uint32_t, uint32_t>> ty_rec;  // (offset, count) in ty_pool
    auto grow = [&](uint32_t need) {
        if (vmark.size() < need) {
            vmark.resize(std::max<size_t>(need, vmark.size() + vmark.size() / 4), 0);
            vtype.resize(vmark.size(), 0);
        }
    };
    grow(n_cur);
    auto alive_now = [&](uint32_t v) -> bool {
        const uint8_t m = vmark[v];
        return m ? m == 1 : alive[v] != 0;
    };
    using Rec = ResolveRec;
    std::vector<Rec>& recs = rs.recs;
    recs.clear();
    const uint64_t lab_lim = label_bytes == 2 ? (1ull << 16) : (1ull << 24);
    uint32_t max_l = 0;
    auto touch = [&](uint32_t v, uint8_t state) {
        if (!vmark[v]) touched.push_back(v);
        vmark[v] = state;
    };
    auto set_types = [&](uint32_t v, const bsim_update& o) {
        ty_rec.emplace_back(static_cast<uint32_t>(ty_pool.size()), o.n_types);
        ty_pool.insert(ty_pool.end(), o.types, o.types + o.n_types);
        vtype[v] = static_cast<uint32_t>(ty_rec.size());
    };
    // the marks of the touched vertices are cleared on every way out,
    // including a throw, so the next call starts from clean scratch
    struct ClearMarks {
        std::vector<uint32_t>& touched;
        std::vector<uint8_t>& vmark;
        std::vector<uint32_t>& vtype;
        ~ClearMarks() {
            for (uint32_t v : touched) vmark[v] = 0, vtype[v] = 0;
        }
    } clear_marks{touched, vmark, vtype};
    // Which ids exist and live changes only with the vertex operations, so
    // they run first, in order, up to the first invalid one; every edge
    // operation is then checked against the positions of those changes, on
    // several threads.  The batch's error is the one of its first invalid
    // operation, as in a sequential pass.
    struct Fail {
        uint64_t pos = UINT64_MAX;
        int status = BSIM_OK;
        const char* msg = nullptr;
    };
    Fail vfail;
    std::vector<uint64_t> add_pos;                     // ADD_V positions, by new id - n0
    std::vector<std::pair<uint32_t, uint64_t>> dels;   // (vertex, DEL_V position)
    // the positions of the vertex operations (and of unknown op codes)
    std::vector<uint64_t>& vpos = rs.vpos;
    vpos.clear();
    {
        const unsigned hwv = std::thread::hardware_concurrency();
        const size_t TV = std::max<size_t>(1, std::min<size_t>({static_cast<size_t>(hwv ? hwv : 1), 8, n_ops / 65536}));
        std::vector<std::vector<uint64_t>> found(TV);
        auto scan = [&](size_t t) {
            for (uint64_t i = n_ops * t / TV, e = n_ops * (t + 1) / TV; i < e; i++)
                if (ops[i].op < BSIM_OP_ADD_E || ops[i].op > BSIM_OP_DEL_E) found[t].push_back(i);
        };
        std::vector<std::thread> th;
        size_t t = 1;
        try {
            for (; t < TV; t++) th.emplace_back(scan, t);
        } catch (...) {
        }
        for (size_t u = t; u < TV; u++) scan(u);
        scan(0);
        for (auto& x : th) x.join();
        for (const auto& f : found) vpos.insert(vpos.end(), f.begin(), f.end());
    }
    // the marks of the vertex kPv operations ahead are fetched meanwhile
    constexpr size_t kPv = 16;
    auto prefetch_v = [&](size_t k) {
        if (k >= vpos.size()) return;
        const uint32_t u = ops[vpos[k]].u;
        if (u < vmark.size()) {
            __builtin_prefetch(&vmark[u]);
            __builtin_prefetch(&vtype[u]);
        }
        if (u < alive.size()) __builtin_prefetch(&alive[u]);
    };
    for (size_t k = 0; k < kPv; k++) prefetch_v(k);
    for (size_t k = 0; k < vpos.size() && vfail.pos == UINT64_MAX; k++) {
        prefetch_v(k + kPv);
        const uint64_t i = vpos[k];
        const bsim_update& o = ops[i];
        const uint32_t op = o.op;
        auto fail = [&](int st, const char* msg) { vfail = Fail{i, st, msg}; };
        if (op < BSIM_OP_ADD_V || op > BSIM_OP_DEL_E) {
            fail(BSIM_E_INVALID, "unknown update op code");
            break;
        }
        // checks in the order: ids in range, ids alive, types
        if (op != BSIM_OP_ADD_V) {
            if (o.u >= n_cur) {
                fail(BSIM_E_RANGE, "vertex id out of range in update");
                break;
            }
            if (!alive_now(o.u)) {
                fail(BSIM_E_INVALID, "update names a deleted vertex");
                break;
            }
        }
        if (op != BSIM_OP_DEL_V) {
            if (o.n_types > kMaxStateTypes) {
                fail(BSIM_E_UNSUPPORTED, "more than 4096 types on a vertex");
                break;
            }
            if (o.n_types && !o.types) {
                fail(BSIM_E_INVALID, "types pointer is NULL");
                break;
            }
        }
        if (op == BSIM_OP_ADD_V) {
            if (n_cur >= 0xFFFFFFF0u) {
                fail(BSIM_E_UNSUPPORTED, "too many vertices");
                break;
            }
            const uint32_t v = n_cur++;
            grow(n_cur);
            touch(v, 1);
            set_types(v, o);
            add_pos.push_back(i);
        } else if (op == BSIM_OP_MOD_V) {
            touch(o.u, 1);
            set_types(o.u, o);
        } else {
            touch(o.u, 2);
            vtype[o.u] = 0;
            dels.emplace_back(o.u, i);
        }
    }
    std::sort(dels.begin(), dels.end());
    // v exists at position i: an old id, or added before i
    auto exists_at = [&](uint32_t v, uint64_t i) {
        return v < n0 || (static_cast<uint64_t>(v) - n0 < add_pos.size() && add_pos[v - n0] < i);
    };
    // v (existing at i) lives at i: alive before the batch or added, and
    // not deleted before i
    auto alive_at = [&](uint32_t v, uint64_t i) {
        if (v < n0 && !alive[v]) return false;
        if (vmark[v] != 2) return true;
        const auto it = std::lower_bound(dels.begin(), dels.end(), std::make_pair(v, uint64_t(0)));
        return !(it != dels.end() && it->first == v && it->second < i);
    };
    const uint64_t lab_lim_e = lab_lim;
    const uint64_t end = std::min<uint64_t>(n_ops, vfail.pos);  // later operations do not count
    const unsigned hw = std::thread::hardware_concurrency();
    const size_t T = std::max<size_t>(1, std::min<size_t>({static_cast<size_t>(hw ? hw : 1), 8, end / 65536}));
    std::vector<std::vector<Rec>>& part = rs.part;
    if (part.size() < T) part.resize(T);
    std::vector<Fail> efail(T);
    std::vector<uint32_t> part_max(T, 0);
    auto check_edges = [&](size_t t) {
        const uint64_t a = end * t / T, b = end * (t + 1) / T;
        std::vector<Rec>& out = part[t];
        out.clear();
        out.reserve((b - a) + (b - a) / 4);
        uint32_t ml = 0;
        // the marks and the alive mask are read at random: the entries of
        // the operation kPf places ahead are fetched meanwhile
        constexpr uint64_t kPf = 24;
        const size_t lim = std::min(vmark.size(), alive.size());
        auto prefetch = [&](const bsim_update& o) {
            if (!lim) return;
            __builtin_prefetch(&alive[std::min<size_t>(o.u, lim - 1)]);
            __builtin_prefetch(&alive[std::min<size_t>(o.w, lim - 1)]);
            __builtin_prefetch(&vmark[std::min<size_t>(o.u, lim - 1)]);
            __builtin_prefetch(&vmark[std::min<size_t>(o.w, lim - 1)]);
        };
        for (uint64_t i = a; i < b && i < a + kPf; i++) prefetch(ops[i]);
        for (uint64_t i = a; i < b; i++) {
            if (i + kPf < b) prefetch(ops[i + kPf]);
            const bsim_update& o = ops[i];
            if (o.op < BSIM_OP_ADD_E || o.op > BSIM_OP_DEL_E) continue;
            // checks in the order: ids in range, ids alive, labels
            if (!exists_at(o.u, i) || !exists_at(o.w, i)) {
                efail[t] = Fail{i, BSIM_E_RANGE, "vertex id out of range in update"};
                break;
            }
            if (!alive_at(o.u, i) || !alive_at(o.w, i)) {
                efail[t] = Fail{i, BSIM_E_INVALID, "update names a deleted vertex"};
                break;
            }
            if (o.label >= lab_lim_e || (o.op == BSIM_OP_MOD_E && o.new_label >= lab_lim_e)) {
                efail[t] = Fail{i, BSIM_E_RANGE, "edge label out of range in update"};
                break;
            }
            out.push_back({o.u, o.w, o.label, o.op == BSIM_OP_ADD_E ? 1u : 0u});
            ml = std::max(ml, o.label);
            if (o.op == BSIM_OP_MOD_E) {
                out.push_back({o.u, o.w, o.new_label, 1});
                ml = std::max(ml, o.new_label);
            }
        }
        part_max[t] = ml;
    };
    {
        std::vector<std::thread> th;
        size_t t = 1;
        try {
            for (; t < T; t++) th.emplace_back(check_edges, t);
        } catch (...) {
        }
        for (size_t u = t; u < T; u++) check_edges(u);  // shares no thread could take
        check_edges(0);
        for (auto& x : th) x.join();
    }
    Fail first = vfail;
    for (const Fail& f : efail)
        if (f.pos < first.pos) first = f;
    if (first.pos != UINT64_MAX) throw DeviceError{first.status, first.msg};
    size_t nrec = 0;
    for (const auto& q : part) nrec += q.size();
    recs.reserve(nrec);
    for (size_t t = 0; t < T; t++) {
        recs.insert(recs.end(), part[t].begin(), part[t].end());
        max_l = std::max(max_l, part_max[t]);
    }
    hb.n_new = n_cur;
    hb.tl = touched;
    std::sort(hb.tl.begin(), hb.tl.end());
    hb.tl_off.reserve(hb.tl.size() + 1);
    hb.tl_off.push_back(0);
    for (size_t k = 0; k < hb.tl.size(); k++) {
        if (k + 16 < hb.tl.size()) {
            __builtin_prefetch(&vmark[hb.tl[k + 16]]);
            __builtin_prefetch(&vtype[hb.tl[k + 16]]);
        }
        const uint32_t v = hb.tl[k];
        if (vmark[v] == 2) {
            hb.dead.push_back(v);
        } else if (vtype[v]) {
            const auto& r = ty_rec[vtype[v] - 1];
            hb.tl_ids.insert(hb.tl_ids.end(), ty_pool.begin() + r.first, ty_pool.begin() + r.first + r.second);
        }
        hb.tl_off.push_back(static_cast<uint32_t>(hb.tl_ids.size()));
    }
    // the deleted vertices as a bitmap (n bits: mostly in cache)
    std::vector<uint64_t>& dbits = rs.dbits;
    const bool any_dead = !hb.dead.empty();
    if (any_dead) {
        dbits.assign((static_cast<size_t>(n_cur) + 63) / 64, 0);
        for (uint32_t v : hb.dead) dbits[v >> 6] |= 1ull << (v & 63);
    }
    auto dead_at_end = [&](uint32_t v) { return any_dead && ((dbits[v >> 6] >> (v & 63)) & 1); };
    // edge records in (u, w, l) order, input order within equal triples:
    // the triple packed in one key when it fits 64 bits (the add flag rides
    // in the value), else a comparison sort
    const int bv = std::max(1, bit_width(n_cur)), bl = std::max(1, bit_width(max_l + 1));
    const size_t nr = recs.size();
    std::vector<uint64_t>& key = rs.key;
    std::vector<uint32_t>& val = rs.val;
    key.clear();
    val.resize(nr);
    auto emit = [&](uint32_t u, uint32_t w, uint32_t l, bool deleted, bool add) {
        if (dead_at_end(u) || dead_at_end(w)) return;
        hb.cu.push_back(u);
        hb.cw.push_back(w);
        hb.cl.push_back(l);
        hb.cf.push_back((deleted ? kChgDeleted : 0u) | (add ? kChgPresent : 0u));
        if (add) {
            hb.n_present++;
            hb.max_label = std::max(hb.max_label, l);
            hb.rw.push_back(w);
            hb.ru.push_back(u);
        }
    };
    hb.cu.reserve(nr);
    hb.cw.reserve(nr);
    hb.cl.reserve(nr);
    hb.cf.reserve(nr);
    if (2 * bv + bl <= 64) {
        key.resize(nr);
        for (size_t i = 0; i < nr; i++) {
            key[i] = (static_cast<uint64_t>(recs[i].u) << (bv + bl)) | (static_cast<uint64_t>(recs[i].w) << bl) |
                     recs[i].l;
            val[i] = recs[i].add;
        }
        host_radix_sort(key, val, 2 * bv + bl, rs.key2, rs.val2);
        const uint64_t lmask = (1ull << bl) - 1, wmask = (1ull << bv) - 1;
        for (size_t i = 0; i < nr;) {
            size_t j = i;
            bool deleted = false;
            while (j < nr && key[j] == key[i]) deleted |= val[j++] == 0;
            emit(static_cast<uint32_t>(key[i] >> (bv + bl)), static_cast<uint32_t>((key[i] >> bl) & wmask),
                 static_cast<uint32_t>(key[i] & lmask), deleted, val[j - 1] != 0);
            i = j;
        }
    } else {
        for (size_t i = 0; i < nr; i++) val[i] = static_cast<uint32_t>(i);
        std::stable_sort(val.begin(), val.end(), [&](uint32_t a, uint32_t b) {
            const Rec &x = recs[a], &y = recs[b];
            if (x.u != y.u) return x.u < y.u;
            if (x.w != y.w) return x.w < y.w;
            return x.l < y.l;
        });
        for (size_t i = 0; i < nr;) {
            const Rec& first = recs[val[i]];
            size_t j = i;
            bool deleted = false;
            while (j < nr && recs[val[j]].u == first.u && recs[val[j]].w == first.w && recs[val[j]].l == first.l)
                deleted |= recs[val[j++]].add == 0;
            emit(first.u, first.w, first.l, deleted, recs[val[j - 1]].add != 0);
            i = j;
        }
    }
    for (size_t i = 0; i < hb.cu.size();) {
        size_t j = i;
        while (j < hb.cu.size() && hb.cu[j] == hb.cu[i]) j++;
        hb.gsrc.push_back(hb.cu[i]);
        hb.gbeg.push_back(static_cast<uint32_t>(i));
        hb.gend.push_back(static_cast<uint32_t>(j));
        i = j;
    }
    // reverse additions, grouped by target (duplicate pairs are harmless)
    std::vector<uint64_t>& rk = rs.key;  // the edge records' keys are done with
    std::vector<uint32_t>& rdummy = rs.val;
    rk.resize(hb.rw.size());
    rdummy.resize(hb.rw.size());
    for (size_t i = 0; i < rk.size(); i++) rk[i] = (static_cast<uint64_t>(hb.rw[i]) << bv) | hb.ru[i];
    host_radix_sort(rk, rdummy, 2 * bv, rs.key2, rs.val2);
    rk.erase(std::unique(rk.begin(), rk.end()), rk.end());
    hb.rw.resize(rk.size());
    hb.ru.resize(rk.size());
    const uint64_t umask = (1ull << bv) - 1;
    for (size_t i = 0; i < rk.size(); i++) {
        hb.rw[i] = static_cast<uint32_t>(rk[i] >> bv);
        hb.ru[i] = static_cast<uint32_t>(rk[i] & umask);
    }
    for (size_t i = 0; i < hb.rw.size();) {
        size_t j = i;
        while (j < hb.rw.size() && hb.rw[j] == hb.rw[i]) j++;
        hb.rgw.push_back(hb.rw[i]);
        hb.rgbeg.push_back(static_cast<uint32_t>(i));
        hb.rgend.push_back(static_cast<uint32_t>(j));
        i = j;
    }
    return hb;
}

// The net effect of the batch as a new HostBatch.
inline HostBatch resolve_ops(uint32_t n0, uint32_t label_bytes, const std::vector<uint8_t>& alive,
                             ResolveScratch& rs, const bsim_update* ops, uint64_t n_ops) {
    HostBatch hb;
    resolve_ops_into(hb, n0, label_bytes, alive, rs, ops, n_ops);
    return hb;
}

}  // namespace bsim
