// bsim_resolve.h -- host-side resolution of an update batch (Sec. 3.2):
// the ordered operations of one bsim_apply_updates call become the net
// change of every touched (u, label, w) triple and the final type set of
// every touched vertex.  Host code only (no HIP), so it also builds into
// the CPU tests, under the address and undefined-behaviour sanitizers.
#pragma once

#include <algorithm>
#include <array>
#include <condition_variable>
#include <cstdint>
#include <exception>
#include <functional>
#include <memory>
#include <mutex>
#include <thread>
#include <utility>
#include <vector>

#include <sys/types.h>
#include <unistd.h>

#include "bsim.h"
#include "bsim_host.h"

namespace bsim {

constexpr uint32_t kChgDeleted = 1u;  // change flags: the triple's old copies go
constexpr uint32_t kChgPresent = 2u;  // ... and it exists after the batch
constexpr uint32_t kMaxStateTypes = 4096;

// Host threads kept for the parallel passes of the resolution.  A large
// batch runs about thirty such passes; starting and joining threads for
// each cost about a fifth of the resolution of a 5 * 10^5-operation batch.
// One pool serves the process (shared_host_pool); a pass that finds it busy
// (another state's resolution on another thread) starts threads of its own.
class HostPool {
  public:
    explicit HostPool(size_t workers) {
        for (size_t i = 0; i < workers; i++) {
            try {
                th_.emplace_back([this, i] { loop(i + 1); });
            } catch (...) {
                break;  // fewer workers; the caller runs their shares
            }
        }
    }
    ~HostPool() {
        {
            std::lock_guard<std::mutex> lk(mu_);
            stop_ = true;
        }
        cv_.notify_all();
        for (auto& t : th_) t.join();
    }
    HostPool(const HostPool&) = delete;
    HostPool& operator=(const HostPool&) = delete;

    // f(0 .. T-1) with shares 1 .. W on the workers (W = min(T - 1,
    // workers)) and the others on the calling thread; returns when all are
    // done and rethrows the first exception of any share.  Returns false
    // at once, running nothing, when the pool is running another job or
    // belongs to another process (a fork keeps no threads).
    bool try_run(size_t T, const std::function<void(size_t)>& f) {
        const size_t W = std::min(T ? T - 1 : 0, th_.size());
        {
            std::lock_guard<std::mutex> lk(mu_);
            if (busy_ || owner_ != getpid()) return false;
            busy_ = true;
            job_ = &f;
            job_n_ = W;
            pending_ = W;
            err_ = nullptr;
            gen_++;
        }
        if (W) cv_.notify_all();
        std::exception_ptr mine;
        for (size_t u = W + 1; u <= T; u++) {  // shares W+1 .. T-1, then 0
            try {
                f(u < T ? u : 0);
            } catch (...) {
                if (!mine) mine = std::current_exception();
            }
        }
        std::unique_lock<std::mutex> lk(mu_);
        done_.wait(lk, [&] { return pending_ == 0; });
        job_ = nullptr;
        busy_ = false;
        if (mine) std::rethrow_exception(mine);
        if (err_) std::rethrow_exception(err_);
        return true;
    }

  private:
    void loop(size_t id) {
        uint64_t seen = 0;
        for (;;) {
            const std::function<void(size_t)>* job;
            {
                std::unique_lock<std::mutex> lk(mu_);
                cv_.wait(lk, [&] { return stop_ || gen_ != seen; });
                if (stop_) return;
                seen = gen_;
                if (id > job_n_) continue;  // not a share of this job
                job = job_;
            }
            std::exception_ptr e;
            try {
                (*job)(id);
            } catch (...) {
                e = std::current_exception();
            }
            std::lock_guard<std::mutex> lk(mu_);
            if (e && !err_) err_ = e;
            if (--pending_ == 0) done_.notify_one();
        }
    }
    std::mutex mu_;
    std::condition_variable cv_, done_;
    std::vector<std::thread> th_;
    const std::function<void(size_t)>* job_ = nullptr;
    size_t job_n_ = 0, pending_ = 0;
    uint64_t gen_ = 0;
    std::exception_ptr err_;
    bool stop_ = false, busy_ = false;
    const pid_t owner_ = getpid();
};

// The process's pool: min(hardware threads, 8) - 1 workers, started on
// first use.  It is never destroyed: its idle workers end with the process,
// and a process forked from this one (which has none of its threads) never
// joins them.
inline HostPool& shared_host_pool() {
    static HostPool* pool = new HostPool([] {
        const unsigned hw = std::thread::hardware_concurrency();
        return static_cast<size_t>(std::min(hw ? hw : 1u, 8u) - 1);
    }());
    return *pool;
}

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
    std::vector<uint64_t> dbits, dfilt;  // deleted vertices, and a small filter of them
    // one thread's share of the changes and reverse additions, with its
    // groups (offsets within the share)
    struct Part {
        std::vector<uint32_t> cu, cw, cl, cf, rw, ru, gsrc, gbeg;
        uint64_t n_present = 0;
        uint32_t max_label = 0;
    };
    std::vector<Part> parts;
    HostBatch hb;  // the result of resolve_ops_into
};

// Run f(0..T-1) on T host threads (share 0 on the calling thread; a share
// whose thread cannot be started runs on the calling thread too), on the
// pool's threads when one is given and free.  Every share runs; the first
// exception of any share is rethrown after all have ended.
template <typename F>
inline void host_parallel(size_t T, F f, HostPool* pool = nullptr) {
    if (T <= 1) {
        if (T) f(0);
        return;
    }
    if (pool && pool->try_run(T, std::function<void(size_t)>(f))) return;
    // threads of the call's own; every share runs, and the first exception
    // of any share is rethrown once all have ended
    std::mutex mu;
    std::exception_ptr err;
    auto share = [&](size_t u) {
        try {
            f(u);
        } catch (...) {
            std::lock_guard<std::mutex> lk(mu);
            if (!err) err = std::current_exception();
        }
    };
    std::vector<std::thread> th;
    size_t t = 1;
    try {
        for (; t < T; t++) th.emplace_back(share, t);
    } catch (...) {
    }
    for (size_t u = t; u < T; u++) share(u);
    share(0);
    for (auto& x : th) x.join();
    if (err) std::rethrow_exception(err);
}

// Host threads for n items: one per 65,536, at most 8 and the hardware's.
inline size_t host_threads(uint64_t n) {
    const unsigned hw = std::thread::hardware_concurrency();
    return std::max<size_t>(1, std::min<size_t>({static_cast<size_t>(hw ? hw : 1), 8, static_cast<size_t>(n / 65536)}));
}

// Boundaries of T ranges over [0, n) that never separate item i from item
// i-1 when same(i) holds (so a group of equal items stays in one range).
template <typename Same>
inline std::vector<size_t> group_cuts(size_t n, size_t T, Same same) {
    std::vector<size_t> cut(T + 1, n);
    cut[0] = 0;
    for (size_t t = 1; t < T; t++) {
        size_t p = std::max(n * t / T, cut[t - 1]);
        while (p > 0 && p < n && same(p)) p++;
        cut[t] = p;
    }
    return cut;
}

// Stable LSD radix sort of (key, val) pairs on the low `bits` bits of key.
// Large inputs are split over host threads: per pass, every thread counts
// the digits of its share, one prefix over (digit, thread) places them, and
// every thread scatters its share (so equal digits keep their order).
// k2 and v2 are buffers of the caller (resized to n; their contents are
// lost).
inline void host_radix_sort(std::vector<uint64_t>& key, std::vector<uint32_t>& val, int bits,
                            std::vector<uint64_t>& k2, std::vector<uint32_t>& v2, HostPool* pool = nullptr) {
    constexpr int kDigit = 11;
    constexpr uint32_t kBuckets = 1u << kDigit;
    const size_t n = key.size();
    if (n < 2) return;
    const size_t T = host_threads(n);
    k2.resize(n);
    v2.resize(n);
    std::vector<uint32_t> cnt(kBuckets * T);
    auto par = [&](auto f) { host_parallel(T, f, pool); };
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
    // the host threads of the parallel passes (the process's pool, started
    // by the first batch large enough to split)
    HostPool* const pool = host_threads(n_ops) > 1 ? &shared_host_pool() : nullptr;
    auto par = [pool](size_t T, auto f) { host_parallel(T, f, pool); };
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
        const size_t TV = host_threads(n_ops);
        std::vector<std::vector<uint64_t>> found(TV);
        par(TV, [&](size_t t) {
            // appends go to a vector of the thread's own (the headers in
            // `found` share cache lines)
            std::vector<uint64_t> f;
            for (uint64_t i = n_ops * t / TV, e = n_ops * (t + 1) / TV; i < e; i++)
                if (ops[i].op < BSIM_OP_ADD_E || ops[i].op > BSIM_OP_DEL_E) f.push_back(i);
            found[t].swap(f);
        });
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
    const size_t T = host_threads(end);
    std::vector<std::vector<Rec>>& part = rs.part;
    if (part.size() < T) part.resize(T);
    std::vector<Fail> efail(T);
    std::vector<uint32_t> part_max(T, 0);
    auto check_edges = [&](size_t t) {
        const uint64_t a = end * t / T, b = end * (t + 1) / T;
        // the thread appends to a vector object of its own, holding part[t]'s
        // storage (the headers in `part` share cache lines)
        std::vector<Rec> out;
        out.swap(part[t]);
        struct Back {
            std::vector<Rec>& a;
            std::vector<Rec>& b;
            ~Back() { a.swap(b); }
        } back{out, part[t]};
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
    par(T, check_edges);
    Fail first = vfail;
    for (const Fail& f : efail)
        if (f.pos < first.pos) first = f;
    if (first.pos != UINT64_MAX) throw DeviceError{first.status, first.msg};
    // the edge records stay in the threads' parts: part[t] holds records
    // roff[t] .. roff[t+1] of the batch, in operation order
    std::vector<size_t> roff(T + 1, 0);
    for (size_t t = 0; t < T; t++) {
        roff[t + 1] = roff[t] + part[t].size();
        max_l = std::max(max_l, part_max[t]);
    }
    hb.n_new = n_cur;
    {
        // the touched vertices in id order (radix: a comparison sort of
        // 10^5 ids costs milliseconds); rs.key/val are free until the edge
        // records' keys
        std::vector<uint64_t>& tk = rs.key;
        std::vector<uint32_t>& tv = rs.val;
        tk.assign(touched.begin(), touched.end());
        tv.resize(touched.size());
        host_radix_sort(tk, tv, std::max(1, bit_width(n_cur)), rs.key2, rs.val2, pool);
        hb.tl.assign(tk.begin(), tk.end());
    }
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
    // ... and a 64 KiB filter of them (bit v mod 2^19) that stays in cache:
    // the emit pass asks for both ends of every change, and most answers
    // are "no" from the filter alone
    std::vector<uint64_t>& dbits = rs.dbits;
    std::vector<uint64_t>& dfilt = rs.dfilt;
    constexpr uint32_t kFiltMask = (1u << 19) - 1;
    const bool any_dead = !hb.dead.empty();
    if (any_dead) {
        dbits.assign((static_cast<size_t>(n_cur) + 63) / 64, 0);
        dfilt.assign((kFiltMask + 1) / 64, 0);
        for (uint32_t v : hb.dead) {
            dbits[v >> 6] |= 1ull << (v & 63);
            dfilt[(v & kFiltMask) >> 6] |= 1ull << (v & 63);
        }
    }
    auto dead_at_end = [&](uint32_t v) {
        return any_dead && ((dfilt[(v & kFiltMask) >> 6] >> (v & 63)) & 1) && ((dbits[v >> 6] >> (v & 63)) & 1);
    };
    // edge records in (u, w, l) order, input order within equal triples:
    // the triple packed in one key when it fits 64 bits (the add flag rides
    // in the value), else a comparison sort
    const int bv = std::max(1, bit_width(n_cur)), bl = std::max(1, bit_width(max_l + 1));
    const size_t nr = roff[T];
    std::vector<uint64_t>& key = rs.key;
    std::vector<uint32_t>& val = rs.val;
    key.clear();
    val.resize(nr);
    // The changes, one per distinct triple, in (u, w, l) order: deleted if
    // any of its records removes it, present if its last record adds it;
    // triples with an endpoint that ends deleted are dropped (the device
    // removes all their edges).  Several threads each take a range of
    // sources and fill a part of their own (with the source groups and the
    // reverse additions); the parts are then joined in order.
    std::vector<ResolveScratch::Part>& parts = rs.parts;
    auto join_parts = [&](size_t TP) {
        std::vector<size_t> co(TP + 1, 0), ro(TP + 1, 0), go(TP + 1, 0);
        for (size_t t = 0; t < TP; t++) {
            co[t + 1] = co[t] + parts[t].cu.size();
            ro[t + 1] = ro[t] + parts[t].rw.size();
            go[t + 1] = go[t] + parts[t].gsrc.size();
            hb.n_present += parts[t].n_present;
            hb.max_label = std::max(hb.max_label, parts[t].max_label);
        }
        for (std::vector<uint32_t>* v : {&hb.cu, &hb.cw, &hb.cl, &hb.cf}) v->resize(co[TP]);
        for (std::vector<uint32_t>* v : {&hb.rw, &hb.ru}) v->resize(ro[TP]);
        for (std::vector<uint32_t>* v : {&hb.gsrc, &hb.gbeg, &hb.gend}) v->resize(go[TP]);
        par(TP, [&](size_t t) {
            const ResolveScratch::Part& P = parts[t];
            std::copy(P.cu.begin(), P.cu.end(), hb.cu.begin() + co[t]);
            std::copy(P.cw.begin(), P.cw.end(), hb.cw.begin() + co[t]);
            std::copy(P.cl.begin(), P.cl.end(), hb.cl.begin() + co[t]);
            std::copy(P.cf.begin(), P.cf.end(), hb.cf.begin() + co[t]);
            std::copy(P.rw.begin(), P.rw.end(), hb.rw.begin() + ro[t]);
            std::copy(P.ru.begin(), P.ru.end(), hb.ru.begin() + ro[t]);
            std::copy(P.gsrc.begin(), P.gsrc.end(), hb.gsrc.begin() + go[t]);
            const size_t ng = P.gsrc.size();
            for (size_t g = 0; g < ng; g++) {
                hb.gbeg[go[t] + g] = static_cast<uint32_t>(co[t] + P.gbeg[g]);
                hb.gend[go[t] + g] = static_cast<uint32_t>(co[t] + (g + 1 < ng ? P.gbeg[g + 1] : P.cu.size()));
            }
        });
    };
    // trip(i): the (u, w, l) of sorted record i; adds(i): whether it adds
    auto emit_all = [&](auto trip, auto adds) {
        const size_t TP = host_threads(nr);
        if (parts.size() < TP) parts.resize(TP);
        const std::vector<size_t> cut = group_cuts(nr, TP, [&](size_t i) { return trip(i)[0] == trip(i - 1)[0]; });
        par(TP, [&](size_t t) {
            // a Part object of the thread's own, holding parts[t]'s storage
            // (the Parts' headers share cache lines)
            ResolveScratch::Part P;
            std::swap(P, parts[t]);
            for (std::vector<uint32_t>* v : {&P.cu, &P.cw, &P.cl, &P.cf, &P.rw, &P.ru, &P.gsrc, &P.gbeg}) v->clear();
            P.n_present = 0;
            P.max_label = 0;
            for (size_t i = cut[t], e = cut[t + 1]; i < e;) {
                const auto x = trip(i);
                size_t j = i;
                bool deleted = false;
                while (j < e && trip(j) == x) deleted |= !adds(j++);
                const bool add = adds(j - 1);
                i = j;
                if (dead_at_end(x[0]) || dead_at_end(x[1])) continue;
                if (P.gsrc.empty() || P.gsrc.back() != x[0]) {
                    P.gsrc.push_back(x[0]);
                    P.gbeg.push_back(static_cast<uint32_t>(P.cu.size()));
                }
                P.cu.push_back(x[0]);
                P.cw.push_back(x[1]);
                P.cl.push_back(x[2]);
                P.cf.push_back((deleted ? kChgDeleted : 0u) | (add ? kChgPresent : 0u));
                if (add) {
                    P.n_present++;
                    P.max_label = std::max(P.max_label, x[2]);
                    P.rw.push_back(x[1]);
                    P.ru.push_back(x[0]);
                }
            }
            std::swap(P, parts[t]);
        });
        join_parts(TP);
    };
    using Trip = std::array<uint32_t, 3>;
    if (2 * bv + bl <= 64) {
        key.resize(nr);
        par(T, [&](size_t t) {
            const std::vector<Rec>& q = part[t];
            for (size_t i = 0, o = roff[t]; i < q.size(); i++, o++) {
                key[o] = (static_cast<uint64_t>(q[i].u) << (bv + bl)) | (static_cast<uint64_t>(q[i].w) << bl) | q[i].l;
                val[o] = q[i].add;
            }
        });
        host_radix_sort(key, val, 2 * bv + bl, rs.key2, rs.val2, pool);
        const uint64_t lmask = (1ull << bl) - 1, wmask = (1ull << bv) - 1;
        emit_all(
            [&](size_t i) {
                return Trip{static_cast<uint32_t>(key[i] >> (bv + bl)), static_cast<uint32_t>((key[i] >> bl) & wmask),
                            static_cast<uint32_t>(key[i] & lmask)};
            },
            [&](size_t i) { return val[i] != 0; });
    } else {
        recs.reserve(nr);
        for (size_t t = 0; t < T; t++) recs.insert(recs.end(), part[t].begin(), part[t].end());
        for (size_t i = 0; i < nr; i++) val[i] = static_cast<uint32_t>(i);
        std::stable_sort(val.begin(), val.end(), [&](uint32_t a, uint32_t b) {
            const Rec &x = recs[a], &y = recs[b];
            if (x.u != y.u) return x.u < y.u;
            if (x.w != y.w) return x.w < y.w;
            return x.l < y.l;
        });
        emit_all([&](size_t i) { return Trip{recs[val[i]].u, recs[val[i]].w, recs[val[i]].l}; },
                 [&](size_t i) { return recs[val[i]].add != 0; });
    }
    // reverse additions, sorted by (w, u) without duplicates and grouped by
    // target: sorted on one thread pool, then de-duplicated and grouped per
    // range of targets
    std::vector<uint64_t>& rk = rs.key;  // the edge records' keys are done with
    std::vector<uint32_t>& rdummy = rs.val;
    const size_t nrv = hb.rw.size();
    rk.resize(nrv);
    rdummy.resize(nrv);
    for (size_t i = 0; i < nrv; i++) rk[i] = (static_cast<uint64_t>(hb.rw[i]) << bv) | hb.ru[i];
    host_radix_sort(rk, rdummy, 2 * bv, rs.key2, rs.val2, pool);
    {
        const uint64_t umask = (1ull << bv) - 1;
        const size_t TP = host_threads(nrv);
        if (parts.size() < TP) parts.resize(TP);
        const std::vector<size_t> cut = group_cuts(nrv, TP, [&](size_t i) { return (rk[i] >> bv) == (rk[i - 1] >> bv); });
        par(TP, [&](size_t t) {
            ResolveScratch::Part P;  // rw, ru, gsrc (targets) and gbeg; parts[t]'s storage
            std::swap(P, parts[t]);
            for (std::vector<uint32_t>* v : {&P.rw, &P.ru, &P.gsrc, &P.gbeg}) v->clear();
            for (size_t i = cut[t], e = cut[t + 1]; i < e; i++) {
                if (i > cut[t] && rk[i] == rk[i - 1]) continue;
                const uint32_t w = static_cast<uint32_t>(rk[i] >> bv);
                if (P.gsrc.empty() || P.gsrc.back() != w) {
                    P.gsrc.push_back(w);
                    P.gbeg.push_back(static_cast<uint32_t>(P.rw.size()));
                }
                P.rw.push_back(w);
                P.ru.push_back(static_cast<uint32_t>(rk[i] & umask));
            }
            std::swap(P, parts[t]);
        });
        std::vector<size_t> ro(TP + 1, 0), go(TP + 1, 0);
        for (size_t t = 0; t < TP; t++) {
            ro[t + 1] = ro[t] + parts[t].rw.size();
            go[t + 1] = go[t] + parts[t].gsrc.size();
        }
        for (std::vector<uint32_t>* v : {&hb.rw, &hb.ru}) v->resize(ro[TP]);
        for (std::vector<uint32_t>* v : {&hb.rgw, &hb.rgbeg, &hb.rgend}) v->resize(go[TP]);
        par(TP, [&](size_t t) {
            const ResolveScratch::Part& P = parts[t];
            std::copy(P.rw.begin(), P.rw.end(), hb.rw.begin() + ro[t]);
            std::copy(P.ru.begin(), P.ru.end(), hb.ru.begin() + ro[t]);
            std::copy(P.gsrc.begin(), P.gsrc.end(), hb.rgw.begin() + go[t]);
            const size_t ng = P.gsrc.size();
            for (size_t g = 0; g < ng; g++) {
                hb.rgbeg[go[t] + g] = static_cast<uint32_t>(ro[t] + P.gbeg[g]);
                hb.rgend[go[t] + g] = static_cast<uint32_t>(ro[t] + (g + 1 < ng ? P.gbeg[g + 1] : P.rw.size()));
            }
        });
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
