// Sanitizer driver for the host-side resolution of update batches
// (csrc/bsim_resolve.h), built by tests/test_sanitizers.py with
// -fsanitize=address,undefined and run on the CPU.
//
// Seeded random batches -- valid ones and ones with an invalid operation
// somewhere -- go through resolve_ops and through a plain sequential model
// of the operations as bsim_apply_updates documents them (ADD_E adds a
// triple unless present, DEL_E removes every copy, MOD_E is DEL_E then
// ADD_E with the new label, DEL_V removes the vertex and every incident
// edge; an operation naming an id not yet created is BSIM_E_RANGE, one
// naming a deleted vertex BSIM_E_INVALID, ...).  Checked:
//   - an invalid batch throws the status of its first invalid operation;
//   - for a valid one, the triple multiplicities that the net change gives
//     (applied to the base graph as the device update applies it) equal the
//     model's, the new vertex count, deleted vertices and final type sets
//     agree, and the derived lists (per-source ranges, reverse additions)
//     are sorted and consistent;
//   - the scratch marks are all zero after every call, thrown or not.
// Batches on a base graph of 1.2M vertices with labels up to 2^24 - 1 take
// the comparison-sort path (the triple does not fit 64 bits).
// Prints "ok <batches>" and exits 0, or the failed check and exits 1.
#include <cstdio>
#include <cstdlib>
#include <map>
#include <set>
#include <tuple>
#include <vector>

#include "bsim_resolve.h"

using bsim::DeviceError;
using bsim::HostBatch;
using bsim::ResolveScratch;

namespace {

uint64_t g_rng = 0x2545F4914F6CDD1Dull;
uint32_t rnd(uint32_t bound) {
    g_rng ^= g_rng << 13;
    g_rng ^= g_rng >> 7;
    g_rng ^= g_rng << 17;
    return bound ? static_cast<uint32_t>(g_rng % bound) : 0u;
}

int g_batch = 0;
#define CHECK(cond, what)                                                                  \
    do {                                                                                   \
        if (!(cond)) {                                                                     \
            std::printf("FAIL batch %d: %s (line %d)\n", g_batch, what, __LINE__);         \
            std::exit(1);                                                                  \
        }                                                                                  \
    } while (0)

using Triple = std::tuple<uint32_t, uint32_t, uint32_t>;  // (u, l, w)

struct Base {
    uint32_t n;
    uint32_t label_bytes;
    std::vector<uint8_t> alive;
    std::map<Triple, uint32_t> edges;  // multiplicities (copies of a triple may repeat)
};

// The sequential semantics; returns 0 or the status of the first invalid op.
struct Model {
    uint32_t n;
    std::vector<uint8_t> alive;
    std::map<Triple, uint32_t> cnt;
    std::set<Triple> touched;
    std::map<uint32_t, std::vector<uint32_t>> types;  // final type sets of vertices with a vertex op
    std::set<uint32_t> deleted;

    int run(const Base& b, const std::vector<bsim_update>& ops) {
        n = b.n;
        alive = b.alive;
        cnt = b.edges;
        const uint64_t lab_lim = b.label_bytes == 2 ? (1ull << 16) : (1ull << 24);
        for (const bsim_update& o : ops) {
            const bool edge = o.op == BSIM_OP_ADD_E || o.op == BSIM_OP_DEL_E || o.op == BSIM_OP_MOD_E;
            if (o.op == BSIM_OP_MOD_V || o.op == BSIM_OP_DEL_V || edge) {
                if (o.u >= n || (edge && o.w >= n)) return BSIM_E_RANGE;
                if (!alive[o.u] || (edge && !alive[o.w])) return BSIM_E_INVALID;
            }
            if (o.op == BSIM_OP_ADD_V || o.op == BSIM_OP_MOD_V) {
                if (o.n_types > bsim::kMaxStateTypes) return BSIM_E_UNSUPPORTED;
                if (o.n_types && !o.types) return BSIM_E_INVALID;
            }
            if (edge && (o.label >= lab_lim || (o.op == BSIM_OP_MOD_E && o.new_label >= lab_lim)))
                return BSIM_E_RANGE;
            switch (o.op) {
                case BSIM_OP_ADD_V:
                    types[n] = std::vector<uint32_t>(o.types, o.types + o.n_types);
                    alive.push_back(1);
                    n++;
                    break;
                case BSIM_OP_MOD_V:
                    types[o.u] = std::vector<uint32_t>(o.types, o.types + o.n_types);
                    break;
                case BSIM_OP_DEL_V:
                    alive[o.u] = 0;
                    deleted.insert(o.u);
                    types.erase(o.u);
                    for (auto& kv : cnt)
                        if (std::get<0>(kv.first) == o.u || std::get<2>(kv.first) == o.u) kv.second = 0;
                    break;
                case BSIM_OP_ADD_E: {
                    const Triple t{o.u, o.label, o.w};
                    touched.insert(t);
                    if (cnt[t] == 0) cnt[t] = 1;
                    break;
                }
                case BSIM_OP_DEL_E: {
                    const Triple t{o.u, o.label, o.w};
                    touched.insert(t);
                    cnt[t] = 0;
                    break;
                }
                case BSIM_OP_MOD_E: {
                    const Triple t{o.u, o.label, o.w}, t2{o.u, o.new_label, o.w};
                    touched.insert(t);
                    touched.insert(t2);
                    cnt[t] = 0;
                    if (cnt[t2] == 0) cnt[t2] = 1;
                    break;
                }
                default:
                    return BSIM_E_INVALID;
            }
        }
        return 0;
    }
};

Base make_base(uint32_t n, uint32_t m, uint32_t label_bytes, uint32_t max_label) {
    Base b;
    b.n = n;
    b.label_bytes = label_bytes;
    b.alive.assign(n, 1);
    for (uint32_t v = 0; v < n; v++)
        if (rnd(10) == 0) b.alive[v] = 0;
    for (uint32_t i = 0; i < m; i++) {
        const uint32_t u = rnd(n), w = rnd(n);
        if (!b.alive[u] || !b.alive[w]) continue;
        b.edges[Triple{u, rnd(max_label + 1), w}] += 1 + (rnd(8) == 0);
    }
    return b;
}

// A random batch; with `invalid`, one operation somewhere is made invalid.
std::vector<bsim_update> make_batch(const Base& b, uint32_t n_ops, uint32_t max_label, bool invalid,
                                    std::vector<std::vector<uint32_t>>& type_pool) {
    std::vector<bsim_update> ops;
    std::vector<uint8_t> alive = b.alive;
    uint32_t n = b.n;
    std::vector<Triple> known;
    for (const auto& kv : b.edges) known.push_back(kv.first);
    auto pick_alive = [&]() -> uint32_t {
        for (int t = 0; t < 64; t++) {
            const uint32_t v = rnd(n);
            if (alive[v]) return v;
        }
        return UINT32_MAX;
    };
    const uint32_t bad_at = invalid ? rnd(n_ops) : UINT32_MAX;
    for (uint32_t i = 0; i < n_ops; i++) {
        bsim_update o{};
        const uint32_t kind = rnd(100);
        if (kind < 6) {
            o.op = BSIM_OP_ADD_V;
            type_pool.emplace_back();
            for (uint32_t j = rnd(4); j > 0; j--) type_pool.back().push_back(rnd(50));
            o.n_types = static_cast<uint32_t>(type_pool.back().size());
            o.types = type_pool.back().data();
            alive.push_back(1);
            n++;
        } else if (kind < 12) {
            o.op = BSIM_OP_MOD_V;
            o.u = pick_alive();
            if (o.u == UINT32_MAX) continue;
            type_pool.emplace_back();
            for (uint32_t j = rnd(4); j > 0; j--) type_pool.back().push_back(rnd(50));
            o.n_types = static_cast<uint32_t>(type_pool.back().size());
            o.types = type_pool.back().data();
        } else if (kind < 15) {
            o.op = BSIM_OP_DEL_V;
            o.u = pick_alive();
            if (o.u == UINT32_MAX) continue;
            alive[o.u] = 0;
        } else {
            const uint32_t e = rnd(3);
            o.op = e == 0 ? BSIM_OP_ADD_E : e == 1 ? BSIM_OP_DEL_E : BSIM_OP_MOD_E;
            if (!known.empty() && rnd(2)) {
                // an existing or earlier triple
                const Triple t = known[rnd(static_cast<uint32_t>(known.size()))];
                o.u = std::get<0>(t);
                o.label = std::get<1>(t);
                o.w = std::get<2>(t);
                if (!alive[o.u] || !alive[o.w]) continue;
            } else {
                o.u = pick_alive();
                o.w = pick_alive();
                if (o.u == UINT32_MAX || o.w == UINT32_MAX) continue;
                o.label = rnd(max_label + 1);
            }
            o.new_label = rnd(max_label + 1);
            known.push_back(Triple{o.u, o.label, o.w});
        }
        if (i == bad_at) {
            switch (rnd(6)) {
                case 0:  // an id not yet created
                    o.op = BSIM_OP_ADD_E;
                    o.u = n + rnd(3);
                    break;
                case 1:  // a deleted vertex (or, if none, an unknown op code)
                    o.op = BSIM_OP_DEL_E;
                    o.u = UINT32_MAX;
                    for (uint32_t v = 0; v < n; v++)
                        if (!alive[v]) {
                            o.u = v;
                            break;
                        }
                    if (o.u == UINT32_MAX) o.op = 99;
                    o.w = 0;
                    break;
                case 2:  // a label out of range
                    o.op = BSIM_OP_MOD_E;
                    o.new_label = b.label_bytes == 2 ? 70000u : (1u << 24);
                    break;
                case 3:  // too many types
                    o.op = BSIM_OP_ADD_V;
                    o.n_types = bsim::kMaxStateTypes + 1;
                    type_pool.emplace_back(o.n_types, 1u);
                    o.types = type_pool.back().data();
                    break;
                case 4:  // types missing
                    o.op = BSIM_OP_ADD_V;
                    o.n_types = 2;
                    o.types = nullptr;
                    break;
                default:
                    o.op = 0;  // unknown op code
            }
        }
        ops.push_back(o);
    }
    return ops;
}

void check_scratch_clear(const ResolveScratch& rs) {
    for (uint8_t x : rs.vmark) CHECK(x == 0, "scratch marks clear");
    for (uint32_t x : rs.vtype) CHECK(x == 0, "scratch type indices clear");
}

void check_batch(const Base& b, const std::vector<bsim_update>& ops, ResolveScratch& rs) {
    g_batch++;
    Model model;
    const int want = model.run(b, ops);
    HostBatch hb;
    int got = 0;
    try {
        hb = bsim::resolve_ops(b.n, b.label_bytes, b.alive, rs, ops.data(), ops.size());
    } catch (const DeviceError& e) {
        got = e.status;
    }
    check_scratch_clear(rs);
    CHECK(got == want, "status of the batch");
    if (want) return;
    CHECK(hb.n_new == model.n, "new vertex count");
    // vertices with a vertex op: sorted, final types, deletions
    std::set<uint32_t> tl_want;
    for (const auto& kv : model.types) tl_want.insert(kv.first);
    for (uint32_t v : model.deleted) tl_want.insert(v);
    CHECK(hb.tl.size() == tl_want.size() && hb.tl_off.size() == hb.tl.size() + 1, "touched vertex list");
    size_t i = 0;
    for (uint32_t v : tl_want) {
        CHECK(hb.tl[i] == v, "touched vertices sorted");
        const std::vector<uint32_t> got_t(hb.tl_ids.begin() + hb.tl_off[i], hb.tl_ids.begin() + hb.tl_off[i + 1]);
        if (model.deleted.count(v))
            CHECK(got_t.empty(), "a deleted vertex has no types");
        else
            CHECK(got_t == model.types[v], "final type set");
        i++;
    }
    CHECK(std::vector<uint32_t>(model.deleted.begin(), model.deleted.end()) == hb.dead, "deleted vertices");
    // changed triples: sorted by (u, w, l), distinct, none with a dead end
    std::set<Triple> emitted;
    uint64_t present = 0;
    uint32_t max_label = 0;
    std::set<std::pair<uint32_t, uint32_t>> rev_want;
    for (size_t c = 0; c < hb.cu.size(); c++) {
        const Triple t{hb.cu[c], hb.cl[c], hb.cw[c]};
        if (c) {
            const auto a = std::make_tuple(hb.cu[c - 1], hb.cw[c - 1], hb.cl[c - 1]);
            CHECK(a < std::make_tuple(hb.cu[c], hb.cw[c], hb.cl[c]), "changes sorted by (u, w, l) and distinct");
        }
        CHECK(model.alive[hb.cu[c]] && model.alive[hb.cw[c]], "no change of an edge with a dead end");
        CHECK(model.touched.count(t), "only touched triples change");
        emitted.insert(t);
        const bool del = hb.cf[c] & bsim::kChgDeleted, pres = hb.cf[c] & bsim::kChgPresent;
        CHECK(del || pres, "a change deletes or ends present");
        const auto it = b.edges.find(t);
        const uint32_t c0 = it == b.edges.end() ? 0u : it->second;
        const uint32_t fin = pres ? (del ? 1u : std::max(c0, 1u)) : (del ? 0u : c0);
        CHECK(fin == model.cnt[t], "final multiplicity");
        if (pres) {
            present++;
            max_label = std::max(max_label, std::get<1>(t));
            rev_want.insert({hb.cw[c], hb.cu[c]});
        }
    }
    for (const Triple& t : model.touched)
        if (model.alive[std::get<0>(t)] && model.alive[std::get<2>(t)])
            CHECK(emitted.count(t), "every touched triple of live vertices changes");
    CHECK(hb.n_present == present && hb.max_label == max_label, "present count and largest label");
    // per-source ranges
    CHECK(hb.gsrc.size() == hb.gbeg.size() && hb.gbeg.size() == hb.gend.size(), "source ranges");
    size_t pos = 0;
    for (size_t g = 0; g < hb.gsrc.size(); g++) {
        CHECK(hb.gbeg[g] == pos && hb.gend[g] > hb.gbeg[g], "source ranges tile the changes");
        for (uint32_t c = hb.gbeg[g]; c < hb.gend[g]; c++) CHECK(hb.cu[c] == hb.gsrc[g], "source range owner");
        pos = hb.gend[g];
    }
    CHECK(pos == hb.cu.size(), "source ranges cover the changes");
    // reverse additions: the distinct (w, u) of present triples, sorted
    CHECK(hb.rw.size() == rev_want.size() && hb.ru.size() == rev_want.size(), "reverse additions");
    i = 0;
    for (const auto& p : rev_want) {
        CHECK(hb.rw[i] == p.first && hb.ru[i] == p.second, "reverse additions sorted and distinct");
        i++;
    }
    pos = 0;
    for (size_t g = 0; g < hb.rgw.size(); g++) {
        CHECK(hb.rgbeg[g] == pos && hb.rgend[g] > hb.rgbeg[g], "reverse ranges tile");
        for (uint32_t c = hb.rgbeg[g]; c < hb.rgend[g]; c++) CHECK(hb.rw[c] == hb.rgw[g], "reverse range owner");
        pos = hb.rgend[g];
    }
    CHECK(pos == hb.rw.size(), "reverse ranges cover the additions");
}

}  // namespace

int main(int argc, char** argv) {
    if (argc > 1) g_rng = std::strtoull(argv[1], nullptr, 10) | 1u;
    // small bases, both label widths, valid and invalid batches, one scratch
    // reused across calls as a state reuses its own
    for (int round = 0; round < 40; round++) {
        const uint32_t label_bytes = round % 2 ? 2u : 4u;
        const uint32_t max_label = round % 3 == 0 ? 3u : (label_bytes == 2 ? 65535u : (1u << 24) - 1);
        const uint32_t n = 1 + rnd(round < 30 ? 60 : 3000);
        const Base b = make_base(n, 4 * n, label_bytes, max_label);
        ResolveScratch rs;
        rs.vmark.assign(n, 0);
        rs.vtype.assign(n, 0);
        for (int k = 0; k < 12; k++) {
            std::vector<std::vector<uint32_t>> pool;
            pool.reserve(8192);
            const auto ops = make_batch(b, 1 + rnd(k < 6 ? 40 : 1500), max_label, k % 3 == 2, pool);
            check_batch(b, ops, rs);
        }
    }
    // a large base with wide labels: the triple no longer fits one 64-bit key
    {
        const Base b = make_base(1200000, 20000, 4, (1u << 24) - 1);
        ResolveScratch rs;
        rs.vmark.assign(b.n, 0);
        rs.vtype.assign(b.n, 0);
        for (int k = 0; k < 6; k++) {
            std::vector<std::vector<uint32_t>> pool;
            pool.reserve(8192);
            const auto ops = make_batch(b, 200 + rnd(2000), (1u << 24) - 1, k % 3 == 2, pool);
            check_batch(b, ops, rs);
        }
    }
    // edge batches large enough for the threaded radix sort (over 2^17
    // records; no vertex deletions, which the model handles in O(edges))
    {
        const Base b = make_base(50000, 100000, 2, 65535);
        ResolveScratch rs;
        rs.vmark.assign(b.n, 0);
        rs.vtype.assign(b.n, 0);
        std::vector<Triple> known;
        for (const auto& kv : b.edges) known.push_back(kv.first);
        auto alive_vertex = [&]() {
            for (;;) {
                const uint32_t v = rnd(b.n);
                if (b.alive[v]) return v;
            }
        };
        for (int k = 0; k < 2; k++) {
            std::vector<bsim_update> ops(150000 + rnd(50000));
            for (bsim_update& o : ops) {
                o = bsim_update{};
                const uint32_t x = rnd(100);
                if (x < 60) {
                    o.op = BSIM_OP_ADD_E;
                    o.u = alive_vertex();
                    o.w = rnd(4) ? alive_vertex() : o.u;
                    o.label = rnd(65536);
                } else {
                    const Triple t = known[rnd(static_cast<uint32_t>(known.size()))];
                    o.op = x < 85 ? BSIM_OP_MOD_E : BSIM_OP_DEL_E;
                    o.u = std::get<0>(t);
                    o.label = std::get<1>(t);
                    o.w = std::get<2>(t);
                    o.new_label = rnd(65536);
                }
            }
            check_batch(b, ops, rs);
        }
    }
    std::printf("ok %d\n", g_batch);
    return 0;
}
