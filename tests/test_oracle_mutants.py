"""Planted mistakes in a copy of the oracle must be caught by the pins.

Each case edits one line of a temporary copy of the C oracle (a dropped term,
a wrong operand, a wrong index, an off-by-one), compiles it with gcc, swaps it
in for the real oracle, and checks that the pin checks fail.  This runs on the
CPU only and never touches the real oracle library.
"""

import subprocess

import numpy as np
import pytest

from oracle import exact
from oracle import oracle as orc
from paper_2111_12493_amd import graphgen as gg

MUTANTS = {
    "drop_label_from_key": ("keys[i] = h_prev[tgt[i]] ^ bo_label_salt(lab[i]);",
                            "keys[i] = h_prev[tgt[i]];"),
    "no_key_dedupe": ("size_t u = unique_u64(keys, (size_t)deg);",
                      "size_t u = (size_t)deg; qsort(keys, u, 8, cmp_u64);"),
    "wrong_gather_index": ("keys[i] = h_prev[tgt[i]] ^ bo_label_salt(lab[i]);",
                           "keys[i] = h_prev[tgt[0]] ^ bo_label_salt(lab[i]);"),
    "no_type_dedupe": ("size_t u = unique_u32(tmp, n_types);",
                       "size_t u = n_types;"),
    "fixpoint_off_by_one": ("if (blocks_per_iter[k] == blocks_per_iter[k - 1]) {",
                            "if (k > 1 && blocks_per_iter[k - 1] == blocks_per_iter[k - 2]) {"),
    "hash_classes_not_grouped": ("uint32_t m = same ? minv[p[i - 1].v] : p[i].v;",
                                 "uint32_t m = p[i].v;"),
    "previous_class_ignored": ("int same = i > 0 && p[i].c == p[i - 1].c && p[i].h == p[i - 1].h;",
                               "int same = i > 0 && p[i].h == p[i - 1].h;"),
    "blocks_numbered_by_largest_vertex": ("for (uint32_t v = 0; v < n; v++)\n        if (is_min[v]) rank[v] = nb++;",
                                          "for (uint32_t v = n; v-- > 0;)\n        if (is_min[v]) rank[v] = nb++;"),
    "summary_edge_transposed": ("tr[ne].d = dst_ids[tgt[e]];",
                                "tr[ne].d = dst_ids[v]; tr[ne].s = block_ids[tgt[e]];"),
    "prev_level_edges_use_final_classes": (
        "const uint32_t* dst_ids = ((flags & BO_PREV_LEVEL_EDGES) && k_done >= 1) ? ncls : block_ids;",
        "const uint32_t* dst_ids = block_ids;"),
    # value-only mistakes: a valid set hash, the same partitions, other hash
    # values; the frozen hash-spec vectors catch them
    "drop_own_type": ("return bo_mix(t_v ^ bo_mix(cs + sum));",
                      "return bo_mix(bo_mix(cs + sum));"),
    "sum_replaced_by_xor": ("for (size_t i = 0; i < u; i++) sum += bo_mix(keys[i] ^ ce);",
                            "for (size_t i = 0; i < u; i++) sum ^= bo_mix(keys[i] ^ ce);"),
    "type_term_unmixed": ("for (size_t i = 0; i < u; i++) sum += bo_mix(ct ^ (uint64_t)tmp[i]);",
                          "for (size_t i = 0; i < u; i++) sum += ct ^ (uint64_t)tmp[i];"),
    "salt_domain_constant_dropped": ("uint64_t bo_label_salt(uint32_t label) { return bo_mix(bo_const_l() + (uint64_t)label); }",
                                     "uint64_t bo_label_salt(uint32_t label) { return bo_mix((uint64_t)label); }"),
    "signature_domain_constant_dropped": ("return bo_mix(t_v ^ bo_mix(cs + sum));",
                                          "return bo_mix(t_v ^ bo_mix(sum));"),
}

def _hash_vectors_hold() -> bool:
    """The frozen hash-spec vectors (HASH_SPEC.md) on the worked graph."""
    import hash_vectors

    v = hash_vectors.load()
    if orc.type_hash([0, 1]) != v["t({0,1})"] or orc.type_hash([3]) != v["t({3})"]:
        return False
    if orc.label_salt(5) != v["salt(5)"]:
        return False
    r = orc.summarize(hash_vectors.graph(v), 2, False)
    return [int(x) for x in r["hashes"]] == v["h2"] and [int(x) for x in r["prev_hashes"]] == v["h1"]


def _pins_hold() -> bool:
    """A compact selection of the pin checks; False as soon as one fails."""
    try:
        if not _hash_vectors_hold():
            return False
        g = gg.paper_example()
        r = orc.summarize(g, 2, False, True)
        if list(r["block_ids"]) != [0, 1, 2, 2] or list(r["blocks_per_iter"]) != [1, 3, 3]:
            return False
        rows = [(0, 0, 1), (0, 1, 2), (1, 2, 2)]
        if list(zip(r["se_src"].tolist(), r["se_label"].tolist(), r["se_dst"].tolist())) != rows:
            return False
        for L in (1, 5):
            r = orc.summarize(gg.chain(L), L + 5, True, True)
            if r["k_done"] != L + 1:
                return False
        # previous-level edges of a chain of 6 edges at k = 3 (closed form:
        # (j, 0, j) for j < k), and at k = 0 the quotient edges
        r = orc.summarize(gg.chain(6), 3, False, True, prev_level_edges=True)
        if list(zip(r["se_src"].tolist(), r["se_label"].tolist(), r["se_dst"].tolist())) != \
                [(0, 0, 0), (1, 0, 1), (2, 0, 2)]:
            return False
        r = orc.summarize(gg.chain(6), 0, False, True, prev_level_edges=True)
        if list(zip(r["se_src"].tolist(), r["se_label"].tolist(), r["se_dst"].tolist())) != [(0, 0, 0)]:
            return False
        rng = np.random.default_rng(21)
        for trial in range(60):
            n = int(rng.integers(2, 30))
            g = gg.random_small_graph(rng, n, int(rng.integers(0, 4 * n)), 3, 3, 3)
            r = orc.summarize(g, 20, True, bool(trial % 2))
            levels, counts, kd = exact.exact_refinement(g, 20, True, bool(trial % 2))
            if r["k_done"] != kd or list(r["blocks_per_iter"]) != counts:
                return False
            if list(r["block_ids"]) != levels[kd]:
                return False
            es = list(zip(r["se_src"].tolist(), r["se_label"].tolist(), r["se_dst"].tolist()))
            if es != exact.quotient_edges(g, levels[kd]):
                return False
        # refinement keeps classes apart even when their hashes coincide
        # (the k-class is the pair (class at k-1, h^k), Sec. 2.5 definition)
        out, nb = orc.refine_classes([0, 1, 0, 1], [7, 7, 9, 7])
        if list(out) != [0, 1, 2, 1] or nb != 3:
            return False
        out, nb = orc.refine_classes([0, 1], [7, 7])
        if list(out) != [0, 1] or nb != 2:
            return False
        # a graph whose vertex has many equal keys: the mixer-sum must see a set
        g = gg.from_edges(5, [0, 0, 0, 1], [2, 3, 4, 2], [0, 0, 0, 0], types=[[]] * 5)
        r = orc.summarize(g, 3, True, True)
        if r["block_ids"][0] != r["block_ids"][1]:
            return False
        return True
    except ValueError:
        return False


def test_real_oracle_passes_the_pin_selection():
    assert _pins_hold()


def _compile_mutant(before, after, tmp_path):
    src = open(orc.SRC).read()
    assert src.count(before) >= 1, "mutation anchor not found"
    mutated = src.replace(before, after, 1)
    c = tmp_path / "mutant.c"
    so = tmp_path / "libmutant.so"
    c.write_text(mutated)
    subprocess.check_call(["gcc", "-O1", "-std=c99", "-w", "-shared", "-fPIC", "-o", str(so), str(c)])
    return str(so)


def _pins_hold_with(lib_path):
    saved = orc._lib
    try:
        orc._lib = orc.load(lib_path)
        return _pins_hold()
    finally:
        orc._lib = saved


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_planted_mistake_is_caught(name, tmp_path):
    before, after = MUTANTS[name]
    assert not _pins_hold_with(_compile_mutant(before, after, tmp_path)), \
        "planted mistake went unnoticed: " + name
