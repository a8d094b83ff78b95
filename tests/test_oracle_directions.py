"""Pins for the oracle's direction and label parameterizations (no GPU).

Sec. 2.4 names a direction parameterization (outgoing, incoming or both
kinds of edges) and a label parameterization (only the edges whose label is
in a set P_l); Sec. 2.5 defines backward bisimulation as forward
bisimulation over incoming edges.  ``oracle.summarize_ext`` computes these;
the tests tie it to things outside itself:

* the hash-free exact refinement and the pairwise brute force, both over the
  (direction, label, partner) edges of ``exact.signature_edges``;
* reductions to the forward oracle, which the other pins already hold:
  backward = forward on the reversed graph; both = forward on the graph plus
  every edge reversed with label l + 2^31; a label set = forward on the
  graph without the other edges;
* closed-form block counts on chains and stars.
"""

import numpy as np
import pytest

from oracle import exact
from oracle import oracle as orc
from paper_2111_12493_amd import graphgen as gg

NONE = 0xFFFFFFFF


def edge_list(g):
    deg = (g.row_off[1:] - g.row_off[:-1]).astype(np.int64)
    src = np.repeat(np.arange(g.n, dtype=np.int64), deg)
    return src, g.tgt.astype(np.int64), g.lab.astype(np.int64)


def rebuild(g, src, dst, lab):
    return gg.from_edges(g.n, src, dst, lab, typ_off=g.typ_off, typ=g.typ, alive=g.alive)


def reversed_graph(g):
    s, d, l = edge_list(g)
    return rebuild(g, d, s, l)


def both_graph(g):
    s, d, l = edge_list(g)
    return rebuild(g, np.concatenate([s, d]), np.concatenate([d, s]), np.concatenate([l, l + (1 << 31)]))


def filtered_graph(g, labels):
    s, d, l = edge_list(g)
    keep = np.isin(l, np.asarray(sorted(labels), dtype=np.int64))
    return rebuild(g, s[keep], d[keep], l[keep])


def check_exact(g, k_max, stop, untyped, direction, labels):
    r = orc.summarize_ext(g, k_max, stop, untyped, direction, labels)
    levels, counts, k_done = exact.exact_refinement(g, k_max, stop, untyped, direction, labels)
    assert r["k_done"] == k_done
    assert list(r["blocks_per_iter"]) == counts
    want = [NONE if b is None else b for b in levels[k_done]]
    assert list(r["block_ids"]) == want
    sizes = np.bincount(np.array([b for b in want if b != NONE], dtype=np.int64), minlength=r["n_blocks"])
    assert list(r["block_sizes"]) == list(sizes)
    edges = list(zip(r["se_src"].tolist(), r["se_label"].tolist(), r["se_dst"].tolist()))
    assert edges == exact.quotient_edges(g, want, labels)
    return r


def random_graphs(seed, count, n_hi=30):
    rng = np.random.default_rng(seed)
    for trial in range(count):
        n = int(rng.integers(1, n_hi))
        g = gg.random_small_graph(rng, n, int(rng.integers(0, 4 * n + 1)), n_labels=int(rng.integers(1, 4)),
                                  n_types=int(rng.integers(1, 4)), max_types=2,
                                  p_alive=1.0 if trial % 3 else 0.8)
        yield trial, rng, g


def test_forward_without_label_set_equals_the_plain_oracle():
    for trial, rng, g in random_graphs(21, 60):
        for k, stop in ((50, True), (int(rng.integers(0, 4)), False)):
            a = orc.summarize_ext(g, k, stop, bool(trial % 2))
            b = orc.summarize(g, k, stop, bool(trial % 2))
            for key in a:
                assert np.array_equal(np.asarray(a[key]), np.asarray(b[key])), key


@pytest.mark.parametrize("direction", ["in", "both", "out"])
def test_partitions_match_exact_refinement(direction):
    for trial, rng, g in random_graphs(22 + len(direction), 80):
        labels = [None, [0], [0, 2], [5]][trial % 4]
        check_exact(g, 50, True, bool(trial % 2), direction, labels)
        check_exact(g, int(rng.integers(0, 4)), False, bool(trial % 2), direction, labels)


@pytest.mark.parametrize("direction", ["in", "both"])
def test_exact_refinement_matches_the_pairwise_definition(direction):
    # the reference itself, against the definition evaluated pair by pair
    rng = np.random.default_rng(31)
    for trial in range(150):
        n = int(rng.integers(1, 8))
        g = gg.random_small_graph(rng, n, int(rng.integers(0, 3 * n)), 2, 2, 1,
                                  p_alive=1.0 if trial % 4 else 0.7)
        k = int(rng.integers(0, 5))
        labels = None if trial % 3 else [1]
        levels, _, _ = exact.exact_refinement(g, k, False, bool(trial % 2), direction, labels)
        assert levels[k] == exact.brute_force_classes(g, k, bool(trial % 2), direction, labels)
        r = orc.summarize_ext(g, k, False, bool(trial % 2), direction, labels)
        assert list(r["block_ids"]) == [NONE if b is None else b for b in levels[k]]


def test_backward_is_forward_on_the_reversed_graph():
    for trial, rng, g in random_graphs(23, 60):
        k = int(rng.integers(0, 6))
        a = orc.summarize_ext(g, k, trial % 2 == 0, False, "in")
        b = orc.summarize(reversed_graph(g), k, trial % 2 == 0, False)
        for key in ("k_done", "fixpoint", "n_blocks", "hashes", "block_ids", "blocks_per_iter", "block_sizes"):
            assert np.array_equal(np.asarray(a[key]), np.asarray(b[key])), key


def test_both_is_forward_with_reversed_edges_on_shifted_labels():
    for trial, rng, g in random_graphs(24, 60):
        k = int(rng.integers(0, 6))
        a = orc.summarize_ext(g, k, trial % 2 == 0, bool(trial % 3 == 0), "both")
        b = orc.summarize(both_graph(g), k, trial % 2 == 0, bool(trial % 3 == 0))
        for key in ("k_done", "fixpoint", "n_blocks", "hashes", "block_ids", "blocks_per_iter", "block_sizes"):
            assert np.array_equal(np.asarray(a[key]), np.asarray(b[key])), key


def test_label_set_is_forward_on_the_kept_edges():
    for trial, rng, g in random_graphs(25, 60):
        labels = [[0], [1, 2], [0, 1, 2], [7]][trial % 4]
        k = int(rng.integers(0, 6))
        for direction, plain in (("out", lambda h: h), ("in", reversed_graph)):
            a = orc.summarize_ext(g, k, True, False, direction, labels)
            b = orc.summarize(plain(filtered_graph(g, labels)), k, True, False)
            for key in ("k_done", "n_blocks", "hashes", "block_ids", "blocks_per_iter"):
                assert np.array_equal(np.asarray(a[key]), np.asarray(b[key])), (direction, key)


@pytest.mark.parametrize("n", [1, 2, 5, 30])
def test_chain_counts_backward_and_both(n):
    # path 0 -> 1 -> ... -> n-1, one label, untyped.  Backward: vertex i
    # sees an incoming chain of length i, so the k-classes are
    # {0}, ..., {k-1}, {k, ..., n-1}: min(k + 1, n) of them.  Both: i is told
    # apart by min(i, k) and min(n - 1 - i, k), the distances to the two ends
    # as far as k steps see.
    g = gg.from_edges(n, list(range(n - 1)), list(range(1, n)), [0] * (n - 1))
    for k in range(0, 8):
        rb = orc.summarize_ext(g, k, False, True, "in")
        assert rb["n_blocks"] == min(k + 1, n)
        pairs = {(min(i, k), min(n - 1 - i, k)) for i in range(n)}
        rf = orc.summarize_ext(g, k, False, True, "both")
        assert rf["n_blocks"] == len(pairs)


def test_star_counts_with_a_label_set():
    # center 0 with l=0 edges to 1..4 and l=1 edges to 5..8, untyped
    leaves = list(range(1, 9))
    g = gg.from_edges(9, [0] * 8, leaves, [0] * 4 + [1] * 4)
    for direction, labels, want in (("out", None, 2),
                                    ("in", None, 3),   # centre, leaves with an l=0 / an l=1 in-edge
                                    ("both", None, 3),
                                    ("out", [0], 2),   # centre vs all leaves (no out-edges)
                                    ("in", [0], 2),    # 1..4 have an in-edge; centre and 5..8 none
                                    ("both", [0], 3),  # centre, kept leaves, dropped leaves
                                    ("both", [5], 1)):  # no edge left
        r = orc.summarize_ext(g, 3, False, True, direction, labels)
        assert r["n_blocks"] == want, (direction, labels)
    r = orc.summarize_ext(g, 3, False, True, "both", [0])
    assert list(r["block_ids"]) == [0, 1, 1, 1, 1, 2, 2, 2, 2]
    assert list(zip(r["se_src"], r["se_label"], r["se_dst"])) == [(0, 0, 1)]


def test_in_edge_salt_is_the_salt_of_the_shifted_label():
    for lab in (0, 1, 63, (1 << 24) - 1):
        assert orc.lib().bo_label_salt_in(lab) == orc.lib().bo_label_salt(lab + (1 << 31))


def test_both_directions_and_backward_flags_exclude_each_other():
    g = gg.from_edges(2, [0], [1], [0])
    row_off, tgt, lab, typ_off, typ, alive = orc._csr(g)
    z = np.zeros(4, dtype=np.uint64)
    u = np.zeros(4, dtype=np.uint32)
    import ctypes
    c32, c64 = ctypes.c_uint32(), ctypes.c_uint64()
    rc = orc.lib().bo_summarize_ext(2, 1, orc._ptr(row_off), orc._ptr(tgt), orc._ptr(lab), orc._ptr(typ_off),
                                    orc._ptr(np.zeros(1, dtype=np.uint32)), None, 2,
                                    orc.BACKWARD | orc.BOTH_DIRECTIONS, None, 0, orc._ptr(z), orc._ptr(u),
                                    orc._ptr(u), ctypes.byref(c32), ctypes.byref(c32), ctypes.byref(c32),
                                    orc._ptr(u), ctypes.byref(c64), orc._ptr(u), orc._ptr(u), orc._ptr(u))
    assert rc != 0


# ------------------------------------------------- planted mistakes (CPU)

EXT_MUTANTS = {
    "backward_partner_is_self": ("partner[fill[w]] = v;", "partner[fill[w]] = w;"),
    "in_edges_salted_like_out_edges": (
        "salt[fill[w]++] = (flags & BO_BOTH_DIRECTIONS) ? bo_label_salt_in(lab[e]) : bo_label_salt(lab[e]);",
        "salt[fill[w]++] = bo_label_salt(lab[e]);"),
    "label_set_values_ignored": ("return !keep_label || (l < n_keep && keep_label[l]);",
                                 "return !keep_label || l < n_keep;"),
    "summary_edges_ignore_label_set": (
        "            if (!kept(keep_label, n_keep, lab[e])) continue;\n            tr[ne].s = block_ids[v];",
        "            tr[ne].s = block_ids[v];"),
}


def _ext_pins_hold() -> bool:
    try:
        for direction in ("in", "both"):
            for trial, rng, g in random_graphs(41, 40):
                labels = [None, [0, 2]][trial % 2]
                check_exact(g, 20, True, bool(trial % 3 == 0), direction, labels)
        for trial, rng, g in random_graphs(42, 30):
            a = orc.summarize_ext(g, 4, False, False, "both")
            b = orc.summarize(both_graph(g), 4, False, False)
            if not np.array_equal(a["hashes"], b["hashes"]):
                return False
        return True
    except (AssertionError, ValueError):
        return False


def test_real_oracle_passes_the_extension_pins():
    assert _ext_pins_hold()


@pytest.mark.parametrize("name", sorted(EXT_MUTANTS))
def test_planted_mistake_in_the_extension_is_caught(name, tmp_path):
    import subprocess

    before, after = EXT_MUTANTS[name]
    src = open(orc.SRC).read()
    assert src.count(before) == 1, "mutation anchor not found"
    c = tmp_path / "mutant.c"
    so = tmp_path / "libmutant.so"
    c.write_text(src.replace(before, after))
    subprocess.check_call(["gcc", "-O1", "-std=c99", "-w", "-shared", "-fPIC", "-o", str(so), str(c)])
    saved = orc._lib
    try:
        orc._lib = orc.load(str(so))
        held = _ext_pins_hold()
    finally:
        orc._lib = saved
    assert not held, "planted mistake went unnoticed: " + name
