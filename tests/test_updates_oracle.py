"""Pins of the sequential update semantics (oracle/updates.py) on hand-built
cases whose resulting graphs are written out by hand, plus the batch
generator's validity."""

import numpy as np
import pytest

from oracle import oracle as orc
from oracle.exact import exact_refinement
from oracle.updates import apply_ops
from paper_2111_12493_amd import graphgen as gg


def rows(g):
    """Sorted (label, target) multiset per alive vertex; None for dead ones."""
    out = []
    for v in range(g.n):
        if g.alive is not None and not g.alive[v]:
            out.append(None)
            continue
        a, b = int(g.row_off[v]), int(g.row_off[v + 1])
        out.append(sorted(zip(g.lab[a:b].tolist(), g.tgt[a:b].tolist())))
    return out


def base():
    # 0 -a-> 1 twice (duplicate triple), 0 -b-> 2, 1 -a-> 2, 2 -a-> 0
    return gg.from_edges(3, [0, 0, 0, 1, 2], [1, 1, 2, 2, 0], [0, 0, 1, 0, 0],
                         types=[[5], [6], [6]])


def test_add_existing_triple_is_noop_and_keeps_multiplicity():
    g = apply_ops(base(), [("add_e", 0, 0, 1)])
    assert rows(g) == [[(0, 1), (0, 1), (1, 2)], [(0, 2)], [(0, 0)]]


def test_delete_removes_every_copy_and_absent_delete_is_noop():
    g = apply_ops(base(), [("del_e", 0, 0, 1), ("del_e", 2, 1, 0)])
    assert rows(g) == [[(1, 2)], [(0, 2)], [(0, 0)]]


def test_delete_then_add_leaves_one_copy():
    g = apply_ops(base(), [("del_e", 0, 0, 1), ("add_e", 0, 0, 1)])
    assert rows(g) == [[(0, 1), (1, 2)], [(0, 2)], [(0, 0)]]


def test_modify_relabels_and_adds_when_absent():
    g = apply_ops(base(), [("mod_e", 0, 1, 2, 3), ("mod_e", 1, 7, 0, 4)])
    assert rows(g) == [[(0, 1), (0, 1), (3, 2)], [(0, 2), (4, 0)], [(0, 0)]]


def test_vertex_ops():
    g = apply_ops(base(), [("add_v", [1, 1, 2]), ("add_e", 3, 2, 0), ("mod_v", 1, []), ("del_v", 2)])
    assert g.n == 4
    assert list(g.alive) == [1, 1, 0, 1]
    assert rows(g) == [[(0, 1), (0, 1)], [], None, [(2, 0)]]
    assert g.types_of(1) == [] and g.types_of(3) == [1, 1, 2] and g.types_of(2) == []


def test_invalid_ops_raise():
    with pytest.raises(ValueError):
        apply_ops(base(), [("del_v", 1), ("add_e", 0, 0, 1)])
    with pytest.raises(IndexError):
        apply_ops(base(), [("add_e", 0, 0, 3)])
    with pytest.raises(ValueError):
        apply_ops(base(), [("del_v", 1), ("mod_v", 1, [2])])


def test_fig1_change_matches_direct_construction():
    # Fig. 1: the change between the two snapshots as one update batch
    before, after = gg.fig1_scenario(False), gg.fig1_scenario(True)
    src_b, src_a = before.src(), after.src()
    eb = set(zip(src_b.tolist(), before.lab.tolist(), before.tgt.tolist()))
    ea = set(zip(src_a.tolist(), after.lab.tolist(), after.tgt.tolist()))
    ops = [("del_e", u, l, w) for (u, l, w) in sorted(eb - ea)] + \
          [("add_e", u, l, w) for (u, l, w) in sorted(ea - eb)]
    for v in range(after.n):
        if before.types_of(v) != after.types_of(v):
            ops.append(("mod_v", v, after.types_of(v)))
    g = apply_ops(before, ops)
    assert orc.summarize(g, 1, False)["block_ids"].tolist() == \
        orc.summarize(after, 1, False)["block_ids"].tolist()


def test_generated_batches_are_valid_and_summaries_match_exact_refinement():
    rng = np.random.default_rng(3)
    for trial in range(6):
        g = gg.random_small_graph(rng, 30, 90, 3, 3, 3)
        d = gg.update_ops(g, rng, 40, n_labels=3, n_types=3)
        g2 = apply_ops(g, gg.ops_as_tuples(d))
        r = orc.summarize(g2, 4, False)
        levels, _, _ = exact_refinement(g2, 4, stop_at_fixpoint=False)
        want = [0xFFFFFFFF if x is None else x for x in levels[-1]]
        assert r["block_ids"].tolist() == want


def test_replay_rows_equals_whole_graph_application():
    # the per-vertex replay used at full size agrees with apply_ops on every
    # vertex of random graphs and batches (including deletions of targets)
    from oracle.updates import replay_rows

    rng = np.random.default_rng(41)
    for trial in range(6):
        g = gg.uniform_graph(150, 700, 5, 6, seed=trial + 3)
        d = gg.update_ops(g, rng, 120, n_labels=6, n_types=5)
        ops = gg.ops_as_tuples(d)
        full = apply_ops(g, ops)
        rows, types, alive = replay_rows(g, ops, range(full.n))
        for v in range(full.n):
            a, b = int(full.row_off[v]), int(full.row_off[v + 1])
            assert rows[v] == sorted(zip(full.lab[a:b].tolist(), full.tgt[a:b].tolist())), (trial, v)
            assert types[v] == sorted(full.types_of(v)), (trial, v)
            assert alive[v] == bool(full.alive[v]), (trial, v)
