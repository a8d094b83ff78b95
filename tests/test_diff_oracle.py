"""Pins for the oracle's snapshot diff (change detection without a change
log, Sec. 3.2's change classes between two snapshots): applying the diff to
the earlier snapshot gives the later one (alive flags, type sets, edge
triple sets), and the diff of a graph with itself is empty; both on random
snapshot pairs made by random update batches."""

import numpy as np
import pytest

from oracle import updates as upd
from paper_2111_12493_amd import graphgen as gg


def as_sets(g):
    alive = [g.alive is None or bool(g.alive[v]) for v in range(g.n)]
    types = [frozenset(int(x) for x in g.typ[int(g.typ_off[v]):int(g.typ_off[v + 1])]) if alive[v] else None
             for v in range(g.n)]
    tri = set()
    for u in range(g.n):
        for e in range(int(g.row_off[u]), int(g.row_off[u + 1])):
            tri.add((u, int(g.lab[e]), int(g.tgt[e])))
    return alive, types, tri


def snapshot_pairs(seed, count):
    rng = np.random.default_rng(seed)
    for trial in range(count):
        n = int(rng.integers(1, 40))
        g = gg.random_small_graph(rng, n, int(rng.integers(0, 4 * n + 1)), 3, 3, 2)
        ops = gg.update_ops(g, rng, int(rng.integers(0, 40)))
        yield g, upd.apply_ops(g, gg.ops_as_tuples(ops))


def test_diff_reproduces_the_later_snapshot():
    for before, after in snapshot_pairs(81, 150):
        ops = upd.diff_snapshots(before, after)
        assert as_sets(upd.apply_ops(before, ops)) == as_sets(after)


def test_diff_of_a_snapshot_with_itself_is_empty():
    for before, after in snapshot_pairs(82, 40):
        assert upd.diff_snapshots(after, after) == []


def test_diff_ignores_copies_and_order():
    # the same triples and type sets in another order, with repeats
    a = gg.from_edges(3, [0, 0, 1], [1, 2, 2], [5, 6, 7], types=[[1, 2], [3], []])
    b = gg.from_edges(3, [1, 0, 0, 0], [2, 2, 1, 2], [7, 6, 5, 6], types=[[2, 1, 1], [3], []])
    assert upd.diff_snapshots(a, b) == []


def test_each_change_class():
    a = gg.from_edges(4, [0, 1, 2], [1, 2, 3], [0, 0, 1], types=[[1], [2], [3], [4]])
    b = gg.from_edges(6, [0, 1, 4, 5], [1, 3, 0, 4], [0, 2, 0, 1], types=[[1], [9], [3], [4], [7], []],
                      alive=np.array([1, 1, 0, 1, 1, 1], dtype=np.uint8))
    ops = upd.diff_snapshots(a, b)
    assert ops == [("add_v", [7]), ("add_v", []), ("mod_v", 1, [9]), ("add_e", 1, 2, 3),
                   ("add_e", 4, 0, 0), ("add_e", 5, 1, 4), ("del_v", 2)]
    assert as_sets(upd.apply_ops(a, ops)) == as_sets(b)


def test_resurrection_and_shrinking_are_rejected():
    a = gg.from_edges(2, [], [], [], alive=np.array([1, 0], dtype=np.uint8))
    with pytest.raises(ValueError):
        upd.diff_snapshots(a, gg.from_edges(2, [], [], []))
    with pytest.raises(ValueError):
        upd.diff_snapshots(gg.from_edges(3, [], [], []), gg.from_edges(2, [], [], []))
