"""Pins of the oracle's previous-level summary edges (Sec. 2.6's inductive
definition of vertex summaries: for the k-bisimulation the primary vertex of
v has an l-edge to the (k-1)-class of each l-neighbour).

* closed form on a chain of L edges: at 1 <= k <= L the edges are
  (j, 0, j) for j < k, while the quotient edges are (j, 0, j + 1) plus
  (0, 0, 0) when L > k;
* against exact naive refinement (no hashing): the triples
  (class_k(v), l, class_{k-1}(w)) from the exact partitions of levels k and
  k-1, on random small graphs, with and without a label set;
* at a fixpoint and at k = 0 they equal the quotient edges.
"""

import numpy as np
import pytest

from oracle import exact
from oracle import oracle as orc
from paper_2111_12493_amd import graphgen as gg


def triples(r):
    return list(zip(r["se_src"].tolist(), r["se_label"].tolist(), r["se_dst"].tolist()))


@pytest.mark.parametrize("L", [1, 2, 5, 9])
def test_chain_closed_form(L):
    for k in range(1, L + 1):
        r = orc.summarize(gg.chain(L), k, False, True, prev_level_edges=True)
        assert triples(r) == [(j, 0, j) for j in range(k)], (L, k)
        q = orc.summarize(gg.chain(L), k, False, True)
        assert triples(q) == sorted(([(0, 0, 0)] if L > k else []) + [(j, 0, j + 1) for j in range(k)]), (L, k)


def test_against_exact_refinement():
    rng = np.random.default_rng(303)
    for trial in range(80):
        n = int(rng.integers(2, 30))
        g = gg.random_small_graph(rng, n, int(rng.integers(0, 4 * n)), 3, 3, 3,
                                  p_alive=1.0 if trial % 3 else 0.8)
        k = int(rng.integers(1, 6))
        untyped = bool(trial % 2)
        labels = [0, 2] if trial % 4 == 1 else None
        levels, counts, kd = exact.exact_refinement(g, k, False, untyped, labels=labels)
        if labels is None:
            r = orc.summarize(g, k, False, untyped, prev_level_edges=True)
        else:
            r = orc.summarize_ext(g, k, False, untyped, "out", labels, prev_level_edges=True)
        assert r["k_done"] == kd == k
        want = exact.quotient_edges(g, levels[kd], labels, dst_ids=levels[kd - 1])
        assert triples(r) == want, trial


def test_fixpoint_and_level_zero_give_the_quotient():
    rng = np.random.default_rng(17)
    for trial in range(40):
        n = int(rng.integers(2, 25))
        g = gg.random_small_graph(rng, n, int(rng.integers(0, 3 * n)), 3, 3, 2)
        a = orc.summarize(g, 64, True, False, prev_level_edges=True)
        b = orc.summarize(g, 64, True, False)
        assert a["fixpoint"] == 1
        assert triples(a) == triples(b)
        a = orc.summarize(g, 0, False, False, prev_level_edges=True)
        b = orc.summarize(g, 0, False, False)
        assert triples(a) == triples(b)


def test_backward_is_rejected():
    g = gg.chain(3)
    with pytest.raises(ValueError):
        orc.summarize_ext(g, 2, False, False, "in", None, prev_level_edges=True)
