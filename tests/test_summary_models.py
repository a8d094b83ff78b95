"""The summary models of the paper's experiments (class collection,
attribute collection, SchemEX; Sec. 5) as parameters of the refinement,
pinned to their definitions: vertices grouped by their type set, by their
set of outgoing edge labels, and by their type set together with the set of
(edge label, neighbour type set) pairs.  The definitions are evaluated here
in plain Python, first-occurrence numbered; the CPU test holds the oracle to
them, the GPU test the HIP path."""

import numpy as np
import pytest

from oracle import oracle as orc
from paper_2111_12493_amd import binding
from paper_2111_12493_amd import graphgen as gg


def first_occurrence(keys):
    ids, out = {}, []
    for k in keys:
        if k is None:
            out.append(0xFFFFFFFF)
            continue
        out.append(ids.setdefault(k, len(ids)))
    return out


def by_definition(g, model):
    alive = [g.alive is None or bool(g.alive[v]) for v in range(g.n)]
    types = [frozenset(g.types_of(v)) for v in range(g.n)]
    keys = []
    for v in range(g.n):
        if not alive[v]:
            keys.append(None)
        elif model == "class_collection":
            keys.append(types[v])
        elif model == "attribute_collection":
            keys.append(frozenset(l for (l, w) in g.out_edges(v)))
        else:
            keys.append((types[v], frozenset((l, types[w]) for (l, w) in g.out_edges(v))))
    return first_occurrence(keys)


def graphs(seed, count):
    rng = np.random.default_rng(seed)
    for trial in range(count):
        n = int(rng.integers(1, 80))
        yield gg.random_small_graph(rng, n, int(rng.integers(0, 4 * n + 1)), int(rng.integers(1, 5)),
                                    int(rng.integers(1, 5)), 3, p_alive=1.0 if trial % 3 else 0.8)


@pytest.mark.parametrize("model", sorted(binding.SUMMARY_MODELS))
def test_oracle_parameters_give_the_model(model):
    p = binding.SUMMARY_MODELS[model]
    for g in graphs(71, 80):
        r = orc.summarize(g, p["k_max"], False, p["untyped"])
        assert list(r["block_ids"]) == by_definition(g, model)


@pytest.mark.gpu
@pytest.mark.parametrize("model", sorted(binding.SUMMARY_MODELS))
def test_gpu_gives_the_model(model):
    from gpu_util import ctx

    p = binding.SUMMARY_MODELS[model]
    for g in list(graphs(72, 40)) + [gg.rmat_graph(14, 1 << 17, n_types=16, n_labels=8, seed=3)]:
        r = binding.summarize_model(ctx(), binding.DeviceGraph(g), model)
        got = r.to_dict()
        r.free()
        ref = orc.summarize(g, p["k_max"], False, p["untyped"])
        assert list(got["block_ids"]) == by_definition(g, model)
        for key in ("hashes", "blocks_per_iter", "block_sizes", "se_src", "se_label", "se_dst"):
            assert np.array_equal(got[key], ref[key]), key
