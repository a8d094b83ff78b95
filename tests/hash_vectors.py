"""The frozen hash-spec vectors (tests/golden/hash_spec_vectors.json) and
their worked graph, for the oracle pins and the GPU parity test."""

import json
import os

from paper_2111_12493_amd import graphgen as gg

PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "hash_spec_vectors.json")


def _ints(x):
    if isinstance(x, str) and x.startswith("0x"):
        return int(x, 16)
    if isinstance(x, list):
        return [_ints(y) for y in x]
    if isinstance(x, dict):
        return {k: _ints(y) for k, y in x.items()}
    return x


def load() -> dict:
    with open(PATH) as f:
        raw = json.load(f)
    graph = raw.pop("graph")
    v = _ints(raw)
    v["graph"] = graph
    return v


def graph(v=None):
    """The worked graph as a graphgen.Graph."""
    v = v or load()
    types = v["graph"]["types"]
    edges = v["graph"]["edges"]
    return gg.from_edges(len(types), [e[0] for e in edges], [e[2] for e in edges], [e[1] for e in edges],
                         types=types)
