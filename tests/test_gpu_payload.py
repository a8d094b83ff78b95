"""GPU check of the source-label payload (Sec. 3.3: a payload function may
memorize each vertex's source label; merging vertices into a block joins
their source lists): the distinct (block, source label) pairs over the
alive vertices, sorted, against that definition evaluated on the oracle's
block ids."""

import numpy as np
import pytest

from oracle import oracle as orc
from paper_2111_12493_amd import binding
from paper_2111_12493_amd import graphgen as gg

from gpu_util import ctx

pytestmark = pytest.mark.gpu


def by_definition(block_ids, labels):
    pairs = sorted({(int(b), int(l)) for b, l in zip(block_ids, labels) if b != 0xFFFFFFFF})
    return (np.array([p[0] for p in pairs], dtype=np.uint32), np.array([p[1] for p in pairs], dtype=np.uint32))


def check(g, labels, **kw):
    r = binding.summarize(ctx(), binding.DeviceGraph(g), **kw)
    got = binding.source_payload(ctx(), r, labels)
    r.free()
    ref = orc.summarize(g, kw.get("k_max", g.n + 2), kw.get("stop_at_fixpoint", True), kw.get("untyped", False))
    want = by_definition(ref["block_ids"], labels)
    assert np.array_equal(got[0], want[0]) and np.array_equal(got[1], want[1])
    return got


def test_small_graphs_and_edge_cases():
    rng = np.random.default_rng(91)
    check(gg.from_edges(0, [], [], []), [])
    for trial in range(40):
        n = int(rng.integers(1, 70))
        g = gg.random_small_graph(rng, n, int(rng.integers(0, 4 * n + 1)), 3, 3, 2,
                                  p_alive=1.0 if trial % 3 else 0.7)
        labels = rng.integers(0, [1, 3, 1 << 32][trial % 3], n, dtype=np.uint64).astype(np.uint32)
        check(g, labels, result_on_host=trial % 5 == 0)


def test_rmat_graph_with_many_sources():
    g = gg.rmat_graph(16, 1 << 19, n_types=32, n_labels=16, seed=12)
    labels = np.random.default_rng(5).integers(0, 1000, g.n).astype(np.uint32)
    b, l = check(g, labels)
    assert b.size >= 1 and np.all(np.diff(b.astype(np.int64) * (1 << 32) + l) > 0)
