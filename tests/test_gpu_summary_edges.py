"""GPU parity of the summary edges (Sec. 2.6) at the size classes of the
source-block segments they are sorted in.

A block's segment holds the (label, target block) values of all out-edges
of its vertices.  Segments of 2..256 values are sorted in tiles of several
segments (whose first values lie in ranges of 3,840 positions), 257..4,096
and 4,097..16,384 values by one workgroup each, longer ones by a global
sort.  These graphs put segments on both sides of every class boundary,
make blocks of many isomorphic vertices (one segment fed by thousands of
vertices, most of its values equal), and mix many small segments so tiles
start and end inside runs of them; every output must equal the oracle's."""

import numpy as np
import pytest

from oracle import oracle as orc
from paper_2111_12493_amd import graphgen as gg

from gpu_util import assert_same, gpu_summarize, ctx
from paper_2111_12493_amd import binding

pytestmark = pytest.mark.gpu

SIZES = [1, 2, 3, 255, 256, 257, 3839, 3840, 3841, 4095, 4096, 4097, 16383, 16384, 16385, 40000]


def segment_graph(seed, n_labels=6, leaf_types=300, wide_labels=False):
    rng = np.random.default_rng(seed)
    n_leaf = 3000
    src, dst, lab, types = [], [], [], []
    leaf0 = 0
    for _ in range(n_leaf):
        types.append([int(rng.integers(0, leaf_types))])

    def label(k):
        if wide_labels:
            return rng.integers(0, 1 << 20, k)
        return rng.integers(0, n_labels, k)

    nxt = n_leaf
    # one singleton block per size: a vertex of its own type with `s` edges
    # into the leaves (repeated (label, leaf type) pairs are de-duplicated)
    for i, s in enumerate(SIZES):
        v = nxt
        nxt += 1
        types.append([10_000 + i])
        src.extend([v] * s)
        dst.extend(rng.integers(leaf0, n_leaf, s).tolist())
        lab.extend(label(s).tolist())
    # blocks of many isomorphic vertices: every member has the same type and
    # the same single edge, so the block's segment is `k` equal values
    for j, k in enumerate([300, 5000, 20000]):
        t = 20_000 + j
        target = int(rng.integers(leaf0, n_leaf))
        for _ in range(k):
            v = nxt
            nxt += 1
            types.append([t])
            src.append(v)
            dst.append(target)
            lab.append(j)
    # two identical twins per size class boundary: their block's segment is
    # twice the vertex degree
    for s in (128, 129, 2048, 2049, 8192, 8193):
        tt = 30_000 + s
        d = rng.integers(leaf0, n_leaf, s).tolist()
        ll = label(s).tolist()
        for _ in range(2):
            v = nxt
            nxt += 1
            types.append([tt])
            src.extend([v] * s)
            dst.extend(d)
            lab.extend(ll)
    # many small vertices of random degree, some sharing a type
    for _ in range(400):
        v = nxt
        nxt += 1
        types.append([int(rng.integers(40_000, 40_050))])
        s = int(rng.integers(1, 300))
        src.extend([v] * s)
        dst.extend(rng.integers(0, nxt, s).tolist())
        lab.extend(label(s).tolist())
    return gg.from_edges(nxt, src, dst, lab, types=types)


@pytest.mark.parametrize("seed", [1, 2])
def test_segment_classes_equal_the_oracle(seed):
    g = segment_graph(seed)
    for k in (1, 2):
        ref = orc.summarize(g, k, False)
        assert_same(gpu_summarize(g, k, stop=False), ref, ("k", k))
    ref = orc.summarize(g, g.n + 2, True)
    assert_same(gpu_summarize(g, binding.K_UNBOUNDED), ref, "fixpoint")


def test_u16_and_wide_labels():
    g = segment_graph(3)
    ref = orc.summarize(g, 2, False)
    assert_same(gpu_summarize(gg.with_u16_labels(g), 2, stop=False), ref, "u16")
    w = segment_graph(4, wide_labels=True)
    ref = orc.summarize(w, 2, False)
    assert_same(gpu_summarize(w, 2, stop=False), ref, "labels up to 2^20")


def test_previous_level_targets():
    g = segment_graph(5)
    for k in (1, 2, 3):
        ref = orc.summarize(g, k, False, prev_level_edges=True)
        r = binding.summarize(ctx(), binding.DeviceGraph(g), k_max=k, stop_at_fixpoint=False,
                              prev_level_edges=True)
        got = r.to_dict()
        r.free()
        assert_same(got, ref, ("prev level", k))


def test_many_small_segments_across_tiles():
    # about 60,000 segments of 2..40 values: thousands of small tiles, with
    # every tile range cutting through runs of them
    rng = np.random.default_rng(8)
    n = 60_000
    deg = rng.integers(0, 41, n)
    src = np.repeat(np.arange(n), deg)
    dst = rng.integers(0, n, src.size)
    lab = rng.integers(0, 3, src.size)
    types = [[int(t)] for t in rng.integers(0, 5, n)]
    g = gg.from_edges(n, src, dst, lab, types=types)
    for k in (1, 2):
        ref = orc.summarize(g, k, False)
        assert_same(gpu_summarize(g, k, stop=False), ref, ("k", k))
