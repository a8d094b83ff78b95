"""The direction and label parameterizations at the size of the R-MAT
refinement workload (2^22 vertices, 2^25 edges, 64 chains of 2,000 edges,
run to the fixpoint), in the launch configuration of bsim_summarize.

The oracle cannot run this size whole; the checks use what fixes the answer
at any size, against the forward path that the other full-size tests hold
to the oracle:
* backward = forward on the reversed graph (hashes, block ids, counts,
  sizes; summary edges as the transposed triples);
* a label set = forward on the graph without the other edges (every output);
* both directions on a 2^18-vertex R-MAT graph against the oracle, whole.
"""

import numpy as np
import pytest

from oracle import oracle as orc
from paper_2111_12493_amd import binding
from paper_2111_12493_amd import graphgen as gg

from gpu_util import assert_same, ctx

pytestmark = pytest.mark.gpu
_g = {}


def rmat22():
    if "g" not in _g:
        _g["g"] = gg.make_config("rmat22_chains")
    return _g["g"]


def edges(g):
    deg = (g.row_off[1:] - g.row_off[:-1]).astype(np.int64)
    return np.repeat(np.arange(g.n, dtype=np.int64), deg), g.tgt.astype(np.int64), g.lab.astype(np.int64)


def run(g, **kw):
    r = binding.summarize(ctx(), binding.DeviceGraph(g), k_max=binding.K_UNBOUNDED, **kw)
    d = r.to_dict()
    r.free()
    return d


def test_backward_equals_forward_of_the_reversed_graph():
    g = rmat22()
    s, d, l = edges(g)
    rev = gg.from_edges(g.n, d, s, l, typ_off=g.typ_off, typ=g.typ)
    a = run(g, direction="in")
    b = run(rev)
    print("rmat22_chains backward: k_done=%d blocks=%d summary edges=%d" % (a["k_done"], a["n_blocks"],
                                                                         len(a["se_src"])), flush=True)
    for key in ("k_done", "fixpoint", "n_blocks", "hashes", "block_ids", "blocks_per_iter", "block_sizes"):
        assert np.array_equal(np.asarray(a[key]), np.asarray(b[key])), key
    ta = np.stack([a["se_src"], a["se_label"], a["se_dst"]], 1).astype(np.int64)
    tb = np.stack([b["se_dst"], b["se_label"], b["se_src"]], 1).astype(np.int64)
    ka = (ta[:, 0] << 40) | (ta[:, 1] << 32) | ta[:, 2]
    kb = np.sort((tb[:, 0] << 40) | (tb[:, 1] << 32) | tb[:, 2])
    assert np.array_equal(ka, kb)


def test_label_set_equals_forward_of_the_kept_edges():
    g = rmat22()
    s, d, l = edges(g)
    keep = l % 3 != 1
    labels = sorted(set(range(int(l.max()) + 1)) - set(range(1, int(l.max()) + 1, 3)))
    kept = gg.from_edges(g.n, s[keep], d[keep], l[keep], typ_off=g.typ_off, typ=g.typ)
    a = run(g, labels=labels)
    b = run(kept)
    print("rmat22_chains label set: %d of %d edges, k_done=%d blocks=%d" % (int(keep.sum()), g.m, a["k_done"],
                                                                           a["n_blocks"]), flush=True)
    assert_same(a, b, "label set")


def test_both_directions_on_rmat18_against_the_oracle():
    g = gg.rmat_graph(18, 1 << 21, n_types=64, n_labels=32, seed=18)
    ref = orc.summarize_ext(g, 6, False, False, "both", None)
    r = binding.summarize(ctx(), binding.DeviceGraph(gg.with_u16_labels(g)), k_max=6, stop_at_fixpoint=False,
                          direction="both")
    gpu = r.to_dict()
    r.free()
    assert_same(gpu, ref, "rmat18 both")
