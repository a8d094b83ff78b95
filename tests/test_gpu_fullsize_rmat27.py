"""GPU parity at the full size of the large R-MAT workload: 2^27 vertices,
2^30 edges, 1,024 types and 256 edge labels (Zipf 1.2, uint16 labels), run
to the fixpoint capped at k = 64, in the launch configuration of a plain
bsim_summarize call.  The graph is drawn on the GPU (devgen).

* Sampled outputs the oracle computes one by one: h^1 of 256 vertices (the
  4 largest hubs among them) and h^2 of 24 (vertices without out-edges and
  random ones), each from the subgraph that fixes it (DeviceCSR.induced,
  pinned on the CPU in test_devgen.py).
* Properties that hold at any size for the run to the fixpoint: the class
  counts rise until they stop; block sizes and ids agree; ids are numbered
  in first-occurrence order; a block has one hash and lies inside one level-1
  block (partition k refines partition 1); the summary edges are exactly the
  distinct (block(v), label, block(w)) of all edges, sorted.
"""

import numpy as np
import pytest

from oracle import oracle as orc
from paper_2111_12493_amd import binding, devgen

from gpu_util import ctx

pytestmark = pytest.mark.gpu
_graph = {}


def rmat27():
    if "g" not in _graph:
        _graph["g"] = devgen.make_device_config("rmat27")
    return _graph["g"]


def seeds_for(g, count, rng, hubs=True):
    import torch

    deg = (g.row_off[1:] - g.row_off[:-1]).to(torch.int64)
    big = torch.topk(deg, 4).indices.tolist() if hubs else []
    empty = torch.nonzero(deg == 0)[:4, 0].tolist()
    rand = rng.integers(0, g.n, count - len(big) - len(empty)).tolist()
    return sorted(set(big) | set(empty) | set(rand))


@pytest.mark.parametrize("depth,count", [(1, 256), (2, 24)])
def test_sampled_levels_match_oracle(depth, count):
    g = rmat27()
    r = binding.summarize(ctx(), g, k_max=depth, stop_at_fixpoint=False, summary_edges=False)
    assert r.k_done == depth
    h = r.fetch_device("hashes")
    r.free()
    # (the largest hubs only at level 1: their level-2 cone is most of the graph)
    seeds = seeds_for(g, count, np.random.default_rng(100 + depth), hubs=depth == 1)
    sub, ids = g.induced(seeds, depth)
    ref, _ = orc.iterate(sub, depth)
    got = h[seeds].cpu().numpy().view(np.uint64)
    print("rmat27 h^%d: %d sampled vertices, oracle subgraph %d vertices / %d edges"
          % (depth, len(seeds), sub.n, sub.m), flush=True)
    assert np.array_equal(got, ref[ids]), ("h^%d" % depth, int(np.sum(got != ref[ids])))


def test_fixpoint_properties():
    import torch

    g = rmat27()
    r1 = binding.summarize(ctx(), g, k_max=1, stop_at_fixpoint=False, summary_edges=False)
    b1 = r1.fetch_device("block_ids").to(torch.int64)
    r1.free()
    r = binding.summarize(ctx(), g, k_max=64, stop_at_fixpoint=True)
    bpi = np.asarray(r.blocks_per_iter, dtype=np.int64)
    assert r.k_done <= 64 and (r.fixpoint == 1 or r.k_done == 64)
    assert np.all(np.diff(bpi) >= 0) and r.n_blocks == bpi[-1]
    if r.fixpoint:
        assert bpi[-1] == bpi[-2]
    bid = r.fetch_device("block_ids").to(torch.int64)
    sizes = r.fetch_device("block_sizes").to(torch.int64)
    h = r.fetch_device("hashes")
    nb = r.n_blocks
    assert int(bid.max()) == nb - 1 and int(sizes.sum()) == g.n
    assert torch.equal(torch.bincount(bid, minlength=nb), sizes)
    # first-occurrence numbering: the first vertex of block b precedes that of b+1
    first = torch.full((nb,), g.n, dtype=torch.int64, device=bid.device)
    first.scatter_reduce_(0, bid, torch.arange(g.n, device=bid.device), reduce="amin")
    assert bool(torch.all(first[1:] > first[:-1]))
    # one hash per block, and every block inside one level-1 block
    for val in (h, b1):
        lo = torch.full((nb,), torch.iinfo(torch.int64).max, dtype=torch.int64, device=bid.device)
        hi = torch.full((nb,), torch.iinfo(torch.int64).min, dtype=torch.int64, device=bid.device)
        lo.scatter_reduce_(0, bid, val, reduce="amin")
        hi.scatter_reduce_(0, bid, val, reduce="amax")
        assert torch.equal(lo, hi)
    # summary edges: the sorted distinct (block(v), label, block(w))
    src = g.src().to(torch.int64)
    lab = g.lab.to(torch.int64) & 0xFFFF
    key = (bid[src] << 35) | (lab << 27) | bid[g.tgt.to(torch.int64)]
    del src, lab
    want = torch.unique(key)
    del key
    ss, sl, sd = (r.fetch_device(f).to(torch.int64) for f in ("se_src", "se_label", "se_dst"))
    got = (ss << 35) | (sl << 27) | sd
    print("rmat27 fixpoint: n=%d m=%d k_done=%d fixpoint=%d blocks=%d summary edges=%d"
          % (g.n, g.m, r.k_done, r.fixpoint, nb, got.numel()), flush=True)
    assert got.numel() == want.numel() and torch.equal(got, want)
    r.free()
