"""GPU parity at the full size of the batched workload: 4,096 R-MAT graphs
(edges log-uniform in [10^2, 10^6], about 4.3e8 in all, average degree
U(4, 16), 32 types and 32 labels, Zipf 1.0), each to its own fixpoint, in
one bsim_batch_summarize call (the launch configuration of the batched
measurement).  The graphs are drawn on the GPU (devgen).

* every graph: block sizes sum to its vertex count and the class counts
  rise until they stop;
* 32 graphs (the largest, the smallest and random ones): every output equal
  to a bsim_summarize call on that graph alone;
* 12 graphs of at most 20,000 edges: every output equal to the oracle's.
"""

import numpy as np
import pytest

from oracle import oracle as orc
from paper_2111_12493_amd import binding, devgen

from gpu_util import assert_same, ctx

pytestmark = pytest.mark.gpu


def test_full_batch_matches_alone_and_oracle():
    graphs = devgen.batched_device(4096, 1e6, seed=23)
    assert sum(g.m for g in graphs) > 4e8
    rs = binding.batch_summarize(ctx(), graphs)
    for g, r in zip(graphs, rs):
        bpi = np.asarray(r.blocks_per_iter, dtype=np.int64)
        assert r.fixpoint == 1 and np.all(np.diff(bpi) >= 0) and bpi[-1] == bpi[-2] == r.n_blocks
        assert int(r.fetch("block_sizes").astype(np.int64).sum()) == g.n
    rng = np.random.default_rng(5)
    by_size = np.argsort([g.m for g in graphs])
    picks = sorted(set(by_size[:8].tolist()) | set(by_size[-8:].tolist()) |
                   set(rng.integers(0, len(graphs), 16).tolist()))
    for i in picks:
        alone = binding.summarize(ctx(), graphs[i])
        assert_same(rs[i].to_dict(), alone.to_dict(), ("batch vs alone", i, graphs[i].m))
        alone.free()
    small = [i for i in rng.permutation(len(graphs)).tolist() if graphs[i].m <= 20000][:12]
    assert len(small) == 12
    for i in small:
        h = graphs[i].to_host()
        assert_same(rs[i].to_dict(), orc.summarize(h, h.n + 2, True), ("batch vs oracle", i, h.m))
    print("batched: %d graphs, %d edges, max k_done %d, %d checked alone, %d against the oracle"
          % (len(graphs), sum(g.m for g in graphs), max(r.k_done for r in rs), len(picks), len(small)), flush=True)
    for r in rs:
        r.free()
