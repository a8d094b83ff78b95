"""GPU parity at the benchmark's full size (R-MAT 2^22 vertices / 2^25 edges
plus 64 chains of 2,000 edges), in the launch configuration bench.py times.

* k = 3 without the fixpoint test: every output compared with the oracle
  element by element.
* the full run to the fixpoint (2,001 iterations): digests of every output
  compared with the oracle's (tests/golden, written by make_digests.py), and
  the chains' closed form checked directly.
"""

import hashlib
import json
import os

import numpy as np
import pytest

from oracle import oracle as orc
from paper_2111_12493_amd import binding
from paper_2111_12493_amd import graphgen as gg

from gpu_util import assert_same, gpu_summarize

pytestmark = pytest.mark.gpu
GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
_graph = {}


def rmat22():
    if "g" not in _graph:
        _graph["g"] = gg.make_config("rmat22_chains")
    return _graph["g"]


def _sha(a):
    return hashlib.sha256(np.ascontiguousarray(a).tobytes()).hexdigest()


def test_full_size_three_iterations_match_oracle():
    g = rmat22()
    ref = orc.summarize(g, 3, False)
    gpu = gpu_summarize(g, 3, stop=False)
    assert_same(gpu, ref, "rmat22_chains k=3")


def test_full_size_fixpoint():
    g = rmat22()
    gpu = gpu_summarize(g, binding.K_UNBOUNDED)
    bpi = np.asarray(gpu["blocks_per_iter"], dtype=np.int64)
    # the 64 identical chains of 2,000 edges add exactly one class per level
    # until level 2,000; the fixpoint is therefore level 2,001
    assert gpu["k_done"] == 2001 and gpu["fixpoint"] == 1
    assert np.all(np.diff(bpi)[100:2000] == 1) and bpi[-1] == bpi[-2]
    assert int(np.sum(gpu["block_sizes"])) == g.n
    path = os.path.join(GOLD, "rmat22_chains_fixpoint.json")
    if not os.path.exists(path):
        pytest.skip("oracle digests for the fixpoint run not generated")
    ref = json.load(open(path))
    assert gpu["k_done"] == ref["k_done"] and gpu["n_blocks"] == ref["n_blocks"]
    assert _sha(bpi.astype(np.uint32)) == ref["blocks_per_iter_sha256"]
    assert _sha(gpu["hashes"]) == ref["hashes_sha256"]
    assert _sha(gpu["block_ids"]) == ref["block_ids_sha256"]
    assert _sha(gpu["block_sizes"]) == ref["block_sizes_sha256"]
    se = np.stack([gpu["se_src"], gpu["se_label"], gpu["se_dst"]]).astype(np.uint32)
    assert _sha(se) == ref["summary_edges_sha256"]
