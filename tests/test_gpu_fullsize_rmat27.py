"""GPU parity at the full size of the large R-MAT workload: 2^27 vertices,
2^30 edges, 1,024 types and 256 edge labels (Zipf 1.2, uint16 labels), run
to the fixpoint capped at k = 64, in the launch configuration of the
benchmark (one plain bsim_summarize call on the device-resident graph).

The graph comes from the counter-based generator (graphgen.cb_rmat_graph),
so the host here draws the same graph that the oracle summarized once in
full: tests/golden/rmat27_fixpoint_cap64.json holds the oracle's k_done,
fixpoint, per-level block counts and the SHA-256 of its final and previous
hashes, block ids, block sizes and sorted summary edges (written by
tests/golden/make_digests.py, which calls only the oracle).  Every one of
them must match bit for bit.
"""

import hashlib
import json
import os

import numpy as np
import pytest

from paper_2111_12493_amd import binding
from paper_2111_12493_amd import graphgen as gg

from gpu_util import ctx

pytestmark = pytest.mark.gpu
GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "rmat27_fixpoint_cap64.json")


def sha(*rows, dtype):
    h = hashlib.sha256()
    for a in rows:
        h.update(np.ascontiguousarray(a, dtype=dtype).data)
    return h.hexdigest()


def test_fixpoint_matches_oracle_digests():
    with open(GOLD) as f:
        want = json.load(f)
    g = gg.make_config("rmat27")
    assert (g.n, g.m) == (want["vertices"], want["edges"])
    dg = binding.DeviceGraph(g)
    del g
    print("rmat27: graph on the device", flush=True)
    r = binding.summarize(ctx(), dg, k_max=64, stop_at_fixpoint=True)
    got = r.to_dict()
    r.free()
    print("rmat27 fixpoint: k_done=%d fixpoint=%d blocks=%d summary edges=%d"
          % (got["k_done"], got["fixpoint"], got["n_blocks"], len(got["se_src"])), flush=True)
    assert got["k_done"] == want["k_done"] and got["fixpoint"] == want["fixpoint"]
    assert got["n_blocks"] == want["n_blocks"]
    assert len(got["se_src"]) == want["n_summary_edges"]
    assert sha(got["blocks_per_iter"], dtype=np.uint32) == want["blocks_per_iter_sha256"]
    assert sha(got["hashes"], dtype=np.uint64) == want["hashes_sha256"]
    assert sha(got["block_ids"], dtype=np.uint32) == want["block_ids_sha256"]
    assert sha(got["block_sizes"], dtype=np.uint32) == want["block_sizes_sha256"]
    assert sha(got["se_src"], got["se_label"], got["se_dst"], dtype=np.uint32) == want["summary_edges_sha256"]
    del got
    # the previous level's hashes: a run capped one level lower
    if want["k_done"] >= 1:
        r = binding.summarize(ctx(), dg, k_max=want["k_done"] - 1, stop_at_fixpoint=False, summary_edges=False)
        prev = r.to_dict()
        r.free()
        assert sha(prev["hashes"], dtype=np.uint64) == want["prev_hashes_sha256"]
