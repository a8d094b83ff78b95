"""Write oracle digests for full-size workloads (tests/golden/<name>.json).

Runs only the CPU oracle (oracle/) on graphs from the input generator, so
every stored value comes from the oracle.  The full fixpoint run of the
rmat22_chains workload takes the single-threaded oracle one to two hours.

    python tests/golden/make_digests.py rmat22_chains [k_max]
"""

import hashlib
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

from oracle import oracle as orc  # noqa: E402
from paper_2111_12493_amd import graphgen as gg  # noqa: E402


def digest(a: np.ndarray) -> str:
    return hashlib.sha256(np.ascontiguousarray(a).tobytes()).hexdigest()


def result_digests(r) -> dict:
    return {
        "k_done": int(r["k_done"]), "fixpoint": int(r["fixpoint"]), "n_blocks": int(r["n_blocks"]),
        "n_summary_edges": int(len(r["se_src"])),
        "blocks_per_iter_sha256": digest(np.asarray(r["blocks_per_iter"], dtype=np.uint32)),
        "blocks_per_iter_head": [int(x) for x in r["blocks_per_iter"][:8]],
        "blocks_per_iter_tail": [int(x) for x in r["blocks_per_iter"][-4:]],
        "hashes_sha256": digest(np.asarray(r["hashes"], dtype=np.uint64)),
        "block_ids_sha256": digest(np.asarray(r["block_ids"], dtype=np.uint32)),
        "block_sizes_sha256": digest(np.asarray(r["block_sizes"], dtype=np.uint32)),
        "summary_edges_sha256": digest(np.stack([r["se_src"], r["se_label"], r["se_dst"]]).astype(np.uint32)),
    }


def main():
    name = sys.argv[1]
    k_max = int(sys.argv[2]) if len(sys.argv) > 2 else None
    g = gg.make_config(name)
    t0 = time.time()
    if k_max is None:
        r = orc.summarize(g, g.n + 2, True)
        tag = "fixpoint"
    else:
        r = orc.summarize(g, k_max, False)
        tag = "k%d" % k_max
    out = {"workload": name, "run": tag, "vertices": g.n, "edges": g.m,
           "oracle_seconds": round(time.time() - t0, 1), **result_digests(r)}
    path = os.path.join(HERE, "%s_%s.json" % (name, tag))
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print("wrote", path)


if __name__ == "__main__":
    main()
