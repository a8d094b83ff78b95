"""Write oracle digests for full-size workloads (tests/golden/<name>_<run>.json).

Runs only the CPU oracle (oracle/) on graphs from the input generator, so
every stored value comes from the oracle.  The full fixpoint run of the
rmat22_chains workload takes the single-threaded oracle one to two hours;
the 2^30-edge rmat27 workload (fixpoint capped at k = 64) needs about 45 GB
of host memory.

    python tests/golden/make_digests.py rmat22_chains            # to the fixpoint
    python tests/golden/make_digests.py rmat27 --k-max 64        # fixpoint, capped
    python tests/golden/make_digests.py NAME --k-max K --no-stop # exactly K levels
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


def digest_rows(*rows) -> str:
    """SHA-256 of the uint32 rows stacked in order (np.stack(rows) bytes),
    without building the stack."""
    h = hashlib.sha256()
    for a in rows:
        h.update(np.ascontiguousarray(a, dtype=np.uint32).data)
    return h.hexdigest()


def result_digests(r) -> dict:
    return {
        "k_done": int(r["k_done"]), "fixpoint": int(r["fixpoint"]), "n_blocks": int(r["n_blocks"]),
        "n_summary_edges": int(len(r["se_src"])),
        "blocks_per_iter_sha256": digest(np.asarray(r["blocks_per_iter"], dtype=np.uint32)),
        "blocks_per_iter_head": [int(x) for x in r["blocks_per_iter"][:8]],
        "blocks_per_iter_tail": [int(x) for x in r["blocks_per_iter"][-4:]],
        "hashes_sha256": digest(np.asarray(r["hashes"], dtype=np.uint64)),
        "prev_hashes_sha256": digest(np.asarray(r["prev_hashes"], dtype=np.uint64)),
        "block_ids_sha256": digest(np.asarray(r["block_ids"], dtype=np.uint32)),
        "block_sizes_sha256": digest(np.asarray(r["block_sizes"], dtype=np.uint32)),
        "summary_edges_sha256": digest_rows(r["se_src"], r["se_label"], r["se_dst"]),
    }


def main():
    import argparse

    ap = argparse.ArgumentParser()
    ap.add_argument("name")
    ap.add_argument("--k-max", type=int, default=None)
    ap.add_argument("--no-stop", action="store_true")
    args = ap.parse_args()
    g = gg.make_config(args.name)
    t0 = time.time()
    if args.k_max is None:
        r = orc.summarize(g, g.n + 2, True)
        tag = "fixpoint"
    elif args.no_stop:
        r = orc.summarize(g, args.k_max, False)
        tag = "k%d" % args.k_max
    else:
        r = orc.summarize(g, args.k_max, True)
        tag = "fixpoint_cap%d" % args.k_max
    out = {"workload": args.name, "run": tag, "vertices": g.n, "edges": g.m,
           "oracle_seconds": round(time.time() - t0, 1), **result_digests(r)}
    path = os.path.join(HERE, "%s_%s.json" % (args.name, tag))
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print("wrote", path)


if __name__ == "__main__":
    main()
