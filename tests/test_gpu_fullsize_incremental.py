"""GPU parity at the full size of the incremental workload: the resident
R-MAT graph of 2^24 vertices and 2^27 edges (128 types, 64 labels, Zipf 1.1,
k = 4) receives update batches of 10^3, 10^5 and 10^6 operations (ADD / MOD /
DEL 60/25/15, R-MAT endpoints for new edges), applied by bsim_apply_updates
as in the incremental measurement.  The graph is drawn on the GPU (devgen).

* after every batch the incremental result equals a batch bsim_summarize of
  the state's graph, bit for bit (Theorem 2: incremental equals batch), in
  both the frontier form and the plain form (every level recomputed);
* the state's graph holds, for 2,000 sampled vertices (touched by the batch
  or not), the out-rows, types and liveness that the oracle's sequential
  replay of every operation so far gives on the generated graph
  (oracle.updates.replay_rows).
"""

import time

import numpy as np
import pytest

from oracle.updates import replay_rows
from paper_2111_12493_amd import binding, devgen
from paper_2111_12493_amd import graphgen as gg

from gpu_util import assert_same, ctx

pytestmark = pytest.mark.gpu


def state_rows(sg, vs):
    rows, types, alive = {}, {}, {}
    for v in vs:
        a, b = int(sg.row_off[v]), int(sg.row_off[v + 1])
        rows[v] = sorted(zip(sg.lab[a:b].tolist(), sg.tgt[a:b].tolist()))
        types[v] = sorted(sg.types_of(v))
        alive[v] = bool(sg.alive[v]) if sg.alive is not None else True
    return rows, types, alive


@pytest.mark.parametrize("pct", [10, 2, 0])
def test_rmat24_batches_equal_batch_summary(pct):
    dg = devgen.make_device_config("rmat24")
    host = dg.to_host()
    c = ctx()
    old = c.get_option("frontier_limit_pct")
    c.set_option("frontier_limit_pct", pct)
    try:
        st = binding.State(c, dg, 4, stop_at_fixpoint=False)
        done = []  # every operation so far, replayed from the generated graph
        n = host.n
        dead = np.zeros(host.n + 2_000_000, dtype=bool)
        rng = np.random.default_rng(31 + pct)
        for size in (1000, 100000, 1000000):
            d = gg.sample_update_ops(host.row_off, host.tgt, host.lab, n, dead, rng, size, 64, 128,
                                     rmat_scale=24)
            n = int(d["n_after"])
            ops = gg.ops_as_tuples(d)
            inc = st.apply(binding.UpdateBatch.from_op_arrays(d))
            full = binding.summarize(c, binding._Borrowed(st.device_graph()), k_max=4, stop_at_fixpoint=False)
            assert_same(inc.to_dict(), full.to_dict(), ("incremental vs batch", size, pct))
            inc.free()
            full.free()
            sg = st.graph()
            assert sg.n == n
            touched = {int(o[1]) for o in ops if o[0] != "add_v"}
            vs = sorted(set(rng.choice(sorted(touched), 1000).tolist()) | set(rng.integers(0, n, 1000).tolist()))
            done += ops
            want = replay_rows(host, done, vs)
            print("rmat24 pct=%d: batch of %d ops, n=%d, %d sampled rows replayed" % (pct, size, n, len(vs)), flush=True)
            assert state_rows(sg, vs) == want, ("state graph", size, pct)
        st.free()
    finally:
        c.set_option("frontier_limit_pct", old)


def test_rmat24_state_checkpoint(tmp_path):
    # a state saved after a batch of 10^5 operations and loaded again gives
    # the same summary, and the next batch gives the same result on both
    dg = devgen.make_device_config("rmat24")
    host = dg.to_host()
    c = ctx()
    st = binding.State(c, dg, 4, stop_at_fixpoint=False)
    dead = np.zeros(host.n + 2_000_000, dtype=bool)
    rng = np.random.default_rng(77)
    n = host.n
    d = gg.sample_update_ops(host.row_off, host.tgt, host.lab, n, dead, rng, 100000, 64, 128, rmat_scale=24)
    n = int(d["n_after"])
    last = st.apply(binding.UpdateBatch.from_op_arrays(d))
    path = tmp_path / "rmat24.bsim"
    t0 = time.perf_counter()
    st.save(path)
    t1 = time.perf_counter()
    ld = binding.State.load(c, path)
    t2 = time.perf_counter()
    print("rmat24 state file: %.2f GB, save %.2f s, load %.2f s" % (path.stat().st_size / 1e9, t1 - t0, t2 - t1),
          flush=True)
    path.unlink()
    assert_same(ld.result.to_dict(), last.to_dict(), "loaded summary")
    last.free()
    d = gg.sample_update_ops(host.row_off, host.tgt, host.lab, n, dead, rng, 100000, 64, 128, rmat_scale=24)
    batch = binding.UpdateBatch.from_op_arrays(d)
    ra, rb = st.apply(batch), ld.apply(batch)
    assert_same(ra.to_dict(), rb.to_dict(), "next batch")
    ra.free()
    rb.free()
    st.free()
    ld.free()
