"""GPU change detection from two snapshots (bsim_diff_snapshots) against
the oracle's diff (the same ordered batch, op for op), and round trips:
the diff applied to a resident state of the earlier snapshot gives the
summary of the later one, bit for bit (Theorem 2 on the GPU path)."""

import numpy as np
import pytest

from oracle import updates as upd
from paper_2111_12493_amd import binding
from paper_2111_12493_amd import graphgen as gg

from gpu_util import ctx

pytestmark = pytest.mark.gpu


def pair(rng, n, m, n_ops, n_labels=3, n_types=3):
    g = gg.random_small_graph(rng, n, m, n_labels, n_types, 2)
    return g, upd.apply_ops(g, gg.ops_as_tuples(gg.update_ops(g, rng, n_ops)))


def test_random_pairs_match_the_oracle():
    rng = np.random.default_rng(211)
    for trial in range(60):
        n = int(rng.integers(1, 50))
        before, after = pair(rng, n, int(rng.integers(0, 4 * n + 1)), int(rng.integers(0, 50)))
        want = upd.diff_snapshots(before, after)
        u16 = trial % 4 == 0
        mk = binding.HostGraph if trial % 3 == 0 else binding.DeviceGraph
        b = mk(gg.with_u16_labels(before) if u16 else before)
        a = mk(gg.with_u16_labels(after) if u16 else after)
        assert binding.diff_snapshots(ctx(), b, a) == want, trial
        assert binding.diff_snapshots(ctx(), a, a) == []


def test_invalid_pairs_are_rejected():
    a = gg.from_edges(2, [], [], [], alive=np.array([1, 0], dtype=np.uint8))
    for before, after in ((a, gg.from_edges(2, [], [], [])), (gg.from_edges(3, [], [], []), gg.from_edges(2, [], [], []))):
        with pytest.raises(binding.BsimError) as err:
            binding.diff_snapshots(ctx(), binding.DeviceGraph(before), binding.DeviceGraph(after))
        assert err.value.status == binding.E_INVALID


def test_rmat_round_trip_through_the_incremental_path():
    rng = np.random.default_rng(17)
    g = gg.rmat_graph(14, 1 << 17, n_types=16, n_labels=8, seed=21)
    after = upd.apply_ops(g, gg.ops_as_tuples(gg.update_ops(g, rng, 3000, rmat_scale=14)))
    ops = binding.diff_snapshots(ctx(), binding.DeviceGraph(g), binding.DeviceGraph(after))
    assert ops == upd.diff_snapshots(g, after)
    st = binding.State(ctx(), binding.DeviceGraph(g), 4)
    st.result.free()
    r = st.apply(binding.UpdateBatch(ops))
    got = r.to_dict()
    r.free()
    st.free()
    ref = binding.summarize(ctx(), binding.DeviceGraph(after), k_max=4, stop_at_fixpoint=False)
    want = ref.to_dict()
    ref.free()
    for key in ("k_done", "n_blocks", "hashes", "block_ids", "blocks_per_iter", "block_sizes", "se_src",
                "se_label", "se_dst"):
        assert np.array_equal(np.asarray(got[key]), np.asarray(want[key])), key


def test_large_state_snapshots():
    # a 2^23-edge R-MAT state after one batch of 10^5 operations: the diff of
    # the two snapshots, applied to a second state of the first snapshot,
    # gives the same summary as the batch itself
    from paper_2111_12493_amd import devgen

    dg = devgen.rmat_device(20, 1 << 23, n_types=64, n_labels=32, seed=44)
    g = dg.to_host()
    rng = np.random.default_rng(45)
    dead = np.zeros(g.n + 200000, dtype=bool)
    d = gg.sample_update_ops(g.row_off, g.tgt, g.lab, g.n, dead, rng, 100000, 32, 64, rmat_scale=20)
    s1 = binding.State(ctx(), dg, 3, summary_edges=False)
    s1.result.free()
    r1 = s1.apply(binding.UpdateBatch.from_op_arrays(d))
    ops = binding.diff_snapshots(ctx(), dg, s1.device_graph())
    kinds = {k: sum(1 for o in ops if o[0] == k) for k in ("add_v", "mod_v", "del_e", "add_e", "del_v")}
    print("2^23-edge snapshots: %d ops %s" % (len(ops), kinds), flush=True)
    s2 = binding.State(ctx(), dg, 3, summary_edges=False)
    s2.result.free()
    r2 = s2.apply(binding.UpdateBatch(ops))
    a, b = r1.to_dict(), r2.to_dict()
    r1.free()
    r2.free()
    s1.free()
    s2.free()
    for key in ("n_blocks", "hashes", "block_ids", "blocks_per_iter", "block_sizes"):
        assert np.array_equal(np.asarray(a[key]), np.asarray(b[key])), key
