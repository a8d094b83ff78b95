"""The context's kept work buffer (ctx option keep_work): summarize and
batched calls give the oracle's results whether the temporaries come from
the buffer, from the pool, or from both (a call that outgrows the buffer
takes the rest from the pool and grows it for the next call)."""

import numpy as np
import pytest

from oracle import oracle as orc
from paper_2111_12493_amd import binding
from paper_2111_12493_amd import graphgen as gg

from gpu_util import assert_same

pytestmark = pytest.mark.gpu
UNB = binding.K_UNBOUNDED


def graphs_of_growing_then_shrinking_size():
    return [gg.uniform_graph(500, 2000, 6, 6, seed=1),
            gg.rmat_graph(12, 30000, n_types=16, n_labels=8, seed=2),   # outgrows the first call's buffer
            gg.uniform_graph(300, 900, 4, 4, seed=3),                   # fits the grown buffer
            gg.rmat_graph(13, 60000, n_types=16, n_labels=8, seed=4),
            gg.chain(50)]


@pytest.mark.parametrize("keep", [1, 0])
def test_summaries_with_and_without_the_kept_buffer(keep):
    ctx = binding.Context(0)
    assert ctx.get_option("keep_work") == 1
    ctx.set_option("keep_work", keep)
    assert ctx.get_option("keep_work") == keep
    for i, g in enumerate(graphs_of_growing_then_shrinking_size()):
        ref = orc.summarize(g, g.n + 2, True)
        for rep in range(2):
            r = binding.summarize(ctx, binding.DeviceGraph(g), k_max=UNB)
            got = r.to_dict()
            r.free()
            assert_same(got, ref, ("graph", i, "call", rep, "keep_work", keep))
    ctx.close()


def test_batched_calls_share_the_buffer_with_single_calls():
    ctx = binding.Context(0)
    rng = np.random.default_rng(8)
    small = [gg.random_small_graph(rng, int(rng.integers(1, 40)), int(rng.integers(0, 120)), 3, 3, 2)
             for _ in range(20)]
    big = gg.rmat_graph(13, 50000, n_types=8, n_labels=4, seed=5)
    refs = [orc.summarize(g, g.n + 2, True) for g in small]
    for rep in range(3):
        rs = binding.batch_summarize(ctx, [binding.DeviceGraph(g) for g in small])
        for i, r in enumerate(rs):
            assert_same(r.to_dict(), refs[i], ("batch", rep, "graph", i))
            r.free()
        # a larger single call between the batches grows the buffer
        r = binding.summarize(ctx, binding.DeviceGraph(big), k_max=UNB)
        assert_same(r.to_dict(), orc.summarize(big, big.n + 2, True), ("single", rep))
        r.free()
    # switching the buffer off releases it; later calls use the pool
    ctx.set_option("keep_work", 0)
    rs = binding.batch_summarize(ctx, [binding.DeviceGraph(g) for g in small])
    for i, r in enumerate(rs):
        assert_same(r.to_dict(), refs[i], ("after release", i))
        r.free()
    ctx.close()


def test_option_range_and_server_refusal():
    ctx = binding.Context(0)
    for bad in (-1, 2):
        with pytest.raises(binding.BsimError) as e:
            ctx.set_option("keep_work", bad)
        assert e.value.status == binding.E_RANGE
    ctx.close()
    srv = binding.Server(0, workers=1)
    with pytest.raises(binding.BsimError) as e:
        srv.set_option("keep_work", 1)
    assert e.value.status == binding.E_UNSUPPORTED
    srv.free()
