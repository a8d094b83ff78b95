"""GPU parity of batched summarization (bsim_batch_summarize): every graph's
result from one batched run equals the oracle's summary of that graph alone,
bit for bit, whatever the other graphs of the batch are."""

import numpy as np
import pytest

from oracle import oracle as orc
from paper_2111_12493_amd import binding
from paper_2111_12493_amd import graphgen as gg

from gpu_util import assert_same, ctx, gpu_summarize

pytestmark = pytest.mark.gpu
UNB = binding.K_UNBOUNDED


def run_batch(graphs, k_max=UNB, stop=True, untyped=False, host=False, on_host=False):
    gs = [binding.HostGraph(g) if host else binding.DeviceGraph(g) for g in graphs]
    rs = binding.batch_summarize(ctx(), gs, k_max=k_max, stop_at_fixpoint=stop, untyped=untyped,
                                 result_on_host=on_host)
    out = [r.to_dict() for r in rs]
    for r in rs:
        r.free()
    return out


def check_batch(graphs, k_max=UNB, stop=True, untyped=False, **kw):
    got = run_batch(graphs, k_max, stop, untyped, **kw)
    assert len(got) == len(graphs)
    for i, (g, r) in enumerate(zip(graphs, got)):
        ref = orc.summarize(g, k_max if k_max != UNB else g.n + 2, stop, untyped)
        assert_same(r, ref, ("graph", i))
    return got


def mixed_graphs(seed, count):
    rng = np.random.default_rng(seed)
    out = []
    for i in range(count):
        kind = i % 5
        if kind == 0:
            out.append(gg.random_small_graph(rng, int(rng.integers(1, 40)), int(rng.integers(0, 120)), 3, 3, 2,
                                             p_alive=1.0 if i % 3 else 0.8))
        elif kind == 1:
            out.append(gg.chain(int(rng.integers(1, 30))))
        elif kind == 2:
            out.append(gg.cycle(int(rng.integers(1, 12)), marked=bool(i % 2)))
        elif kind == 3:
            out.append(gg.from_edges(0, [], [], []))
        else:
            out.append(gg.rmat_graph(8, int(rng.integers(100, 3000)), n_types=8, n_labels=4, seed=int(i)))
    return out


def test_batch_equals_each_graph_alone():
    graphs = mixed_graphs(41, 60)
    check_batch(graphs)
    check_batch(graphs, k_max=3, stop=False)
    check_batch(graphs, k_max=5, stop=True, untyped=True)


def test_batch_of_one_and_host_inputs():
    g = gg.make_config("uniform_10k_50k")
    check_batch([g], k_max=10)
    check_batch(mixed_graphs(43, 12), host=True, on_host=True)


def test_batch_with_hubs_and_long_chain():
    # graphs stop at very different levels; hubs share the hub launches
    rng = np.random.default_rng(47)
    hub = gg.from_edges(6000, np.zeros(5000, dtype=np.int64), rng.integers(0, 6000, 5000),
                        rng.integers(0, 5, 5000), types=[[int(x)] for x in rng.integers(0, 3, 6000)])
    graphs = [gg.chain(300), hub, gg.rmat_graph(12, 1 << 15, n_types=16, n_labels=8, seed=3), gg.chain(2)]
    check_batch(graphs)


def test_batch_equals_single_gpu_calls():
    graphs = mixed_graphs(53, 30)
    got = run_batch(graphs)
    for g, r in zip(graphs, got):
        assert_same(r, gpu_summarize(g, UNB))


def test_batch_rejects_bad_graph():
    good = gg.chain(3)
    bad = gg.Graph(**{**good.__dict__, "tgt": np.array([1, 2, 9], dtype=np.uint32)})
    with pytest.raises(binding.BsimError) as e:
        run_batch([good, bad])
    assert e.value.status == binding.E_RANGE
    check_batch([good, good])
