"""GPU parity of the persistent small-graph launch of batched summarization
(bsim_small.hip) and of the batched-schedule autotuner.

With the schedule forced (ctx option batch_small_edges), every graph of a
batch that fits one workgroup (at most 1,024 vertices and 1,535 edges) is
refined to its own stop level inside LDS, the rest by the union's
launches; every graph's result must equal the oracle's summary of it alone,
bit for bit, with the launch on and off, next to large graphs, with deep
fixpoints (chains of up to 1,000 edges), caps with and without the fixpoint
test, dead vertices, untyped runs and 16-bit labels, and at the capacity
boundary."""

import numpy as np
import pytest

from oracle import oracle as orc
from paper_2111_12493_amd import binding
from paper_2111_12493_amd import graphgen as gg

from gpu_util import assert_same

pytestmark = pytest.mark.gpu
UNB = binding.K_UNBOUNDED


def run(ctx, graphs, k_max=UNB, stop=True, untyped=False):
    gs = [binding.DeviceGraph(g) for g in graphs]
    rs = binding.batch_summarize(ctx, gs, k_max=k_max, stop_at_fixpoint=stop, untyped=untyped)
    out = [r.to_dict() for r in rs]
    for r in rs:
        r.free()
    return out


def check(ctx, graphs, k_max=UNB, stop=True, untyped=False, what=""):
    got = run(ctx, graphs, k_max, stop, untyped)
    for i, (g, r) in enumerate(zip(graphs, got)):
        ref = orc.summarize(g, k_max if k_max != UNB else g.n + 2, stop, untyped)
        assert_same(r, ref, (what, i))
    return got


def small_and_large(seed):
    rng = np.random.default_rng(seed)
    out = []
    for i in range(48):
        kind = i % 6
        if kind == 0:
            out.append(gg.random_small_graph(rng, int(rng.integers(1, 200)), int(rng.integers(0, 600)), 4, 3, 3,
                                             p_alive=1.0 if i % 4 else 0.7))
        elif kind == 1:
            out.append(gg.chain(int(rng.integers(1, 1000))))
        elif kind == 2:
            out.append(gg.cycle(int(rng.integers(1, 300)), marked=bool(i % 2)))
        elif kind == 3:
            out.append(gg.from_edges(int(rng.integers(0, 5)), [], [], []))
        elif kind == 4:
            out.append(gg.rmat_graph(8, int(rng.integers(100, 1500)), n_types=8, n_labels=4, seed=int(i)))
        else:
            # too large for one workgroup: the union's launches
            out.append(gg.rmat_graph(12, int(rng.integers(3000, 20000)), n_types=8, n_labels=4, seed=int(i)))
    return out


@pytest.mark.parametrize("small_edges", [0, 10 ** 9])
def test_forced_schedules_equal_the_oracle(small_edges):
    ctx = binding.Context(0)
    ctx.set_option("batch_small_edges", small_edges)
    graphs = small_and_large(71)
    check(ctx, graphs, what="fixpoint")
    check(ctx, graphs, k_max=3, stop=False, what="k=3")
    check(ctx, graphs, k_max=7, stop=True, untyped=True, what="untyped, capped")
    check(ctx, graphs, k_max=0, stop=False, what="k=0")
    assert ctx.get_option("batch_small_edges") == small_edges
    ctx.close()


def test_capacity_boundary_and_u16_labels():
    ctx = binding.Context(0)
    ctx.set_option("batch_small_edges", 10 ** 9)
    rng = np.random.default_rng(5)

    def rand_graph(n, m):
        return gg.from_edges(n, rng.integers(0, n, m), rng.integers(0, n, m), rng.integers(0, 6, m),
                             types=[[int(x)] for x in rng.integers(0, 4, n)])

    # at the capacity (1,024 vertices, 1,535 edges), and one past it each way
    graphs = [rand_graph(1024, 1535), rand_graph(1025, 1535), rand_graph(1024, 1536), gg.chain(1000),
              rand_graph(2, 1535), rand_graph(1024, 0)]
    check(ctx, graphs, what="boundary")
    check(ctx, [gg.with_u16_labels(g) for g in graphs], what="u16 labels")
    ctx.close()


def test_all_graphs_small():
    # every graph refined by the persistent launch: the run ends without
    # any refinement launch doing work
    ctx = binding.Context(0)
    ctx.set_option("batch_small_edges", 10 ** 9)
    rng = np.random.default_rng(9)
    graphs = [gg.random_small_graph(rng, int(rng.integers(1, 60)), int(rng.integers(0, 200)), 3, 3, 2)
              for _ in range(300)] + [gg.chain(700)]
    check(ctx, graphs, what="all small")
    check(ctx, graphs, k_max=4, stop=False, what="all small, k=4")
    ctx.close()


def test_autotuner_picks_and_caches_a_schedule():
    ctx = binding.Context(0)
    assert ctx.get_option("autotune") == 1
    graphs = small_and_large(73)
    first = check(ctx, graphs, what="tuned, first call")
    picked = (ctx.get_option("batch_small_edges"), ctx.get_option("batch_hub_table_slots"))
    assert picked[1] in (4096, 16384)
    second = check(ctx, graphs, what="tuned, cached")
    assert (ctx.get_option("batch_small_edges"), ctx.get_option("batch_hub_table_slots")) == picked
    for a, b in zip(first, second):
        assert_same(a, b, "same schedule, same result")
    ctx.close()
