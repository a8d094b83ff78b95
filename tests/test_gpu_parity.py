"""GPU parity: the HIP path (through the C ABI) against the CPU oracle,
bit-exact on hashes, block ids, per-iteration block counts, block sizes and
summary edges.  Integer work, so the bar is exact equality."""

import numpy as np
import pytest

from oracle import oracle as orc
from paper_2111_12493_amd import binding
from paper_2111_12493_amd import graphgen as gg

from gpu_util import check, ctx, gpu_summarize, assert_same

pytestmark = pytest.mark.gpu
UNB = binding.K_UNBOUNDED


def test_paper_example_and_fig1():
    for untyped in (False, True):
        for k in (0, 1, 2, 5):
            check(gg.paper_example(), k, stop=False, untyped=untyped, what=("paper", untyped, k))
        check(gg.paper_example(), UNB, untyped=untyped)
    gpu, _ = check(gg.paper_example(), 2, stop=False, untyped=True)
    assert list(gpu["block_ids"]) == [0, 1, 2, 2]
    for after in (False, True):
        check(gg.fig1_scenario(after), 1, stop=False)


def test_hash_spec_vectors():
    # the frozen hash-spec vectors (HASH_SPEC.md), independent of the oracle
    import hash_vectors

    v = hash_vectors.load()
    g = hash_vectors.graph(v)
    for k, want in ((0, v["t"]), (1, v["h1"]), (2, v["h2"])):
        gpu = gpu_summarize(g, k, stop=False)
        assert [int(x) for x in gpu["hashes"]] == want, k
    gpu = gpu_summarize(g, 0, stop=False, untyped=True)
    assert [int(x) for x in gpu["hashes"]] == [v["t({})"]] * g.n


@pytest.mark.parametrize("L", [1, 7, 300])
def test_chain_closed_form(L):
    gpu, _ = check(gg.chain(L), UNB, untyped=True)
    assert gpu["k_done"] == L + 1
    assert list(gpu["blocks_per_iter"]) == [min(k + 1, L + 1) for k in range(L + 2)]


def test_cycles_stars_trees():
    for n in (1, 2, 9):
        check(gg.cycle(n), UNB)
        check(gg.cycle(n, marked=True), n + 3, stop=False)
    check(gg.out_star(9), UNB, untyped=True)
    for D in (1, 3, 6):
        check(gg.binary_tree(D), UNB, untyped=True)


def test_empty_and_edgeless():
    check(gg.from_edges(0, [], [], []), UNB)
    check(gg.from_edges(1, [], [], [], types=[[3]]), UNB)
    check(gg.from_edges(600, [], [], [], types=[[i % 5] for i in range(600)]), UNB)


def test_random_small_graphs():
    rng = np.random.default_rng(101)
    for trial in range(120):
        n = int(rng.integers(1, 60))
        g = gg.random_small_graph(rng, n, int(rng.integers(0, 5 * n + 1)),
                                  int(rng.integers(1, 5)), int(rng.integers(1, 5)), 3,
                                  p_alive=1.0 if trial % 3 else 0.75)
        stop = trial % 4 != 0
        k = UNB if stop else int(rng.integers(0, 6))
        check(g, k, stop=stop, untyped=bool(trial % 5 == 0), what=("random", trial))


def test_uniform_10k_50k():
    g = gg.make_config("uniform_10k_50k")
    gpu, ref = check(g, 10, stop=True, what="uniform_10k_50k")
    assert gpu["fixpoint"] == ref["fixpoint"]


def test_host_and_device_inputs_agree():
    g = gg.make_config("uniform_10k_50k")
    a = gpu_summarize(g, 10, host_input=True)
    b = gpu_summarize(g, 10, host_input=False)
    assert_same(a, b)


def _hub_graph(seed, degs, n_extra=3000, n_labels=7, dup_every=5):
    """Vertices 0..len(degs)-1 have the given out-degrees (hubs when > 1024),
    with repeated triples every `dup_every` edges; the rest is sparse."""
    rng = np.random.default_rng(seed)
    n = len(degs) + n_extra
    src, dst, lab = [], [], []
    for v, d in enumerate(degs):
        t = rng.integers(0, n, size=d)
        l = rng.integers(0, n_labels, size=d)
        t[::dup_every] = t[0]
        l[::dup_every] = l[0]
        src.append(np.full(d, v))
        dst.append(t)
        lab.append(l)
    m2 = 4 * n_extra
    src.append(rng.integers(len(degs), n, size=m2))
    dst.append(rng.integers(0, n, size=m2))
    lab.append(rng.integers(0, n_labels, size=m2))
    types = [[int(x)] for x in rng.integers(0, 3, size=n)]
    return gg.from_edges(n, np.concatenate(src), np.concatenate(dst), np.concatenate(lab),
                         types=types, n_labels=n_labels)


def test_hub_vertices():
    # degrees around the tile limit, the solo-hub limit (3072) and well above
    # it (several buckets)
    g = _hub_graph(7, [1023, 1024, 1025, 2046, 2047, 2048, 2049, 3071, 3072, 3073, 3100, 5000, 20000, 70000])
    check(g, UNB, what="hubs")
    check(g, 3, stop=False, untyped=True, what="hubs untyped")


def test_hub_with_more_than_256_chunks():
    # one hub of 600,000 edges: its bucket keys span more than one batch of runs
    g = _hub_graph(8, [600_000, 3000], n_extra=20000, n_labels=5, dup_every=3)
    check(g, 4, stop=False, what="600k hub")


def test_hub_bucket_resplit():
    # a tiny hub table forces buckets to overflow and re-split by more bits
    c = ctx()
    old = c.get_option("hub_table_slots")
    try:
        c.set_option("hub_table_slots", 64)
        g = _hub_graph(9, [30000, 4000, 1500], n_extra=4000, n_labels=9, dup_every=4)
        check(g, UNB, what="resplit")
    finally:
        c.set_option("hub_table_slots", old)


def test_hub_with_few_distinct_keys():
    # a hub whose 50,000 edges carry only 3 distinct (label, target-class) pairs
    n = 50005
    src = np.zeros(50000, dtype=np.int64)
    dst = 1 + (np.arange(50000) % 3)
    lab = np.zeros(50000, dtype=np.int64)
    g = gg.from_edges(n, src, dst, lab, types=[[0]] + [[1]] * (n - 1))
    check(g, UNB, what="low-distinct hub")


def test_ragged_tiles_and_u16_labels():
    rng = np.random.default_rng(5)
    # long runs of zero-degree vertices, single huge-but-tiled vertices, u16 labels
    degs = np.zeros(5000, dtype=np.int64)
    degs[rng.integers(0, 5000, 300)] = rng.integers(1, 1025, 300)
    degs[::997] = 1024
    degs[5::1499] = 2047  # the largest degree that still fits one tile
    src = np.repeat(np.arange(5000), degs)
    dst = rng.integers(0, 5000, size=src.size)
    lab = rng.integers(0, 40000, size=src.size)
    g = gg.from_edges(5000, src, dst, lab, types=[[int(x)] for x in rng.integers(0, 4, 5000)],
                      n_labels=40000)
    check(g, UNB, what="ragged u32")
    check(gg.with_u16_labels(g), UNB, what="ragged u16")


def test_rmat_with_chains_reduced():
    g = gg.rmat_graph(14, 1 << 17, n_types=64, n_labels=16, seed=9)
    g = gg.append_chains(g, 4, 60, type_id=64)
    gpu, ref = check(g, UNB, what="rmat14 chains")
    assert gpu["k_done"] >= 61


def test_determinism():
    g = gg.rmat_graph(13, 1 << 16, n_types=16, n_labels=8, seed=3)
    a = gpu_summarize(g, UNB)
    for _ in range(3):
        assert_same(gpu_summarize(g, UNB), a)


def test_invalid_inputs_are_rejected():
    g = gg.from_edges(3, [0, 1], [1, 2], [0, 0])
    bad = gg.Graph(**{**g.__dict__, "tgt": np.array([1, 7], dtype=np.uint32)})
    with pytest.raises(binding.BsimError) as e:
        gpu_summarize(bad, 3)
    assert e.value.status == binding.E_RANGE
    bad = gg.Graph(**{**g.__dict__, "row_off": np.array([0, 2, 1, 2], dtype=np.uint64)})
    with pytest.raises(binding.BsimError) as e:
        gpu_summarize(bad, 3)
    assert e.value.status == binding.E_INVALID
    dead = gg.Graph(**{**g.__dict__, "alive": np.array([1, 1, 0], dtype=np.uint8)})
    with pytest.raises(binding.BsimError) as e:
        gpu_summarize(dead, 3)
    assert e.value.status == binding.E_INVALID
    # the context still works after errors
    check(g, UNB)
