"""GPU parity of the previous-level summary edges (BSIM_PREV_LEVEL_EDGES:
Sec. 2.6's vertex summaries, whose edges lead to the targets' classes of the
previous level) through the C ABI, against the oracle bit for bit, plus a
full-size check on the R-MAT refinement workload from two forward runs."""

import ctypes

import numpy as np
import pytest

from oracle import oracle as orc
from paper_2111_12493_amd import binding
from paper_2111_12493_amd import graphgen as gg

from gpu_util import assert_same, ctx

pytestmark = pytest.mark.gpu
UNB = binding.K_UNBOUNDED


def check_prev(g, k_max, stop=False, untyped=False, labels=None, host_input=False, u16=False, what=""):
    kk = k_max if k_max != UNB else g.n + 2
    if labels is None:
        ref = orc.summarize(g, kk, stop, untyped, prev_level_edges=True)
    else:
        ref = orc.summarize_ext(g, kk, stop, untyped, "out", labels, prev_level_edges=True)
    src = gg.with_u16_labels(g) if u16 else g
    graph = binding.HostGraph(src) if host_input else binding.DeviceGraph(src)
    r = binding.summarize(ctx(), graph, k_max=k_max, stop_at_fixpoint=stop, untyped=untyped, labels=labels,
                          prev_level_edges=True)
    gpu = r.to_dict()
    r.free()
    assert_same(gpu, ref, (what, k_max, stop, labels))
    return gpu, ref


def test_closed_forms():
    for L in (1, 6, 40):
        for k in (0, 1, 3, L):
            gpu, _ = check_prev(gg.chain(L), k, untyped=True, what="chain")
            if 1 <= k <= L:
                got = list(zip(gpu["se_src"].tolist(), gpu["se_label"].tolist(), gpu["se_dst"].tolist()))
                assert got == [(j, 0, j) for j in range(k)], (L, k)
    for n in (1, 2, 9):
        check_prev(gg.cycle(n, marked=True), 3, what="marked cycle")
    for D in (1, 4):
        check_prev(gg.binary_tree(D), 2, untyped=True, what="tree")
        check_prev(gg.binary_tree(D), UNB, stop=True, untyped=True, what="tree fixpoint")


def test_random_small_graphs():
    rng = np.random.default_rng(404)
    for trial in range(40):
        n = int(rng.integers(1, 60))
        g = gg.random_small_graph(rng, n, int(rng.integers(0, 5 * n)), 4, 4, 3,
                                  p_alive=1.0 if trial % 3 else 0.8)
        k = int(rng.integers(0, 7))
        labels = [0, 2, 3] if trial % 4 == 1 else None
        check_prev(g, k, stop=bool(trial % 5 == 0), untyped=bool(trial % 2), labels=labels,
                   host_input=bool(trial % 2), u16=bool(trial % 3 == 0), what=("random", trial))


@pytest.mark.parametrize("k", [1, 3, 8])
def test_rmat_graph_with_chains(k):
    # R-MAT part plus chains: at a cap the previous-level edges differ from
    # the quotient edges; hubs and tiles both take part
    g = gg.rmat_graph(15, 1 << 18, n_types=32, n_labels=16, seed=13)
    check_prev(g, k, u16=True, what="rmat15")
    check_prev(g, k, labels=list(range(0, 16, 3)), what="rmat15 filtered")


def test_combinations_that_are_refused():
    g = gg.rmat_graph(10, 1 << 12, n_types=4, n_labels=4, seed=2)
    for direction in ("in", "both"):
        with pytest.raises(binding.BsimError) as e:
            binding.summarize(ctx(), binding.DeviceGraph(g), k_max=3, stop_at_fixpoint=False,
                              direction=direction, prev_level_edges=True)
        assert e.value.status == binding.E_INVALID
    gs = binding.HostGraph(g).struct()
    params = binding.BsimParams(3, binding.PREV_LEVEL_EDGES)
    out = ctypes.POINTER(binding.BsimResult)()
    st = ctypes.c_void_p()
    rc = binding.lib().bsim_summarize(ctx().handle, ctypes.byref(gs), ctypes.byref(params), ctypes.byref(st),
                                      ctypes.byref(out))
    assert rc == binding.E_UNSUPPORTED and not st.value and not out
    arr = (binding.BsimGraph * 1)(gs)
    outs = (ctypes.POINTER(binding.BsimResult) * 1)()
    rc = binding.lib().bsim_batch_summarize(ctx().handle, arr, 1, ctypes.byref(params), outs)
    assert rc == binding.E_UNSUPPORTED
    # the context still works
    check_prev(g, 3, what="after refusals")


def test_rmat22_chains_at_a_cap():
    # the R-MAT refinement workload (2^22 vertices, 2^25 edges, 64 chains of
    # 2,000 edges) capped at k = 5, where it is far from its fixpoint: the
    # triples must be (block_5(v), l, block_4(w)) with both block arrays from
    # the forward path (held to the oracle by the full-size tests)
    g = gg.make_config("rmat22_chains")
    dg = binding.DeviceGraph(g)

    def run(k, prev):
        r = binding.summarize(ctx(), dg, k_max=k, stop_at_fixpoint=False, prev_level_edges=prev)
        d = r.to_dict()
        r.free()
        return d

    a = run(5, True)
    b5, b4 = run(5, False), run(4, False)
    for key in ("k_done", "hashes", "block_ids", "blocks_per_iter", "block_sizes"):
        assert np.array_equal(np.asarray(a[key]), np.asarray(b5[key])), key
    deg = (g.row_off[1:] - g.row_off[:-1]).astype(np.int64)
    src = np.repeat(np.arange(g.n, dtype=np.int64), deg)
    key = (b5["block_ids"].astype(np.int64)[src] << 40) | (g.lab.astype(np.int64) << 32) | \
        b4["block_ids"].astype(np.int64)[g.tgt.astype(np.int64)]
    want = np.unique(key)
    got = (a["se_src"].astype(np.int64) << 40) | (a["se_label"].astype(np.int64) << 32) | \
        a["se_dst"].astype(np.int64)
    print("rmat22_chains k=5: %d blocks, %d previous-level edges, %d quotient edges" %
          (a["n_blocks"], len(got), len(b5["se_src"])), flush=True)
    assert np.array_equal(got, want)
