"""bsim_summarize_noalloc (no device allocation, scratch in a static device
array) against bsim_summarize: bit-identical results on consecutive calls,
the second one smaller, so nothing of a call's scratch may leak into the
next; oversized graphs are refused with the caller's arrays untouched."""

import numpy as np
import pytest

from paper_2111_12493_amd import binding
from paper_2111_12493_amd import graphgen as gg

from gpu_util import assert_same, ctx, gpu_summarize

pytestmark = pytest.mark.gpu
UNB = binding.K_UNBOUNDED


def compare(g, k_max=UNB, stop=True, untyped=False, edges=True, what=""):
    dg = binding.DeviceGraph(g)
    got = binding.summarize_noalloc(ctx(), dg, k_max=k_max, stop_at_fixpoint=stop, untyped=untyped,
                                    summary_edges=edges)
    ref = gpu_summarize(g, k_max, stop, untyped, edges=edges)
    assert_same(got, ref, what, edges=edges)
    assert 0 < got["scratch_used"] <= lib_scratch()
    print("%s: n=%d m=%d k_done=%d scratch %.1f MiB" % (what, g.n, g.m, got["k_done"],
                                                       got["scratch_used"] / 2 ** 20), flush=True)
    return got


def lib_scratch():
    return int(binding.lib().bsim_noalloc_scratch_bytes())


def test_two_calls_in_a_row_second_smaller():
    big = gg.append_chains(gg.rmat_graph(15, 1 << 20, n_types=64, n_labels=16, seed=8), 4, 300, type_id=64)
    small = gg.rmat_graph(10, 6000, n_types=8, n_labels=4, seed=9)
    compare(big, what="first call (R-MAT scale 15 with chains, hubs)")
    compare(small, what="second call (smaller)")
    compare(small, k_max=3, stop=False, untyped=True, edges=False, what="third call (capped, untyped, no edges)")


def test_hub_and_empty_graphs():
    star = gg.out_star(9000)                       # one hub of 9,000 edges: the hub-bucket path
    compare(star, what="out-star hub")
    compare(gg.from_edges(0, [], [], []), what="empty graph")
    compare(gg.from_edges(50, [], [], [], types=[[i % 3] for i in range(50)]), what="edgeless graph")


def test_oversized_graph_is_refused_untouched():
    import torch

    g = gg.uniform_graph(3_000_000, 6_000_000, 4, 4, seed=2)
    dg = binding.DeviceGraph(g)
    marker = torch.full((g.n,), 7, dtype=torch.int32, device="cuda")
    o = binding.BsimNoallocOut()
    hashes = torch.zeros(g.n, dtype=torch.int64, device="cuda")
    bsz = torch.zeros(g.n, dtype=torch.int32, device="cuda")
    se = [torch.zeros(g.m, dtype=torch.int32, device="cuda") for _ in range(3)]
    bpi = np.zeros(g.n + 2, dtype=np.uint32)
    o.hashes, o.block_ids, o.block_sizes = hashes.data_ptr(), marker.data_ptr(), bsz.data_ptr()
    o.se_src, o.se_label, o.se_dst = (t.data_ptr() for t in se)
    o.blocks_per_iter, o.blocks_per_iter_cap = bpi.ctypes.data, bpi.size
    params = binding.BsimParams(UNB, binding.STOP_AT_FIXPOINT)
    gs = dg.struct()
    import ctypes

    rc = binding.lib().bsim_summarize_noalloc(ctx().handle, ctypes.byref(gs), ctypes.byref(params), ctypes.byref(o))
    assert rc == binding.E_UNSUPPORTED
    assert bool((marker == 7).all())
    # and the entry point still works afterwards
    compare(gg.rmat_graph(9, 3000, n_types=4, n_labels=4, seed=3), what="after a refusal")
