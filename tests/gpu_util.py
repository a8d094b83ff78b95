"""Helpers shared by the GPU parity tests: run the HIP path through the
C ABI and the oracle on the same graph, and compare every output."""

import numpy as np

from oracle import oracle as orc
from paper_2111_12493_amd import binding

_ctx = None


def ctx():
    global _ctx
    if _ctx is None:
        _ctx = binding.Context(0)
    return _ctx


def gpu_summarize(g, k_max, stop=True, untyped=False, host_input=False, edges=True):
    graph = binding.HostGraph(g) if host_input else binding.DeviceGraph(g)
    r = binding.summarize(ctx(), graph, k_max=k_max, stop_at_fixpoint=stop, untyped=untyped,
                          summary_edges=edges)
    d = r.to_dict()
    d["n_iter_launches"] = r.n_iter_launches
    d["ms_iterate"] = r.ms_iterate
    r.free()
    return d


def assert_same(gpu, ref, what="", edges=True):
    assert gpu["k_done"] == ref["k_done"], (what, gpu["k_done"], ref["k_done"])
    assert gpu["fixpoint"] == ref["fixpoint"], what
    assert np.array_equal(gpu["blocks_per_iter"], ref["blocks_per_iter"]), what
    assert np.array_equal(gpu["hashes"], ref["hashes"]), what
    assert np.array_equal(gpu["block_ids"], ref["block_ids"]), what
    assert gpu["n_blocks"] == ref["n_blocks"], what
    assert np.array_equal(gpu["block_sizes"], ref["block_sizes"]), what
    if edges:
        for f in ("se_src", "se_label", "se_dst"):
            assert np.array_equal(gpu[f], ref[f]), (what, f)


def check(g, k_max, stop=True, untyped=False, what="", **kw):
    ref = orc.summarize(g, k_max if k_max != binding.K_UNBOUNDED else g.n + 2, stop, untyped)
    gpu = gpu_summarize(g, k_max, stop, untyped, **kw)
    assert_same(gpu, ref, what)
    return gpu, ref
