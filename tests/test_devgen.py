"""The device graph generator (torch; run here on the CPU) and its induced
subgraphs: the oracle's h^j of a seed vertex on the subgraph that
DeviceCSR.induced cuts out must equal its h^j on the whole graph, which is
what lets the full-size GPU tests check sampled vertices against the oracle."""

import numpy as np
import pytest

from oracle import oracle as orc
from paper_2111_12493_amd import devgen


@pytest.fixture(scope="module")
def small():
    return devgen.rmat_device(scale=11, m=1 << 14, n_types=16, n_labels=300, types_lo=0, types_hi=3,
                              s_types=1.2, s_labels=1.2, seed=3, label_u16=True, device="cpu")


def test_csr_is_well_formed(small):
    g = small.to_host()
    assert g.n == 1 << 11 and g.m == 1 << 14
    assert g.row_off[0] == 0 and g.row_off[-1] == g.m and np.all(np.diff(g.row_off.astype(np.int64)) >= 0)
    assert g.tgt.max() < g.n and g.lab.max() < 300 and g.typ.max() < 16
    cnt = np.diff(g.typ_off.astype(np.int64))
    assert cnt.min() >= 0 and cnt.max() <= 3
    # R-MAT skew: the lowest ids carry the most out-edges
    deg = np.diff(g.row_off.astype(np.int64))
    assert deg[:64].mean() > 4 * deg.mean()


def test_same_seed_same_graph(small):
    again = devgen.rmat_device(scale=11, m=1 << 14, n_types=16, n_labels=300, types_lo=0, types_hi=3,
                               s_types=1.2, s_labels=1.2, seed=3, label_u16=True, device="cpu")
    a, b = small.to_host(), again.to_host()
    for f in ("row_off", "tgt", "lab", "typ_off", "typ"):
        assert np.array_equal(getattr(a, f), getattr(b, f)), f


@pytest.mark.parametrize("depth", [1, 2, 3])
def test_induced_subgraph_fixes_seed_hashes(small, depth):
    g = small.to_host()
    full, _ = orc.iterate(g, depth)
    rng = np.random.default_rng(depth)
    deg = np.diff(g.row_off.astype(np.int64))
    seeds = sorted(set(rng.integers(0, g.n, 24).tolist()) | {int(np.argmax(deg)), int(np.argmin(deg))})
    sub, ids = small.induced(seeds, depth)
    assert sub.n < g.n or depth == 3
    part, _ = orc.iterate(sub, depth)
    assert np.array_equal(part[ids], full[np.array(seeds)])


def test_induced_keeps_too_little_for_deeper_levels(small):
    # planted check on the method itself: one level deeper than the cut
    # no longer agrees for some seed (the subgraph is not the whole graph)
    g = small.to_host()
    full, _ = orc.iterate(g, 3)
    deg = np.diff(g.row_off.astype(np.int64))
    seeds = [int(v) for v in np.argsort(-deg)[:8]]
    sub, ids = small.induced(seeds, 1)
    part, _ = orc.iterate(sub, 3)
    assert not np.array_equal(part[ids], full[np.array(seeds)])
