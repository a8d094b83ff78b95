"""Seeded synthetic input graphs generated on the GPU with torch.

The full-size workloads (an R-MAT graph of 2^27 vertices and 2^30 edges,
thousands of batched R-MAT graphs, the 2^27-edge resident graph) take
minutes to draw on the host; here the same recipes run as torch operations
on the device in seconds.  Like ``graphgen`` this module only produces
inputs: it holds none of the summarization arithmetic, so the CPU oracle
(through ``to_host``/``induced``) and the HIP library (through ``struct``)
consume the same graphs.  A (recipe, seed) pair names one graph for a given
torch build and GPU model (torch's device generator is counter based).

Recipes (the graph model of ``graphgen``): R-MAT endpoints with recursive
quadrant probabilities (a, b, c, 1-a-b-c), no noise or permutation, self
loops and multi-edges kept; edge labels Zipf(s) over n_labels; per vertex a
type count uniform in [lo, hi] and type ids Zipf(s) over n_types (duplicate
ids may remain, which set semantics ignore).
"""

from __future__ import annotations

import dataclasses
from typing import Optional, Sequence

import numpy as np

from . import graphgen as gg
from .binding import PackedGraph

_CHUNK = 1 << 25


def _torch():
    import torch

    return torch


def _zipf(gen, k: int, s: float, size: int, device) -> "torch.Tensor":
    """``size`` ids from a finite Zipf law on {0..k-1}: P(i) ~ (i+1)^-s."""
    torch = _torch()
    w = 1.0 / torch.arange(1, k + 1, dtype=torch.float64, device=device).pow(s)
    cdf = torch.cumsum(w, 0)
    cdf = cdf / cdf[-1]
    out = torch.empty(size, dtype=torch.int32, device=device)
    for lo in range(0, size, _CHUNK):
        hi = min(size, lo + _CHUNK)
        u = torch.rand(hi - lo, generator=gen, dtype=torch.float64, device=device)
        out[lo:hi] = torch.clamp(torch.searchsorted(cdf, u, right=True), max=k - 1).to(torch.int32)
    return out


def _type_lists(gen, n: int, k: int, s: float, lo: int, hi: int, device):
    torch = _torch()
    cnt = torch.randint(lo, hi + 1, (n,), generator=gen, device=device, dtype=torch.int64)
    off = torch.zeros(n + 1, dtype=torch.int64, device=device)
    torch.cumsum(cnt, 0, out=off[1:])
    total = int(off[-1])
    ids = _zipf(gen, k, s, total, device) if total else torch.zeros(1, dtype=torch.int32, device=device)
    return off, ids


def _rmat_endpoints(gen, scale: int, m: int, a: float, b: float, c: float, device):
    torch = _torch()
    src = torch.empty(m, dtype=torch.int64, device=device)
    dst = torch.empty(m, dtype=torch.int64, device=device)
    ab, abc = a + b, a + b + c
    for lo in range(0, m, _CHUNK):
        hi = min(m, lo + _CHUNK)
        s = torch.zeros(hi - lo, dtype=torch.int64, device=device)
        d = torch.zeros(hi - lo, dtype=torch.int64, device=device)
        for _ in range(scale):
            r = torch.rand(hi - lo, generator=gen, device=device)
            s = s * 2 + (r >= ab).to(torch.int64)
            d = d * 2 + (((r >= a) & (r < ab)) | (r >= abc)).to(torch.int64)
        src[lo:hi] = s
        dst[lo:hi] = d
    return src, dst


@dataclasses.dataclass
class DeviceCSR(PackedGraph):
    """A CSR graph held as torch tensors on the GPU (int32 views of the
    unsigned arrays, int16 labels when ``label_bytes`` is 2)."""

    n: int
    m: int
    row_off: "torch.Tensor"
    tgt: "torch.Tensor"
    lab: "torch.Tensor"
    type_off: "torch.Tensor"
    typ: "torch.Tensor"
    label_bytes: int
    n_labels: int
    n_types: int

    def _make_struct(self):
        from .binding import BsimGraph, MEM_DEVICE

        return BsimGraph(self.n, self.label_bytes, self.m, self.row_off.data_ptr(), self.tgt.data_ptr(),
                         self.lab.data_ptr(), self.type_off.data_ptr(), self.typ.data_ptr(), None,
                         MEM_DEVICE, 0)

    def src(self) -> "torch.Tensor":
        torch = _torch()
        deg = (self.row_off[1:] - self.row_off[:-1]).to(torch.int64)
        return torch.repeat_interleave(torch.arange(self.n, device=self.tgt.device, dtype=torch.int32), deg)

    def to_host(self) -> gg.Graph:
        """The whole graph as a host ``graphgen.Graph``."""
        lab = self.lab.cpu().numpy()
        lab = lab.view(np.uint16) if self.label_bytes == 2 else lab.view(np.uint32)
        return gg.Graph(n=self.n, row_off=self.row_off.cpu().numpy().view(np.uint32).astype(np.uint64),
                        tgt=self.tgt.cpu().numpy().view(np.uint32),
                        lab=lab.astype(np.uint32),
                        typ_off=self.type_off.cpu().numpy().view(np.uint32).astype(np.uint64),
                        typ=self.typ[:max(int(self.type_off[-1]), 0)].cpu().numpy().view(np.uint32),
                        n_labels=self.n_labels, n_types=self.n_types)

    def induced(self, seeds: Sequence[int], depth: int):
        """The part of the graph that fixes h^depth of ``seeds``.

        h^j of a vertex depends on its types, its out-edges and h^{j-1} of
        their targets, so it is fixed by the out-rows of every vertex within
        depth-1 hops of a seed plus the types of every vertex within depth
        hops.  Returns (host ``graphgen.Graph`` on those vertices with rows
        kept only for the first group, ids of the seeds in it); vertices past
        the first group keep no out-edges, so only the seeds' own h^depth is
        meaningful in the subgraph.
        """
        torch = _torch()
        ro = self.row_off
        frontier = torch.unique(torch.as_tensor(list(seeds), dtype=torch.int64, device=ro.device))
        rows = frontier
        for _ in range(depth - 1):
            nxt = self._targets(frontier)
            frontier = torch.unique(nxt)
            rows = torch.unique(torch.cat([rows, frontier]))
        leaves = torch.unique(torch.cat([rows, self._targets(rows)]))
        # row vertices first (their rows kept), then the rest
        is_row = torch.zeros(self.n, dtype=torch.bool, device=ro.device)
        is_row[rows] = True
        rest = leaves[~is_row[leaves]]
        order = torch.cat([rows, rest])
        remap = torch.full((self.n,), -1, dtype=torch.int64, device=ro.device)
        remap[order] = torch.arange(order.numel(), device=ro.device)
        beg = ro[rows].to(torch.int64)
        deg = (ro[rows + 1] - ro[rows]).to(torch.int64)
        eidx = torch.repeat_interleave(beg, deg) + (
            torch.arange(int(deg.sum()), device=ro.device) - torch.repeat_interleave(torch.cumsum(deg, 0) - deg, deg))
        src = torch.repeat_interleave(torch.arange(rows.numel(), device=ro.device), deg)
        dst = remap[self.tgt[eidx].to(torch.int64)]
        lab = self.lab[eidx].to(torch.int64)
        if self.label_bytes == 2:
            lab = lab & 0xFFFF
        toff = self.type_off.to(torch.int64)
        tlen = (toff[order + 1] - toff[order])
        tidx = torch.repeat_interleave(toff[order], tlen) + (
            torch.arange(int(tlen.sum()), device=ro.device) - torch.repeat_interleave(torch.cumsum(tlen, 0) - tlen, tlen))
        typ_off = np.zeros(order.numel() + 1, dtype=np.uint64)
        np.cumsum(tlen.cpu().numpy(), out=typ_off[1:])
        typ = self.typ[tidx].cpu().numpy().view(np.uint32) if tidx.numel() else np.zeros(0, dtype=np.uint32)
        g = gg.from_edges(order.numel(), src.cpu().numpy(), dst.cpu().numpy(), lab.cpu().numpy(),
                          typ_off=typ_off, typ=typ, n_labels=self.n_labels, n_types=self.n_types)
        seed_ids = remap[torch.as_tensor(list(seeds), dtype=torch.int64, device=ro.device)].cpu().numpy()
        return g, seed_ids

    def _targets(self, vs: "torch.Tensor") -> "torch.Tensor":
        torch = _torch()
        ro = self.row_off
        beg = ro[vs].to(torch.int64)
        deg = (ro[vs + 1] - ro[vs]).to(torch.int64)
        if int(deg.sum()) == 0:
            return vs[:0]
        eidx = torch.repeat_interleave(beg, deg) + (
            torch.arange(int(deg.sum()), device=ro.device) - torch.repeat_interleave(torch.cumsum(deg, 0) - deg, deg))
        return self.tgt[eidx].to(torch.int64)


def rmat_device(scale: int, m: int, n_types: int, n_labels: int, types_lo: int = 0, types_hi: int = 4,
                s_types: float = 1.1, s_labels: float = 1.1, a: float = 0.57, b: float = 0.19,
                c: float = 0.19, seed: int = 2, label_u16: bool = False, n: Optional[int] = None,
                device: str = "cuda") -> DeviceCSR:
    """R-MAT graph on 2^scale vertices (or the first ``n`` of them, drawing
    again for edges with an endpoint >= n), built on the GPU."""
    torch = _torch()
    gen = torch.Generator(device=device)
    gen.manual_seed(seed)
    full = n is None
    n = (1 << scale) if full else int(n)
    if m >= 1 << 31 or n >= 1 << 31 or n > 1 << scale:
        raise ValueError("int32 offsets: at most 2^31 - 1 edges and vertices, n <= 2^scale")
    if full:
        src, dst = _rmat_endpoints(gen, scale, m, a, b, c, device)
    else:
        parts, have = [], 0
        while have < m:
            s, d = _rmat_endpoints(gen, scale, int((m - have) * 1.3) + 64, a, b, c, device)
            keep = (s < n) & (d < n)
            parts.append((s[keep], d[keep]))
            have += int(keep.sum())
        src = torch.cat([p[0] for p in parts])[:m]
        dst = torch.cat([p[1] for p in parts])[:m]
    order = torch.sort(src, stable=True).indices
    tgt = dst[order].to(torch.int32)
    if m == 0:
        tgt = torch.zeros(1, dtype=torch.int32, device=device)
    del dst
    counts = torch.bincount(src, minlength=n)
    del src, order
    row_off = torch.zeros(n + 1, dtype=torch.int64, device=device)
    torch.cumsum(counts, 0, out=row_off[1:])
    lab = _zipf(gen, n_labels, s_labels, max(m, 1), device)
    lab = lab.to(torch.int16) if label_u16 else lab
    toff, typ = _type_lists(gen, n, n_types, s_types, types_lo, types_hi, device)
    return DeviceCSR(n=n, m=m, row_off=row_off.to(torch.int32), tgt=tgt, lab=lab,
                     type_off=toff.to(torch.int32), typ=typ, label_bytes=2 if label_u16 else 4,
                     n_labels=n_labels, n_types=n_types)


# Full-size named recipes (the host ``graphgen.CONFIGS`` hold the others).
def uniform_device(n: int, m: int, n_types: int, n_labels: int, types_lo: int = 1, types_hi: int = 3,
                   s_types: float = 1.0, s_labels: float = 1.0, seed: int = 1, label_u16: bool = False,
                   device: str = "cuda") -> DeviceCSR:
    """Uniform random directed graph built on the GPU: endpoints i.i.d.
    uniform, a self loop's target moved to the next vertex."""
    torch = _torch()
    gen = torch.Generator(device=device)
    gen.manual_seed(seed)
    if m >= 1 << 31 or n >= 1 << 31 or n < 2:
        raise ValueError("int32 offsets: at most 2^31 - 1 edges and vertices, at least 2 vertices")
    src = torch.randint(0, n, (m,), generator=gen, device=device, dtype=torch.int64)
    dst = torch.randint(0, n, (m,), generator=gen, device=device, dtype=torch.int64)
    dst = torch.where(dst == src, (dst + 1) % n, dst)
    order = torch.sort(src, stable=True).indices
    tgt = dst[order].to(torch.int32)
    del dst
    counts = torch.bincount(src, minlength=n)
    del src, order
    row_off = torch.zeros(n + 1, dtype=torch.int64, device=device)
    torch.cumsum(counts, 0, out=row_off[1:])
    lab = _zipf(gen, n_labels, s_labels, max(m, 1), device)
    lab = lab.to(torch.int16) if label_u16 else lab
    toff, typ = _type_lists(gen, n, n_types, s_types, types_lo, types_hi, device)
    return DeviceCSR(n=n, m=m, row_off=row_off.to(torch.int32), tgt=tgt, lab=lab,
                     type_off=toff.to(torch.int32), typ=typ, label_bytes=2 if label_u16 else 4,
                     n_labels=n_labels, n_types=n_types)


def batched_recipe(count: int, max_edges: float, seed: int):
    """(m, n, scale, seed) of each graph of the batched workload: edges
    log-uniform in [10^2, max_edges], average degree uniform in [4, 16]."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(count):
        m = int(round(10 ** rng.uniform(2, np.log10(max_edges))))
        n = max(2, int(round(m / rng.uniform(4, 16))))
        out.append((m, n, max(1, int(np.ceil(np.log2(n)))), int(rng.integers(1, 1 << 30))))
    return out


def batched_device(count: int, max_edges: float = 1e6, seed: int = 23, device: str = "cuda"):
    """The batched workload: ``count`` R-MAT graphs with 32 types (0-3 per
    vertex) and 32 edge labels, Zipf 1.0."""
    return [rmat_device(scale, m, n_types=32, n_labels=32, types_lo=0, types_hi=3, s_types=1.0, s_labels=1.0,
                        seed=gs, n=n, device=device) for m, n, scale, gs in batched_recipe(count, max_edges, seed)]


DEVICE_CONFIGS = {
    # R-MAT scale 27, 2^30 edges, 1,024 types (0-4 per vertex) and 256 edge
    # labels, Zipf 1.2, labels stored as uint16.
    "rmat27": dict(scale=27, m=1 << 30, n_types=1024, n_labels=256, types_lo=0, types_hi=4,
                   s_types=1.2, s_labels=1.2, seed=27, label_u16=True),
    # R-MAT scale 24, 2^27 edges, 128 types, 64 labels, Zipf 1.1 (the resident
    # base graph of the incremental / serving workload).
    "rmat24": dict(scale=24, m=1 << 27, n_types=128, n_labels=64, types_lo=0, types_hi=4,
                   s_types=1.1, s_labels=1.1, seed=5),
    # Uniform random graph of the same size (2^24 vertices, 2^27 edges, 128
    # types, 64 labels): without hubs, an update's change reaches few
    # vertices per level, the case incremental maintenance is made for.
    "uniform24": dict(kind="uniform", n=1 << 24, m=1 << 27, n_types=128, n_labels=64, types_lo=0, types_hi=4,
                      s_types=1.1, s_labels=1.1, seed=6),
}


def make_device_config(name: str, seed: Optional[int] = None, device: str = "cuda") -> DeviceCSR:
    cfg = dict(DEVICE_CONFIGS[name])
    if seed is not None:
        cfg["seed"] = seed
    if cfg.pop("kind", "rmat") == "uniform":
        return uniform_device(device=device, **cfg)
    return rmat_device(device=device, **cfg)
