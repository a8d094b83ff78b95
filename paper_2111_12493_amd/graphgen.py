"""Seeded synthetic input graphs for k-bisimulation summarization.

This module only *produces inputs*: labeled directed graphs in CSR form with a
type (vertex-label) list per vertex.  It holds none of the summarization
arithmetic, so both the CPU oracle and the HIP path can consume the same
graphs.  Every generator takes an explicit seed and uses numpy's PCG64
generator, so a (config, seed) pair names one graph on every machine running
the same numpy.

Graph model (Sec. 2.2, labeled property graphs): directed edges (v, l, w) with
one edge label l each; a vertex carries a *set* of vertex labels ("types"),
possibly empty.  Multi-edges, duplicate triples and duplicate type ids are
allowed in the input; the method has set semantics so they never change a
result (they exercise the de-duplication).

Workload shapes (stand-ins for the paper's LUBM/BSBM/DyLDO data, which are not
available): uniform random graphs, R-MAT power-law graphs with Zipf-skewed
type and edge-label alphabets, and long directed chains that force many
refinement iterations (long k-chaining, Sec. 3.3).
"""

from __future__ import annotations

import dataclasses
from typing import List, Optional, Sequence, Tuple

import numpy as np


@dataclasses.dataclass
class Graph:
    """A labeled directed graph in CSR form (host numpy arrays).

    row_off[v]..row_off[v+1] index the out-edges of v in ``tgt``/``lab``;
    typ_off[v]..typ_off[v+1] index v's type ids in ``typ``.  ``alive`` is None
    (all vertices alive) or a uint8 mask; dead vertices must have no incident
    edges.
    """

    n: int
    row_off: np.ndarray  # uint64 [n+1]
    tgt: np.ndarray      # uint32 [m]
    lab: np.ndarray      # uint32 [m]
    typ_off: np.ndarray  # uint64 [n+1]
    typ: np.ndarray      # uint32 [sum |types|]
    alive: Optional[np.ndarray] = None  # uint8 [n] or None
    n_labels: int = 0
    n_types: int = 0

    @property
    def m(self) -> int:
        return int(self.tgt.shape[0])

    def src(self) -> np.ndarray:
        """Source vertex of every edge (expanded from the CSR offsets)."""
        deg = np.diff(self.row_off).astype(np.int64)
        return np.repeat(np.arange(self.n, dtype=np.uint32), deg)

    def types_of(self, v: int) -> List[int]:
        return [int(x) for x in self.typ[int(self.typ_off[v]):int(self.typ_off[v + 1])]]

    def out_edges(self, v: int) -> List[Tuple[int, int]]:
        a, b = int(self.row_off[v]), int(self.row_off[v + 1])
        return [(int(self.lab[e]), int(self.tgt[e])) for e in range(a, b)]


def from_edges(n: int, src, dst, lab, types: Optional[Sequence[Sequence[int]]] = None,
               typ_off=None, typ=None, alive=None, n_labels: int = 0,
               n_types: int = 0) -> Graph:
    """Build a CSR graph from an edge list.

    Edges keep their relative input order within a source (stable sort), so
    the CSR is a deterministic function of the edge list.
    """
    src = np.asarray(src, dtype=np.int64).reshape(-1)
    dst = np.asarray(dst, dtype=np.int64).reshape(-1)
    lab = np.asarray(lab, dtype=np.int64).reshape(-1)
    if not (src.shape == dst.shape == lab.shape):
        raise ValueError("src, dst, lab must have equal length")
    if src.size and (src.min() < 0 or src.max() >= n or dst.min() < 0 or dst.max() >= n):
        raise ValueError("edge endpoint out of range")
    order = np.argsort(src, kind="stable")
    counts = np.bincount(src, minlength=n).astype(np.uint64)
    row_off = np.zeros(n + 1, dtype=np.uint64)
    np.cumsum(counts, out=row_off[1:])
    if types is not None:
        lens = np.array([len(t) for t in types], dtype=np.uint64)
        typ_off = np.zeros(n + 1, dtype=np.uint64)
        np.cumsum(lens, out=typ_off[1:])
        flat = [int(x) for t in types for x in t]
        typ = np.array(flat, dtype=np.uint32)
    elif typ_off is None:
        typ_off = np.zeros(n + 1, dtype=np.uint64)
        typ = np.zeros(0, dtype=np.uint32)
    g = Graph(n=n, row_off=row_off, tgt=dst[order].astype(np.uint32),
              lab=lab[order].astype(np.uint32),
              typ_off=np.asarray(typ_off, dtype=np.uint64),
              typ=np.asarray(typ, dtype=np.uint32),
              alive=None if alive is None else np.asarray(alive, dtype=np.uint8),
              n_labels=int(n_labels) if n_labels else (int(lab.max()) + 1 if lab.size else 0),
              n_types=int(n_types))
    if g.n_types == 0 and g.typ.size:
        g.n_types = int(g.typ.max()) + 1
    return g


# ---------------------------------------------------------------------------
# Samplers
# ---------------------------------------------------------------------------

def zipf_sample(rng: np.random.Generator, k: int, s: float, size: int) -> np.ndarray:
    """Draw ``size`` ids from a finite Zipf law on {0..k-1}: P(i) ~ (i+1)^-s."""
    w = 1.0 / np.power(np.arange(1, k + 1, dtype=np.float64), s)
    cdf = np.cumsum(w)
    cdf /= cdf[-1]
    u = rng.random(size)
    out = np.searchsorted(cdf, u, side="right")
    return np.minimum(out, k - 1).astype(np.uint32)


def zipf_type_lists(rng: np.random.Generator, n: int, k: int, s: float,
                    lo: int, hi: int) -> Tuple[np.ndarray, np.ndarray]:
    """Per-vertex type lists: count uniform in {lo..hi}, ids Zipf(k, s).

    Ids are drawn without replacement where a few redraws manage it; any
    duplicate left over stays in the list (set semantics make it harmless and
    it exercises the type de-duplication).
    """
    cnt = rng.integers(lo, hi + 1, size=n).astype(np.int64)
    total = int(cnt.sum())
    ids = zipf_sample(rng, k, s, total).astype(np.int64)
    off = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(cnt, out=off[1:])
    owner = np.repeat(np.arange(n, dtype=np.int64), cnt)
    for _ in range(4):
        key = owner * (k + 1) + ids
        order = np.lexsort((np.arange(total), key))
        dup = np.zeros(total, dtype=bool)
        ks = key[order]
        dup[order[1:]] = ks[1:] == ks[:-1]
        nd = int(dup.sum())
        if nd == 0:
            break
        ids[dup] = zipf_sample(rng, k, s, nd)
    return off.astype(np.uint64), ids.astype(np.uint32)


def rmat_edges(rng: np.random.Generator, scale: int, m: int, a: float, b: float,
               c: float, chunk: int = 1 << 24) -> Tuple[np.ndarray, np.ndarray]:
    """R-MAT edge endpoints (Chakrabarti et al.): ``scale`` recursive quadrant
    choices with probabilities (a, b, c, 1-a-b-c); no noise, no permutation."""
    src = np.zeros(m, dtype=np.uint32)
    dst = np.zeros(m, dtype=np.uint32)
    ab, abc = a + b, a + b + c
    for lo in range(0, m, chunk):
        hi = min(m, lo + chunk)
        s = np.zeros(hi - lo, dtype=np.uint32)
        d = np.zeros(hi - lo, dtype=np.uint32)
        for _ in range(scale):
            r = rng.random(hi - lo, dtype=np.float32)
            ubit = (r >= ab).astype(np.uint32)
            vbit = ((r >= a) & (r < ab)) | (r >= abc)
            s = (s << 1) | ubit
            d = (d << 1) | vbit.astype(np.uint32)
        src[lo:hi] = s
        dst[lo:hi] = d
    return src, dst


# ---------------------------------------------------------------------------
# Workload graphs
# ---------------------------------------------------------------------------

def uniform_graph(n: int, m: int, n_types: int, n_labels: int, types_lo: int = 1,
                  types_hi: int = 3, s_types: float = 1.0, s_labels: float = 1.0,
                  seed: int = 1, self_loops: bool = False) -> Graph:
    """Uniform random directed labeled graph: endpoints i.i.d. uniform
    (resampled while u == w unless self loops are allowed)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    src = rng.integers(0, n, size=m, dtype=np.int64)
    dst = rng.integers(0, n, size=m, dtype=np.int64)
    if not self_loops:
        bad = src == dst
        while bad.any():
            dst[bad] = rng.integers(0, n, size=int(bad.sum()), dtype=np.int64)
            bad = src == dst
    lab = zipf_sample(rng, n_labels, s_labels, m)
    typ_off, typ = zipf_type_lists(rng, n, n_types, s_types, types_lo, types_hi)
    return from_edges(n, src, dst, lab, typ_off=typ_off, typ=typ,
                      n_labels=n_labels, n_types=n_types)


def rmat_graph(scale: int, m: int, n_types: int, n_labels: int, types_lo: int = 0,
               types_hi: int = 4, s_types: float = 1.1, s_labels: float = 1.1,
               a: float = 0.57, b: float = 0.19, c: float = 0.19,
               seed: int = 2, n: Optional[int] = None) -> Graph:
    """R-MAT graph on 2^scale vertices (or the first ``n`` of them, rejecting
    edges with an endpoint >= n); self loops and duplicate edges are kept."""
    rng = np.random.Generator(np.random.PCG64(seed))
    nv = (1 << scale) if n is None else int(n)
    if n is None:
        src, dst = rmat_edges(rng, scale, m, a, b, c)
    else:
        src_l, dst_l, have = [], [], 0
        while have < m:
            want = int((m - have) * 1.3) + 64
            s, d = rmat_edges(rng, scale, want, a, b, c)
            keep = (s < nv) & (d < nv)
            s, d = s[keep], d[keep]
            src_l.append(s)
            dst_l.append(d)
            have += s.size
        src = np.concatenate(src_l)[:m]
        dst = np.concatenate(dst_l)[:m]
    lab = zipf_sample(rng, n_labels, s_labels, m)
    typ_off, typ = zipf_type_lists(rng, nv, n_types, s_types, types_lo, types_hi)
    return from_edges(nv, src, dst, lab, typ_off=typ_off, typ=typ,
                      n_labels=n_labels, n_types=n_types)


def append_chains(g: Graph, n_chains: int, length: int, type_id: int,
                  label: int = 0) -> Graph:
    """Append ``n_chains`` disjoint directed chains of ``length`` edges
    (length+1 vertices each).  Chain vertices carry the single type
    ``type_id`` and every chain edge has ``label``; the chains force the
    refinement to run at least length+1 iterations to reach its fixpoint."""
    n0 = g.n
    per = length + 1
    nv = n0 + n_chains * per
    base = n0 + np.arange(n_chains, dtype=np.int64)[:, None] * per
    step = np.arange(length, dtype=np.int64)[None, :]
    csrc = (base + step).reshape(-1)
    cdst = csrc + 1
    src = np.concatenate([g.src().astype(np.int64), csrc])
    dst = np.concatenate([g.tgt.astype(np.int64), cdst])
    lab = np.concatenate([g.lab.astype(np.int64), np.full(csrc.size, label, dtype=np.int64)])
    t_lens = np.concatenate([np.diff(g.typ_off).astype(np.int64),
                             np.ones(n_chains * per, dtype=np.int64)])
    typ_off = np.zeros(nv + 1, dtype=np.uint64)
    np.cumsum(t_lens, out=typ_off[1:])
    typ = np.concatenate([g.typ, np.full(n_chains * per, type_id, dtype=np.uint32)])
    return from_edges(nv, src, dst, lab, typ_off=typ_off, typ=typ,
                      n_labels=max(g.n_labels, label + 1),
                      n_types=max(g.n_types, type_id + 1))


def with_u16_labels(g: Graph) -> Graph:
    """Same graph with labels stored as uint16 (alphabets of <= 65536 labels)."""
    if g.lab.size and int(g.lab.max()) > 0xFFFF:
        raise ValueError("labels do not fit in 16 bits")
    return dataclasses.replace(g, lab=g.lab.astype(np.uint16))


# ---------------------------------------------------------------------------
# Counter-based generator (cbgen.c) for the largest workload
# ---------------------------------------------------------------------------

_cb = None


def _cbgen():
    """The compiled counter-based generator (built on first use if absent)."""
    global _cb
    if _cb is None:
        import ctypes
        import os

        from . import build as _build

        if not os.path.exists(_build.CBGEN_LIB) or \
                os.path.getmtime(_build.CBGEN_LIB) < os.path.getmtime(_build.CBGEN_SRC):
            _build.build_cbgen()
        L = ctypes.CDLL(_build.CBGEN_LIB)
        u64, u32, i32, dbl, p = ctypes.c_uint64, ctypes.c_uint32, ctypes.c_int, ctypes.c_double, ctypes.c_void_p
        L.cb_philox_out.argtypes = [u32, u32, u32, u32, u32, u32, p]
        L.cb_philox_out.restype = None
        L.cb_rmat_edges.argtypes = [u64, u32, u64, dbl, dbl, dbl, u32, dbl, p, p, p, i32]
        L.cb_rmat_edges.restype = i32
        L.cb_csr.argtypes = [u32, u64, p, p, p, i32, p, p, p]
        L.cb_csr.restype = i32
        L.cb_type_counts.argtypes = [u64, u32, u32, u32, p]
        L.cb_type_counts.restype = None
        L.cb_type_ids.argtypes = [u64, u32, u32, dbl, p, p]
        L.cb_type_ids.restype = i32
        L.cb_threads.argtypes = []
        L.cb_threads.restype = i32
        _cb = L
    return _cb


def philox4x32_10(counter: Sequence[int], key: Sequence[int]) -> Tuple[int, int, int, int]:
    """One block of the Philox4x32-10 generator that cb_rmat_graph draws from."""
    out = np.zeros(4, dtype=np.uint32)
    _cbgen().cb_philox_out(*[int(c) & 0xFFFFFFFF for c in counter], *[int(k) & 0xFFFFFFFF for k in key],
                           out.ctypes.data)
    return tuple(int(x) for x in out)


def cb_rmat_graph(scale: int, m: int, n_types: int, n_labels: int, types_lo: int = 0, types_hi: int = 4,
                  s_types: float = 1.1, s_labels: float = 1.1, a: float = 0.57, b: float = 0.19,
                  c: float = 0.19, seed: int = 27, label_u16: bool = False) -> Graph:
    """R-MAT graph on 2^scale vertices from the counter-based generator
    (cbgen.c): the same recipe as rmat_graph, with every random draw a pure
    function of (seed, item), so the graph is identical on every host and
    for any thread count.  Edge labels are uint16 when ``label_u16``."""
    L = _cbgen()
    n = 1 << scale
    src = np.empty(max(m, 1), dtype=np.uint32)
    dst = np.empty(max(m, 1), dtype=np.uint32)
    lab = np.empty(max(m, 1), dtype=np.uint16 if label_u16 else np.uint32)
    if L.cb_rmat_edges(seed, scale, m, a, b, c, n_labels, s_labels, src.ctypes.data, dst.ctypes.data,
                       lab.ctypes.data, 1 if label_u16 else 0) != 0:
        raise MemoryError("generator out of memory")
    row_off = np.empty(n + 1, dtype=np.uint64)
    tgt = np.empty(max(m, 1), dtype=np.uint32)
    lab_csr = np.empty_like(lab)
    rc = L.cb_csr(n, m, src.ctypes.data, dst.ctypes.data, lab.ctypes.data, lab.itemsize, row_off.ctypes.data,
                  tgt.ctypes.data, lab_csr.ctypes.data)
    del src, dst, lab
    if rc != 0:
        raise MemoryError("CSR build failed (%d)" % rc)
    cnt = np.empty(n, dtype=np.uint32)
    L.cb_type_counts(seed, n, types_lo, types_hi, cnt.ctypes.data)
    typ_off = np.zeros(n + 1, dtype=np.uint64)
    np.cumsum(cnt, out=typ_off[1:])
    del cnt
    typ = np.empty(max(int(typ_off[-1]), 1), dtype=np.uint32)
    if L.cb_type_ids(seed, n, n_types, s_types, typ_off.ctypes.data, typ.ctypes.data) != 0:
        raise MemoryError("generator out of memory")
    return Graph(n=n, row_off=row_off, tgt=tgt[:m], lab=lab_csr[:m], typ_off=typ_off, typ=typ[:int(typ_off[-1])],
                 n_labels=n_labels, n_types=n_types)


# ---------------------------------------------------------------------------
# Named workloads
# ---------------------------------------------------------------------------

CONFIGS = {
    # 10,000 vertices, 50,000 uniform edges, 1-3 types of 8 (Zipf 1.0),
    # 16 edge labels (Zipf 1.0), no self loops.
    "uniform_10k_50k": dict(kind="uniform", n=10_000, m=50_000, n_types=8, n_labels=16,
                            types_lo=1, types_hi=3, s_types=1.0, s_labels=1.0, seed=1),
    # R-MAT scale 22, 2^25 edges, 256 types (Zipf 1.1, 0-4 per vertex), 64 edge
    # labels (Zipf 1.1), plus 64 chains of 2,000 edges.
    "rmat22_chains": dict(kind="rmat", scale=22, m=1 << 25, n_types=256, n_labels=64,
                          types_lo=0, types_hi=4, s_types=1.1, s_labels=1.1, seed=2,
                          chains=64, chain_len=2000),
    # R-MAT scale 24, 2^27 edges, 128 types, 64 labels (Zipf 1.1): the resident
    # base graph of the incremental / serving workload.
    "rmat24": dict(kind="rmat", scale=24, m=1 << 27, n_types=128, n_labels=64,
                   types_lo=0, types_hi=4, s_types=1.1, s_labels=1.1, seed=5),
    # R-MAT scale 27, 2^30 edges, 1,024 types (0-4 per vertex) and 256 edge
    # labels, Zipf 1.2, labels stored as uint16; counter-based generator.
    "rmat27": dict(kind="cb_rmat", scale=27, m=1 << 30, n_types=1024, n_labels=256, types_lo=0, types_hi=4,
                   s_types=1.2, s_labels=1.2, seed=27, label_u16=True),
    # The same recipe at reduced sizes (tests that must stay fast).
    "cb_rmat16": dict(kind="cb_rmat", scale=16, m=1 << 19, n_types=1024, n_labels=256, types_lo=0, types_hi=4,
                      s_types=1.2, s_labels=1.2, seed=27, label_u16=True),
    "cb_rmat22": dict(kind="cb_rmat", scale=22, m=1 << 25, n_types=1024, n_labels=256, types_lo=0, types_hi=4,
                      s_types=1.2, s_labels=1.2, seed=27, label_u16=True),
    # Reduced shapes of the same recipes, for tests that must stay fast.
    "rmat16_chains": dict(kind="rmat", scale=16, m=1 << 19, n_types=256, n_labels=64,
                          types_lo=0, types_hi=4, s_types=1.1, s_labels=1.1, seed=2,
                          chains=8, chain_len=200),
    "rmat18": dict(kind="rmat", scale=18, m=1 << 21, n_types=128, n_labels=64,
                   types_lo=0, types_hi=4, s_types=1.1, s_labels=1.1, seed=5),
}


def make_config(name: str, seed: Optional[int] = None) -> Graph:
    cfg = dict(CONFIGS[name])
    if seed is not None:
        cfg["seed"] = seed
    kind = cfg.pop("kind")
    if kind == "uniform":
        return uniform_graph(**cfg)
    if kind == "cb_rmat":
        return cb_rmat_graph(**cfg)
    chains = cfg.pop("chains", 0)
    chain_len = cfg.pop("chain_len", 0)
    g = rmat_graph(**cfg)
    if chains:
        # one reserved type id that the Zipf sampler never draws
        g = append_chains(g, chains, chain_len, type_id=cfg["n_types"], label=0)
    return g


# ---------------------------------------------------------------------------
# Small structured graphs (closed-form block counts) and paper fixtures
# ---------------------------------------------------------------------------

def chain(length: int, typed_end: bool = False) -> Graph:
    """Directed path 0 -> 1 -> ... -> length with one edge label."""
    n = length + 1
    src = np.arange(length)
    types = [[] for _ in range(n)]
    if typed_end:
        types[-1] = [1]
    return from_edges(n, src, src + 1, np.zeros(length, dtype=np.int64), types=types)


def cycle(n: int, marked: bool = False) -> Graph:
    """Directed n-cycle with one edge label; ``marked`` gives vertex 0 a
    distinct type."""
    src = np.arange(n)
    types = [[] for _ in range(n)]
    if marked:
        types[0] = [7]
    return from_edges(n, src, (src + 1) % n, np.zeros(n, dtype=np.int64), types=types)


def out_star(leaves: int, label: int = 0) -> Graph:
    """Vertex 0 with one edge of the same label to each of ``leaves`` leaves."""
    n = leaves + 1
    src = np.zeros(leaves, dtype=np.int64)
    return from_edges(n, src, np.arange(1, n), np.full(leaves, label), types=[[] for _ in range(n)])


def binary_tree(depth: int) -> Graph:
    """Complete binary tree of the given depth, edges pointing to children."""
    n = (1 << (depth + 1)) - 1
    src, dst = [], []
    for v in range(n):
        for ch in (2 * v + 1, 2 * v + 2):
            if ch < n:
                src.append(v)
                dst.append(ch)
    return from_edges(n, src, dst, np.zeros(len(src), dtype=np.int64), types=[[] for _ in range(n)])


# Label / type dictionaries for the paper's Sec. 2.2 example graph.
PAPER_EXAMPLE_LABELS = {"author": 0, "title": 1, "name": 2}
PAPER_EXAMPLE_TYPES = {"Proceedings": 0, "Person": 1}


def paper_example(typed: bool = True) -> Graph:
    """The labeled property graph of Sec. 2.2 (the figure next to the LPG
    definition): v1 -author-> v2, v1 -title-> v3, v2 -name-> v4; v1 is a
    Proceedings, v2 a Person, v3 and v4 carry no type.  Vertices are numbered
    v1..v4 -> 0..3."""
    L = PAPER_EXAMPLE_LABELS
    T = PAPER_EXAMPLE_TYPES
    types = [[T["Proceedings"]], [T["Person"]], [], []] if typed else [[], [], [], []]
    return from_edges(4, [0, 0, 1], [1, 2, 3], [L["author"], L["title"], L["name"]],
                      types=types, n_labels=3, n_types=2)


FIG1_TYPES = {"Book": 0, "Person": 1, "Subject": 2, "Agent": 3}
FIG1_LABELS = {"author": 0, "topic": 1}


def fig1_scenario(after_change: bool) -> Graph:
    """The evolving graph of the introduction, rebuilt from its text (the
    figure itself is not available): two books v1, v7, each with an author
    (v2, v8: Person) and a topic (v3, v9: Subject).  At time t+1 vertex v8 is
    an Agent instead of a Person.  Vertices v1, v2, v3, v7, v8, v9 are
    numbered 0..5."""
    T, L = FIG1_TYPES, FIG1_LABELS
    types = [[T["Book"]], [T["Person"]], [T["Subject"]],
             [T["Book"]], [T["Agent"] if after_change else T["Person"]], [T["Subject"]]]
    return from_edges(6, [0, 0, 3, 3], [1, 2, 4, 5],
                      [L["author"], L["topic"], L["author"], L["topic"]], types=types,
                      n_labels=2, n_types=4)


def random_small_graph(rng: np.random.Generator, n: int, m: int, n_labels: int,
                       n_types: int, max_types: int = 2, p_alive: float = 1.0) -> Graph:
    """Small random multigraph (self loops and duplicate triples allowed) for
    exhaustive comparisons.  With p_alive < 1 some vertices are dead; dead
    vertices keep no incident edges."""
    alive = (rng.random(n) < p_alive).astype(np.uint8) if p_alive < 1.0 else None
    src = rng.integers(0, n, size=m)
    dst = rng.integers(0, n, size=m)
    lab = rng.integers(0, max(1, n_labels), size=m)
    if alive is not None:
        keep = (alive[src] == 1) & (alive[dst] == 1)
        src, dst, lab = src[keep], dst[keep], lab[keep]
    types = []
    for _ in range(n):
        c = int(rng.integers(0, max_types + 1)) if n_types > 0 else 0
        types.append([int(x) for x in rng.integers(0, max(1, n_types), size=c)])
    return from_edges(n, src, dst, lab, types=types, alive=alive,
                      n_labels=max(1, n_labels), n_types=max(1, n_types))


# ---------------------------------------------------------------------------
# Update batches (ADD / MOD / DEL of vertices and edges)
# ---------------------------------------------------------------------------

OP_KINDS = ("add_v", "mod_v", "del_v", "add_e", "mod_e", "del_e")


def update_ops(g: Graph, rng: np.random.Generator, n_ops: int, mix=(0.60, 0.25, 0.15),
               vertex_frac: float = 0.10, n_labels: Optional[int] = None,
               n_types: Optional[int] = None, rmat_scale: Optional[int] = None,
               max_types: int = 4) -> dict:
    """A seeded, valid ordered batch of update operations for graph g.

    Kinds: ADD / MOD / DEL with probabilities `mix`; within each class a
    `vertex_frac` share are vertex operations, the rest edge operations.
    Vertices deleted by the batch are chosen first and no other operation of
    the batch touches them; edge ops use vertices that exist when the batch
    starts.  DEL_E / MOD_E pick existing edges uniformly; ADD_E endpoints are
    uniform, or drawn by the R-MAT sampler when `rmat_scale` is given
    (rejecting ids >= n).  Returns numpy arrays (op, u, w, label, new_label)
    and the type lists of the vertex ops as a CSR (t_off, t_ids), with t_off
    indexed by operation.
    """
    n, m = g.n, g.m
    n_labels = n_labels or max(g.n_labels, 1)
    n_types = n_types or max(g.n_types, 1)
    alive = np.ones(n, dtype=bool) if g.alive is None else g.alive.astype(bool)
    cls = rng.choice(3, size=n_ops, p=np.asarray(mix) / sum(mix))       # 0 add, 1 mod, 2 del
    is_v = rng.random(n_ops) < vertex_frac
    op = np.where(is_v, cls + 1, cls + 4).astype(np.uint32)            # 1..3 vertex, 4..6 edge
    u = np.zeros(n_ops, dtype=np.uint32)
    w = np.zeros(n_ops, dtype=np.uint32)
    lab = np.zeros(n_ops, dtype=np.uint32)
    nlab = np.zeros(n_ops, dtype=np.uint32)
    live = np.flatnonzero(alive)
    # deleted vertices: distinct alive vertices
    n_del_v = int(np.sum(op == 3))
    if n_del_v > live.size // 2:
        op[np.flatnonzero(op == 3)[live.size // 2:]] = 2
        n_del_v = int(np.sum(op == 3))
    dead = rng.choice(live, size=n_del_v, replace=False) if n_del_v else np.zeros(0, dtype=np.int64)
    u[op == 3] = dead
    keep = np.ones(n, dtype=bool)
    keep[dead] = False
    keep &= alive
    pool = np.flatnonzero(keep)
    if pool.size == 0:
        op[(op == 2) | (op >= 4)] = 1
    else:
        mv = op == 2
        u[mv] = rng.choice(pool, size=int(mv.sum()))
        # edges usable by DEL_E / MOD_E: both endpoints stay alive
        src = g.src()
        ok = keep[src] & keep[g.tgt] if m else np.zeros(0, dtype=bool)
        eidx = np.flatnonzero(ok)
        de = (op == 5) | (op == 6)
        if eidx.size == 0:
            op[de] = 4
            de[:] = False
        pick = eidx[rng.integers(0, eidx.size, size=int(de.sum()))] if de.any() else np.zeros(0, dtype=np.int64)
        u[de] = src[pick]
        w[de] = g.tgt[pick]
        lab[de] = g.lab[pick]
        nlab[op == 5] = rng.integers(0, n_labels, size=int(np.sum(op == 5)))
        ae = op == 4
        k = int(ae.sum())
        if rmat_scale is not None and k:
            got_u, got_w = [], []
            need = k
            while need > 0:
                s_, d_ = rmat_edges(rng, rmat_scale, 2 * need + 16, 0.57, 0.19, 0.19)
                okm = (s_ < n) & (d_ < n)
                s_, d_ = s_[okm], d_[okm]
                okm = keep[s_] & keep[d_]
                got_u.append(s_[okm][:need])
                got_w.append(d_[okm][:need])
                need -= len(got_u[-1])
            u[ae] = np.concatenate(got_u)[:k]
            w[ae] = np.concatenate(got_w)[:k]
        else:
            u[ae] = rng.choice(pool, size=k)
            w[ae] = rng.choice(pool, size=k)
        lab[ae] = zipf_sample(rng, n_labels, 1.1, k) if k else lab[ae]
    # type lists of ADD_V / MOD_V
    tv = (op == 1) | (op == 2)
    cnt = np.zeros(n_ops, dtype=np.int64)
    cnt[tv] = rng.integers(0, max_types + 1, size=int(tv.sum()))
    t_off = np.zeros(n_ops + 1, dtype=np.int64)
    np.cumsum(cnt, out=t_off[1:])
    t_ids = rng.integers(0, n_types, size=int(t_off[-1])).astype(np.uint32)
    return dict(op=op, u=u, w=w, label=lab, new_label=nlab, t_off=t_off, t_ids=t_ids)


def ops_as_tuples(d: dict) -> List[tuple]:
    """The same batch as tuples ("add_v", types), ("mod_v", u, types),
    ("del_v", u), ("add_e", u, l, w), ("mod_e", u, l, w, l2), ("del_e", u, l, w)."""
    out = []
    for i, o in enumerate(d["op"]):
        ty = [int(x) for x in d["t_ids"][d["t_off"][i]:d["t_off"][i + 1]]]
        u, w, l, l2 = int(d["u"][i]), int(d["w"][i]), int(d["label"][i]), int(d["new_label"][i])
        if o == 1:
            out.append(("add_v", ty))
        elif o == 2:
            out.append(("mod_v", u, ty))
        elif o == 3:
            out.append(("del_v", u))
        elif o == 4:
            out.append(("add_e", u, l, w))
        elif o == 5:
            out.append(("mod_e", u, l, w, l2))
        else:
            out.append(("del_e", u, l, w))
    return out


def sample_update_ops(row_off: np.ndarray, tgt: np.ndarray, lab: np.ndarray, n: int, dead: np.ndarray,
                      rng: np.random.Generator, n_ops: int, n_labels: int, n_types: int,
                      mix=(0.60, 0.25, 0.15), vertex_frac: float = 0.10,
                      rmat_scale: Optional[int] = None, max_types: int = 4) -> dict:
    """A valid update batch for a large resident graph, built by sampling.

    Same operation mix as `update_ops`, but DEL_E / MOD_E sample edges of the
    given CSR (the graph the state started from; an edge already deleted by
    an earlier batch makes a valid no-op delete) and only vertices with
    dead[v] == False are used.  `dead` has at least n entries and is updated
    in place with the vertices this batch deletes; new vertices take ids
    n, n+1, ...  Returns the arrays of `update_ops` plus "n_after".
    """
    m = int(tgt.size)
    cls = rng.choice(3, size=n_ops, p=np.asarray(mix) / sum(mix))
    is_v = rng.random(n_ops) < vertex_frac
    op = np.where(is_v, cls + 1, cls + 4).astype(np.uint32)
    u = np.zeros(n_ops, dtype=np.uint32)
    w = np.zeros(n_ops, dtype=np.uint32)
    lb = np.zeros(n_ops, dtype=np.uint32)
    nl = np.zeros(n_ops, dtype=np.uint32)

    def alive_vertices(k):
        out = []
        need = k
        while need > 0:
            c = rng.integers(0, n, size=2 * need + 8)
            c = c[~dead[c]]
            out.append(c[:need])
            need -= len(out[-1])
        return np.concatenate(out)[:k] if k else np.zeros(0, dtype=np.int64)

    # vertices deleted by this batch: distinct, alive, and untouched by the rest
    dv = op == 3
    victims = np.unique(alive_vertices(int(dv.sum())))
    op[np.flatnonzero(dv)[victims.size:]] = 2
    u[np.flatnonzero(op == 3)] = victims
    dead[victims] = True
    mv = op == 2
    u[mv] = alive_vertices(int(mv.sum()))
    de = (op == 5) | (op == 6)
    k = int(de.sum())
    if k:
        su, sw, sl = [], [], []
        need = k
        while need > 0:
            e = rng.integers(0, m, size=2 * need + 8)
            s_ = np.searchsorted(row_off, e, side="right") - 1
            ok = ~dead[s_] & ~dead[tgt[e]]
            su.append(s_[ok][:need])
            sw.append(tgt[e][ok][:need])
            sl.append(lab[e][ok][:need])
            need -= len(su[-1])
        u[de], w[de], lb[de] = np.concatenate(su)[:k], np.concatenate(sw)[:k], np.concatenate(sl)[:k]
    nl[op == 5] = rng.integers(0, n_labels, size=int(np.sum(op == 5)))
    ae = op == 4
    k = int(ae.sum())
    if k:
        if rmat_scale is not None:
            su, sw = [], []
            need = k
            while need > 0:
                s_, d_ = rmat_edges(rng, rmat_scale, 2 * need + 16, 0.57, 0.19, 0.19)
                ok = (s_ < n) & (d_ < n)
                s_, d_ = s_[ok], d_[ok]
                ok = ~dead[s_] & ~dead[d_]
                su.append(s_[ok][:need])
                sw.append(d_[ok][:need])
                need -= len(su[-1])
            u[ae], w[ae] = np.concatenate(su)[:k], np.concatenate(sw)[:k]
        else:
            u[ae], w[ae] = alive_vertices(k), alive_vertices(k)
        lb[ae] = zipf_sample(rng, n_labels, 1.1, k)
    tv = (op == 1) | (op == 2)
    cnt = np.zeros(n_ops, dtype=np.int64)
    cnt[tv] = rng.integers(0, max_types + 1, size=int(tv.sum()))
    t_off = np.zeros(n_ops + 1, dtype=np.int64)
    np.cumsum(cnt, out=t_off[1:])
    t_ids = rng.integers(0, n_types, size=int(t_off[-1])).astype(np.uint32)
    return dict(op=op, u=u, w=w, label=lb, new_label=nl, t_off=t_off, t_ids=t_ids,
                n_after=n + int(np.sum(op == 1)))
