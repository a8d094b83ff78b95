"""Hash-free references that pin the oracle's partitions.

TEST INFRASTRUCTURE ONLY.  Pure Python, no hashing at all, so a mistake in
the hash spec or in the C oracle cannot hide here.

exact_refinement  -- naive partition refinement written straight from the
                     forward k-bisimulation definition (Sec. 2.5, typed
                     variant): u, v are k-bisimilar iff they are
                     (k-1)-bisimilar and their sets of (edge label,
                     (k-1)-class of target) pairs are equal.  Classes are
                     interned in vertex order, so class ids are the
                     first-occurrence block ids.
brute_force_classes -- the definition evaluated pairwise: relation R_k is
                     the set of pairs in R_{k-1} such that every l-edge of u
                     is matched by an l-edge of v into R_{k-1}, and vice
                     versa (the symmetric reading, as in the complex schema
                     element of Sec. 2.4).

Both take the direction parameterization (outgoing edges, incoming edges as
in backward bisimulation, or both, told apart by a direction tag) and the
label parameterization (only edges whose label is in a given set) of
Sec. 2.4 through ``signature_edges``.
"""

from __future__ import annotations

from typing import Dict, List, Optional, Sequence, Tuple


def _alive(g, v: int) -> bool:
    return g.alive is None or bool(g.alive[v])


def _intern(keys: Sequence) -> Tuple[List[int], int]:
    """Number distinct keys in order of first appearance (None = no block)."""
    ids: Dict = {}
    out = []
    for k in keys:
        if k is None:
            out.append(None)
            continue
        if k not in ids:
            ids[k] = len(ids)
        out.append(ids[k])
    return out, len(ids)


def signature_edges(g, direction: str = "out", labels=None) -> List[List[Tuple]]:
    """Per vertex, the edges its signature looks at, as (direction tag, label,
    partner): outgoing edges (tag "o", partner = target), incoming edges
    (tag "i", partner = source) or both (Sec. 2.4 direction
    parameterization; Sec. 2.5 backward bisimulation), keeping only labels
    in ``labels`` when it is given (label parameterization)."""
    keep = None if labels is None else set(int(x) for x in labels)
    sig: List[List[Tuple]] = [[] for _ in range(g.n)]
    for v in range(g.n):
        for (l, w) in g.out_edges(v):
            if keep is not None and l not in keep:
                continue
            if direction in ("out", "both"):
                sig[v].append(("o", l, w))
            if direction in ("in", "both"):
                sig[w].append(("i", l, v))
    return sig


def exact_refinement(g, k_max: int, stop_at_fixpoint: bool = True,
                     untyped: bool = False, direction: str = "out", labels=None):
    """Returns (levels, counts, k_done): levels[k][v] is v's first-occurrence
    block id in the k-partition (None for dead vertices)."""
    n = g.n
    types = [frozenset(g.types_of(v)) if not untyped else frozenset() for v in range(n)]
    edges = [[((d, l), w) for (d, l, w) in es] for es in signature_edges(g, direction, labels)]
    cls, cnt = _intern([types[v] if _alive(g, v) else None for v in range(n)])
    levels = [cls]
    counts = [cnt]
    k_done = 0
    for k in range(1, k_max + 1):
        prev = levels[-1]
        sig = []
        for v in range(n):
            if not _alive(g, v):
                sig.append(None)
                continue
            sig.append((prev[v], frozenset((l, prev[w]) for (l, w) in edges[v])))
        cls, cnt = _intern(sig)
        levels.append(cls)
        counts.append(cnt)
        k_done = k
        if stop_at_fixpoint and cnt == counts[-2]:
            break
    return levels, counts, k_done


def brute_force_classes(g, k: int, untyped: bool = False, direction: str = "out",
                        labels=None) -> List[Optional[int]]:
    """First-occurrence class ids of the k-bisimulation, from the pairwise
    definition (quadratic in n; tiny graphs only).  A (direction, label) pair
    plays the role of the label."""
    n = g.n
    alive = [v for v in range(n) if _alive(g, v)]
    types = {v: (frozenset() if untyped else frozenset(g.types_of(v))) for v in alive}
    sig = signature_edges(g, direction, labels)
    out = {v: [((d, l), w) for (d, l, w) in sig[v]] for v in alive}
    rel = {(u, v) for u in alive for v in alive if types[u] == types[v]}
    for _ in range(k):
        nxt = set()
        for (u, v) in rel:
            ok = all(any(l2 == l1 and (u1, v1) in rel for (l2, v1) in out[v])
                     for (l1, u1) in out[u])
            ok = ok and all(any(l2 == l1 and (u1, v1) in rel for (l2, u1) in out[u])
                            for (l1, v1) in out[v])
            if ok:
                nxt.add((u, v))
        rel = nxt
    # first-occurrence numbering of the equivalence classes
    ids: Dict[int, int] = {}
    res: List[Optional[int]] = [None] * n
    nb = 0
    for v in range(n):
        if not _alive(g, v):
            continue
        rep = min(u for u in alive if (u, v) in rel)
        if rep not in ids:
            ids[rep] = nb
            nb += 1
        res[v] = ids[rep]
    return res


def quotient_edges(g, block_ids, labels=None, dst_ids=None) -> List[Tuple[int, int, int]]:
    """Distinct (block(v), label, block(w)) over all edges (over the edges
    whose label is in ``labels`` when it is given), sorted.  With ``dst_ids``
    the target end takes its id from there instead (the vertex-summary
    edges of Sec. 2.6 into the neighbours' classes of the previous level)."""
    keep = None if labels is None else set(int(x) for x in labels)
    dst = block_ids if dst_ids is None else dst_ids
    s = set()
    for v in range(g.n):
        for (l, w) in g.out_edges(v):
            if keep is None or l in keep:
                s.add((int(block_ids[v]), int(l), int(dst[w])))
    return sorted(s)
