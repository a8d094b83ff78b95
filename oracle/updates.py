"""Sequential application of an update batch to a graph -- test
infrastructure, like the rest of oracle/.

The change classes of Sec. 3.2 (a summary or payload element added,
modified or deleted) arise from these operations on the data graph:

  ("add_v", types)          new vertex with id n and the given type set
  ("mod_v", u, types)       replace the type set of u
  ("del_v", u)              delete u: its types and every edge into or out of it
  ("add_e", u, l, w)        add the triple (u, l, w) unless it already exists
  ("del_e", u, l, w)        delete every copy of (u, l, w) (no-op when absent)
  ("mod_e", u, l, w, l2)    ("del_e", u, l, w) then ("add_e", u, l2, w)

Operations apply one after the other; one that names a vertex id not yet
created raises IndexError, one that names a deleted vertex raises ValueError.
Vertex ids are stable: a deleted vertex keeps its id and is marked dead.
By Theorem 2 the incremental summary after the batch equals the batch
summary of the graph this returns.
"""

from __future__ import annotations

import numpy as np

from paper_2111_12493_amd.graphgen import Graph


def apply_ops(g: Graph, ops) -> Graph:
    n = g.n
    alive = [True] * n if g.alive is None else [bool(x) for x in g.alive]
    types = [[int(x) for x in g.typ[g.typ_off[v]:g.typ_off[v + 1]]] for v in range(n)]
    out = [[(int(l), int(w)) for l, w in zip(g.lab[g.row_off[v]:g.row_off[v + 1]],
                                              g.tgt[g.row_off[v]:g.row_off[v + 1]])] for v in range(n)]

    def live(v):
        if v >= len(alive):
            raise IndexError("vertex %d does not exist" % v)
        if not alive[v]:
            raise ValueError("vertex %d is deleted" % v)

    for o in ops:
        kind = o[0]
        if kind == "add_v":
            types.append([int(x) for x in o[1]])
            alive.append(True)
            out.append([])
        elif kind == "mod_v":
            live(o[1])
            types[o[1]] = [int(x) for x in o[2]]
        elif kind == "del_v":
            u = o[1]
            live(u)
            alive[u] = False
            types[u] = []
            out[u] = []
            for s in range(len(out)):
                if out[s]:
                    out[s] = [e for e in out[s] if e[1] != u]
        elif kind in ("add_e", "del_e", "mod_e"):
            u, l, w = o[1], o[2], o[3]
            live(u)
            live(w)
            if kind != "add_e":
                out[u] = [e for e in out[u] if e != (l, w)]
            if kind != "del_e":
                ln = o[4] if kind == "mod_e" else l
                if (ln, w) not in out[u]:
                    out[u].append((ln, w))
        else:
            raise ValueError("unknown op " + str(kind))
    n = len(out)
    row_off = np.zeros(n + 1, dtype=np.uint64)
    row_off[1:] = np.cumsum([len(r) for r in out]) if n else []
    tgt = np.array([w for r in out for (_, w) in r], dtype=np.uint32)
    lab = np.array([l for r in out for (l, _) in r], dtype=g.lab.dtype)
    typ_off = np.zeros(n + 1, dtype=np.uint64)
    typ_off[1:] = np.cumsum([len(t) for t in types]) if n else []
    typ = np.array([x for t in types for x in t], dtype=np.uint32)
    return Graph(n=n, row_off=row_off, tgt=tgt, lab=lab, typ_off=typ_off, typ=typ,
                 alive=np.array(alive, dtype=np.uint8), n_labels=g.n_labels, n_types=g.n_types)


def replay_rows(g: Graph, ops, vertices):
    """Out-rows, type lists and liveness of the given vertices after the
    operations, by the sequential semantics of apply_ops.

    An operation changes the out-row of its source, the type list of its
    vertex, or (a vertex deletion) every edge into the deleted vertex.  Once
    deleted, a vertex can be named by no later operation, so no edge into it
    can come back: removing those edges at the end, by the final liveness of
    the targets, gives the same rows as removing them at the deletion.  So
    only the asked-for rows are followed (as multisets of (label, target)),
    while every operation is still validated against the liveness of all
    vertices, as apply_ops does.  Returns {v: sorted [(label, target), ...]},
    {v: sorted types}, {v: alive}.
    """
    want = set(int(v) for v in vertices)
    alive = list(np.ones(g.n, dtype=bool) if g.alive is None else g.alive.astype(bool))
    rows = {}
    types = {}
    for v in want:
        if v < g.n:
            a, b = int(g.row_off[v]), int(g.row_off[v + 1])
            r = {}
            for e in zip(g.lab[a:b].tolist(), g.tgt[a:b].tolist()):
                r[e] = r.get(e, 0) + 1
            rows[v] = r
            types[v] = [int(x) for x in g.typ[int(g.typ_off[v]):int(g.typ_off[v + 1])]]

    def live(v):
        if v >= len(alive):
            raise IndexError("vertex %d does not exist" % v)
        if not alive[v]:
            raise ValueError("vertex %d is deleted" % v)

    for o in ops:
        kind = o[0]
        if kind == "add_v":
            v = len(alive)
            alive.append(True)
            if v in want:
                rows[v] = {}
                types[v] = [int(x) for x in o[1]]
        elif kind == "mod_v":
            live(o[1])
            if o[1] in want:
                types[o[1]] = [int(x) for x in o[2]]
        elif kind == "del_v":
            u = o[1]
            live(u)
            alive[u] = False
            if u in want:
                rows[u] = {}
                types[u] = []
        elif kind in ("add_e", "del_e", "mod_e"):
            u, l, w = o[1], o[2], o[3]
            live(u)
            live(w)
            if u not in want:
                continue
            if kind != "add_e":
                rows[u].pop((l, w), None)
            if kind != "del_e":
                ln = o[4] if kind == "mod_e" else l
                if (ln, w) not in rows[u]:
                    rows[u][(ln, w)] = 1
        else:
            raise ValueError("unknown op " + str(kind))
    out = {}
    for v, r in rows.items():
        out[v] = sorted(e for e, c in r.items() for _ in range(c) if alive[e[1]])
    return out, {v: sorted(t) for v, t in types.items()}, {v: bool(alive[v]) for v in want if v < len(alive)}


def diff_snapshots(before: Graph, after: Graph):
    """Change detection from two snapshots without a change log: the ordered
    batch that turns ``before`` into ``after`` (equal alive flags, type sets
    and sets of edge triples).  Vertex ids are shared; ids before.n ..
    after.n - 1 are new vertices.  The batch, in this order:

      add_v  for every new id, ascending, with after's stored type list;
      mod_v  for every vertex alive in both whose type *set* changed, with
             after's stored type list;
      del_e  for every distinct triple of before absent from after whose two
             endpoints stay alive, in order of its first copy in before;
      add_e  for every distinct triple of after absent from before, in order
             of its first copy in after;
      del_v  for every vertex alive in before (or new) and dead in after.

    Edges of a deleted vertex go with its del_v.  A vertex dead in before
    and alive in after cannot arise from updates (ids are never reused):
    ValueError, as for after.n < before.n."""
    n0, n1 = before.n, after.n
    if n1 < n0:
        raise ValueError("the later snapshot has fewer vertex ids")

    def alive(g, v):
        return g.alive is None or bool(g.alive[v])

    def types(g, v):
        return [int(x) for x in g.typ[int(g.typ_off[v]):int(g.typ_off[v + 1])]]

    def triples(g):
        seen, order = set(), []
        for u in range(g.n):
            for e in range(int(g.row_off[u]), int(g.row_off[u + 1])):
                t = (u, int(g.lab[e]), int(g.tgt[e]))
                if t not in seen:
                    seen.add(t)
                    order.append(t)
        return seen, order

    for v in range(n0):
        if not alive(before, v) and alive(after, v):
            raise ValueError("vertex %d is dead before and alive after" % v)
    ops = [("add_v", types(after, v)) for v in range(n0, n1)]
    for v in range(n0):
        if alive(before, v) and alive(after, v) and set(types(before, v)) != set(types(after, v)):
            ops.append(("mod_v", v, types(after, v)))
    sb, ob = triples(before)
    sa, oa = triples(after)
    for (u, l, w) in ob:
        if (u, l, w) not in sa and alive(after, u) and alive(after, w):
            ops.append(("del_e", u, l, w))
    for (u, l, w) in oa:
        if (u, l, w) not in sb:
            ops.append(("add_e", u, l, w))
    for v in range(n1):
        if (v >= n0 or alive(before, v)) and not alive(after, v):
            ops.append(("del_v", v))
    return ops
