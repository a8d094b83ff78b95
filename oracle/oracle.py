"""ctypes wrapper around the C oracle (``bsim_oracle.c``).

TEST INFRASTRUCTURE ONLY (see the package docstring).  Argument marshalling
only: all arithmetic lives in the C file.
"""

from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Dict, Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "bsim_oracle.c")
LIB = os.path.join(HERE, "libbsim_oracle.so")

STOP_AT_FIXPOINT = 1
UNTYPED = 4
PREV_LEVEL_EDGES = 128
BACKWARD = 32
BOTH_DIRECTIONS = 64


def build(force: bool = True) -> str:
    """Compile the C oracle into ``oracle/libbsim_oracle.so`` with gcc."""
    if force or not os.path.exists(LIB):
        tmp = LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-Wall", "-Wextra", "-shared",
                               "-fPIC", "-o", tmp, SRC])
        os.replace(tmp, LIB)
    return LIB


_lib = None


def load(path: str) -> ctypes.CDLL:
    """Load a compiled oracle library and declare its signatures."""
    L = ctypes.CDLL(path)
    u64, u32, p = ctypes.c_uint64, ctypes.c_uint32, ctypes.c_void_p
    L.bo_mix.restype = u64
    L.bo_mix.argtypes = [u64]
    for name in ("bo_const_t", "bo_const_l", "bo_const_s", "bo_const_e"):
        getattr(L, name).restype = u64
        getattr(L, name).argtypes = []
    L.bo_type_hash.restype = u64
    L.bo_type_hash.argtypes = [p, u32, u32]
    L.bo_label_salt.restype = u64
    L.bo_label_salt.argtypes = [u32]
    L.bo_vertex_step.restype = u64
    L.bo_vertex_step.argtypes = [u64, p, p, u64, p]
    L.bo_block_ids.restype = u32
    L.bo_block_ids.argtypes = [p, p, u32, p]
    L.bo_refine_classes.restype = u32
    L.bo_refine_classes.argtypes = [p, p, p, u32, p]
    L.bo_summarize.restype = ctypes.c_int
    L.bo_summarize.argtypes = [u32, u64, p, p, p, p, p, p, u32, u32,
                               p, p, p, p, p, p, p, p, p, p, p, p]
    L.bo_iterate.restype = ctypes.c_int
    L.bo_iterate.argtypes = [u32, p, p, p, p, p, u32, u32, p, p]
    L.bo_label_salt_in.restype = u64
    L.bo_label_salt_in.argtypes = [u32]
    L.bo_type_hashes.restype = None
    L.bo_type_hashes.argtypes = [u32, p, p, u32, p]
    L.bo_step_strided.restype = ctypes.c_int
    L.bo_step_strided.argtypes = [u32, p, p, p, p, p, u32, u32, u32, p]
    L.bo_summarize_ext.restype = ctypes.c_int
    L.bo_summarize_ext.argtypes = [u32, u64, p, p, p, p, p, p, u32, u32, p, u32,
                                   p, p, p, p, p, p, p, p, p, p, p]
    return L


def lib() -> ctypes.CDLL:
    global _lib
    if _lib is None:
        if not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
            build()
        _lib = load(LIB)
    return _lib


def _ptr(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def mix(z: int) -> int:
    return int(lib().bo_mix(ctypes.c_uint64(z & 0xFFFFFFFFFFFFFFFF)))


def type_hash(types, untyped: bool = False) -> int:
    a = np.ascontiguousarray(np.asarray(types, dtype=np.uint32))
    return int(lib().bo_type_hash(_ptr(a), a.size, 1 if untyped else 0))


def label_salt(label: int) -> int:
    return int(lib().bo_label_salt(label))


def vertex_step(t_v: int, tgt, lab, h_prev: np.ndarray) -> int:
    tgt = np.ascontiguousarray(np.asarray(tgt, dtype=np.uint32))
    lab = np.ascontiguousarray(np.asarray(lab, dtype=np.uint32))
    h_prev = np.ascontiguousarray(h_prev, dtype=np.uint64)
    return int(lib().bo_vertex_step(t_v, _ptr(tgt), _ptr(lab), tgt.size, _ptr(h_prev)))


def block_ids(h: np.ndarray, alive: Optional[np.ndarray] = None):
    h = np.ascontiguousarray(h, dtype=np.uint64)
    out = np.zeros(h.size, dtype=np.uint32)
    al = None if alive is None else np.ascontiguousarray(alive, dtype=np.uint8)
    nb = lib().bo_block_ids(_ptr(h), _ptr(al), h.size, _ptr(out))
    return out, int(nb)


def refine_classes(cls, h, alive=None):
    """One refinement step: new class = (cls[v], h[v]), first-occurrence ids."""
    h = np.ascontiguousarray(h, dtype=np.uint64)
    c = np.ascontiguousarray(cls, dtype=np.uint32)
    out = np.zeros(max(h.size, 1), dtype=np.uint32)
    al = None if alive is None else np.ascontiguousarray(alive, dtype=np.uint8)
    nb = lib().bo_refine_classes(_ptr(c), _ptr(h), _ptr(al), h.size, _ptr(out))
    return out[:h.size], int(nb)


def _csr(g):
    row_off = np.ascontiguousarray(g.row_off, dtype=np.uint64)
    tgt = np.ascontiguousarray(g.tgt, dtype=np.uint32)
    lab = np.ascontiguousarray(g.lab, dtype=np.uint32)
    typ_off = np.ascontiguousarray(g.typ_off, dtype=np.uint64)
    typ = np.ascontiguousarray(g.typ, dtype=np.uint32)
    if typ.size == 0:
        typ = np.zeros(1, dtype=np.uint32)
    alive = None if g.alive is None else np.ascontiguousarray(g.alive, dtype=np.uint8)
    return row_off, tgt, lab, typ_off, typ, alive


def summarize(g, k_max: int, stop_at_fixpoint: bool = True, untyped: bool = False,
              prev_level_edges: bool = False) -> Dict:
    """Batch summarization of graph ``g``; returns a dict of numpy arrays and
    scalars (see ``bo_summarize`` in the C file).  ``prev_level_edges``: the
    summary edges lead to the targets' (k_done-1)-classes."""
    n, m = g.n, g.m
    row_off, tgt, lab, typ_off, typ, alive = _csr(g)
    if tgt.size == 0:
        tgt = np.zeros(1, dtype=np.uint32)
        lab = np.zeros(1, dtype=np.uint32)
    flags = ((STOP_AT_FIXPOINT if stop_at_fixpoint else 0) | (UNTYPED if untyped else 0)
             | (PREV_LEVEL_EDGES if prev_level_edges else 0))
    hashes = np.zeros(max(n, 1), dtype=np.uint64)
    prev = np.zeros(max(n, 1), dtype=np.uint64)
    bids = np.zeros(max(n, 1), dtype=np.uint32)
    bpi = np.zeros(k_max + 1, dtype=np.uint32)
    bsz = np.zeros(max(n, 1), dtype=np.uint32)
    se_s = np.zeros(max(m, 1), dtype=np.uint32)
    se_l = np.zeros(max(m, 1), dtype=np.uint32)
    se_d = np.zeros(max(m, 1), dtype=np.uint32)
    k_done = ctypes.c_uint32()
    fix = ctypes.c_uint32()
    nb = ctypes.c_uint32()
    nse = ctypes.c_uint64()
    rc = lib().bo_summarize(n, m, _ptr(row_off), _ptr(tgt), _ptr(lab), _ptr(typ_off),
                            _ptr(typ), _ptr(alive), k_max, flags, _ptr(hashes), _ptr(prev),
                            _ptr(bids), _ptr(bpi), ctypes.byref(k_done), ctypes.byref(fix),
                            ctypes.byref(nb), _ptr(bsz), ctypes.byref(nse), _ptr(se_s),
                            _ptr(se_l), _ptr(se_d))
    if rc != 0:
        raise ValueError("oracle rejected the graph (status %d)" % rc)
    kd, nbv, ns = k_done.value, nb.value, nse.value
    return dict(k_done=kd, fixpoint=fix.value, n_blocks=nbv, hashes=hashes[:n],
                prev_hashes=prev[:n], block_ids=bids[:n], blocks_per_iter=bpi[:kd + 1],
                block_sizes=bsz[:nbv], se_src=se_s[:ns], se_label=se_l[:ns], se_dst=se_d[:ns])


def summarize_ext(g, k_max: int, stop_at_fixpoint: bool = True, untyped: bool = False,
                  direction: str = "out", labels=None, prev_level_edges: bool = False) -> Dict:
    """Summarization under the direction parameterization ("out", "in" or
    "both") and the label parameterization (``labels``: the kept label set
    P_l, None for every label); see ``bo_summarize_ext`` in the C file."""
    n, m = g.n, g.m
    row_off, tgt, lab, typ_off, typ, alive = _csr(g)
    if tgt.size == 0:
        tgt = np.zeros(1, dtype=np.uint32)
        lab = np.zeros(1, dtype=np.uint32)
    flags = ((STOP_AT_FIXPOINT if stop_at_fixpoint else 0) | (UNTYPED if untyped else 0)
             | {"out": 0, "in": BACKWARD, "both": BOTH_DIRECTIONS}[direction]
             | (PREV_LEVEL_EDGES if prev_level_edges else 0))
    keep = None
    if labels is not None:
        ls = np.asarray(list(labels), dtype=np.int64)
        keep = np.zeros(int(ls.max()) + 1 if ls.size else 1, dtype=np.uint8)
        keep[ls] = 1
    hashes = np.zeros(max(n, 1), dtype=np.uint64)
    bids = np.zeros(max(n, 1), dtype=np.uint32)
    bpi = np.zeros(k_max + 1, dtype=np.uint32)
    bsz = np.zeros(max(n, 1), dtype=np.uint32)
    se_s = np.zeros(max(m, 1), dtype=np.uint32)
    se_l = np.zeros(max(m, 1), dtype=np.uint32)
    se_d = np.zeros(max(m, 1), dtype=np.uint32)
    k_done = ctypes.c_uint32()
    fix = ctypes.c_uint32()
    nb = ctypes.c_uint32()
    nse = ctypes.c_uint64()
    rc = lib().bo_summarize_ext(n, m, _ptr(row_off), _ptr(tgt), _ptr(lab), _ptr(typ_off),
                                _ptr(typ), _ptr(alive), k_max, flags, _ptr(keep),
                                0 if keep is None else keep.size, _ptr(hashes), _ptr(bids),
                                _ptr(bpi), ctypes.byref(k_done), ctypes.byref(fix),
                                ctypes.byref(nb), _ptr(bsz), ctypes.byref(nse), _ptr(se_s),
                                _ptr(se_l), _ptr(se_d))
    if rc != 0:
        raise ValueError("oracle rejected the graph (status %d)" % rc)
    kd, nbv, ns = k_done.value, nb.value, nse.value
    return dict(k_done=kd, fixpoint=fix.value, n_blocks=nbv, hashes=hashes[:n],
                block_ids=bids[:n], blocks_per_iter=bpi[:kd + 1],
                block_sizes=bsz[:nbv], se_src=se_s[:ns], se_label=se_l[:ns], se_dst=se_d[:ns])


def iterate(g, iters: int, untyped: bool = False):
    """h^iters (no fixpoint test, all vertices alive) and n_0..n_iters."""
    row_off, tgt, lab, typ_off, typ, _ = _csr(g)
    out = np.zeros(max(g.n, 1), dtype=np.uint64)
    counts = np.zeros(iters + 1, dtype=np.uint32)
    rc = lib().bo_iterate(g.n, _ptr(row_off), _ptr(tgt), _ptr(lab), _ptr(typ_off), _ptr(typ),
                          iters, UNTYPED if untyped else 0, _ptr(out), _ptr(counts))
    if rc != 0:
        raise RuntimeError("oracle iterate failed (%d)" % rc)
    return out[:g.n], counts


def type_hashes(g, untyped: bool = False) -> np.ndarray:
    """t(v) for every vertex of g (alive or not)."""
    typ_off = np.ascontiguousarray(g.typ_off, dtype=np.uint64)
    typ = np.ascontiguousarray(g.typ, dtype=np.uint32)
    if typ.size == 0:
        typ = np.zeros(1, dtype=np.uint32)
    out = np.zeros(max(g.n, 1), dtype=np.uint64)
    lib().bo_type_hashes(g.n, _ptr(typ_off), _ptr(typ), UNTYPED if untyped else 0, _ptr(out))
    return out[:g.n]


def step_strided(g, t: np.ndarray, h_prev: np.ndarray, v0: int, stride: int, count: int) -> np.ndarray:
    """The refinement step of every stride-th vertex from v0 (h^k from
    h_prev = h^{k-1}), as in the full runs."""
    row_off = np.ascontiguousarray(g.row_off, dtype=np.uint64)
    tgt = np.ascontiguousarray(g.tgt, dtype=np.uint32)
    lab = np.ascontiguousarray(g.lab, dtype=np.uint32)
    out = np.zeros(max(count, 1), dtype=np.uint64)
    rc = lib().bo_step_strided(g.n, _ptr(row_off), _ptr(tgt), _ptr(lab), _ptr(np.ascontiguousarray(t)),
                               _ptr(np.ascontiguousarray(h_prev)), v0, stride, count, _ptr(out))
    if rc != 0:
        raise ValueError("oracle rejected the sample (%d)" % rc)
    return out[:count]
