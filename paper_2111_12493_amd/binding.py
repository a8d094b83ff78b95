"""Thin ctypes binding of the C ABI in ``include/bsim.h``.

Argument marshalling only: every step of the summarization runs in the HIP
library ``libbsim.so``.  PyTorch supplies device memory and the HIP stream.
Loading fails loudly when the library has not been built -- there is no
fallback path.
"""

from __future__ import annotations

import ctypes
import os
from typing import Dict, List, Optional, Sequence

import numpy as np

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libbsim.so")

# bsim.h constants
OK = 0
E_INVALID, E_RANGE, E_NOMEM, E_DEVICE, E_UNSUPPORTED, E_BUSY, E_IO = -1, -2, -3, -4, -5, -6, -7
MEM_HOST, MEM_DEVICE = 0, 1
STOP_AT_FIXPOINT, KEEP_LEVELS, UNTYPED, RESULT_ON_HOST, NO_SUMMARY_EDGES = 1, 2, 4, 8, 16
BACKWARD, BOTH_DIRECTIONS = 32, 64
PREV_LEVEL_EDGES = 128
DIRECTION_FLAGS = {"out": 0, "in": BACKWARD, "both": BOTH_DIRECTIONS}
K_UNBOUNDED = 0xFFFFFFFF
OP_ADD_V, OP_MOD_V, OP_DEL_V, OP_ADD_E, OP_MOD_E, OP_DEL_E = 1, 2, 3, 4, 5, 6

_p = ctypes.c_void_p
_u32 = ctypes.c_uint32
_u64 = ctypes.c_uint64


class BsimGraph(ctypes.Structure):
    _fields_ = [("n_vertices", _u32), ("label_bytes", _u32), ("n_edges", _u64),
                ("row_off", _p), ("targets", _p), ("labels", _p), ("type_off", _p),
                ("type_ids", _p), ("alive", _p), ("mem_kind", _u32), ("reserved", _u32)]


class BsimParams(ctypes.Structure):
    _fields_ = [("k_max", _u32), ("flags", _u32)]


class BsimResult(ctypes.Structure):
    _fields_ = [("n_vertices", _u32), ("k_done", _u32), ("fixpoint", _u32), ("n_blocks", _u32),
                ("n_summary_edges", _u64), ("mem_kind", _u32), ("n_iter_launches", _u32),
                ("hashes", _p), ("block_ids", _p), ("block_sizes", _p),
                ("blocks_per_iter", ctypes.POINTER(_u32)), ("se_src", _p), ("se_label", _p),
                ("se_dst", _p), ("ms_stage", ctypes.c_float), ("ms_iterate", ctypes.c_float),
                ("ms_finalize", ctypes.c_float), ("ms_total", ctypes.c_float),
                ("ms_iter_kernels", ctypes.c_float), ("ms_hub_kernels", ctypes.c_float),
                ("n_timed_launches", _u32), ("n_split_launches", _u32), ("ms_resolve", ctypes.c_float),
                ("priv", _p)]


class BsimUpdate(ctypes.Structure):
    _fields_ = [("op", _u32), ("u", _u32), ("w", _u32), ("label", _u32), ("new_label", _u32),
                ("n_types", _u32), ("types", ctypes.POINTER(_u32))]


class BsimRequest(ctypes.Structure):
    _fields_ = [("kind", _u32), ("keep_state", _u32), ("graph", ctypes.POINTER(BsimGraph)),
                ("params", BsimParams), ("state", _p), ("ops", ctypes.POINTER(BsimUpdate)), ("n_ops", _u64)]


class BsimServerStats(ctypes.Structure):
    _fields_ = [("submitted", _u64), ("completed", _u64), ("failed", _u64), ("bytes_in_use", _u64),
                ("bytes_budget", _u64), ("p50_ms", ctypes.c_double * 3), ("p99_ms", ctypes.c_double * 3),
                ("busy_ms", ctypes.c_double)]


class BsimNoallocOut(ctypes.Structure):
    _fields_ = [("hashes", _p), ("block_ids", _p), ("block_sizes", _p), ("se_src", _p), ("se_label", _p),
                ("se_dst", _p), ("blocks_per_iter", _p), ("blocks_per_iter_cap", _u32), ("k_done", _u32),
                ("fixpoint", _u32), ("n_blocks", _u32), ("n_summary_edges", _u64), ("scratch_used", _u64)]


REQ_SUMMARIZE, REQ_UPDATE = 1, 2

EXPORTS = {
    "bsim_status_string": (ctypes.c_char_p, [ctypes.c_int]),
    "bsim_ctx_create": (ctypes.c_int, [ctypes.c_int, _p, ctypes.POINTER(_p)]),
    "bsim_ctx_free": (None, [_p]),
    "bsim_last_error": (ctypes.c_char_p, [_p]),
    "bsim_ctx_set_option": (ctypes.c_int, [_p, ctypes.c_char_p, ctypes.c_int64]),
    "bsim_ctx_get_option": (ctypes.c_int, [_p, ctypes.c_char_p, ctypes.POINTER(ctypes.c_int64)]),
    "bsim_option_names": (ctypes.c_char_p, []),
    "bsim_summarize": (ctypes.c_int, [_p, ctypes.POINTER(BsimGraph), ctypes.POINTER(BsimParams),
                                      ctypes.POINTER(_p), ctypes.POINTER(ctypes.POINTER(BsimResult))]),
    "bsim_summarize_labels": (ctypes.c_int, [_p, ctypes.POINTER(BsimGraph), ctypes.POINTER(BsimParams),
                                             _p, _u32, ctypes.POINTER(ctypes.POINTER(BsimResult))]),
    "bsim_source_payload": (ctypes.c_int, [_p, ctypes.POINTER(BsimResult), _p, _u32, _p, _p,
                                           ctypes.POINTER(_u64)]),
    "bsim_diff_snapshots": (ctypes.c_int, [_p, ctypes.POINTER(BsimGraph), ctypes.POINTER(BsimGraph),
                                           ctypes.POINTER(ctypes.POINTER(BsimUpdate)), ctypes.POINTER(_u64)]),
    "bsim_updates_free": (None, [ctypes.POINTER(BsimUpdate)]),
    "bsim_result_free": (None, [ctypes.POINTER(BsimResult)]),
    "bsim_result_copy": (ctypes.c_int, [ctypes.POINTER(BsimResult), ctypes.c_char_p, _p, _u32]),
    "bsim_apply_updates": (ctypes.c_int, [_p, ctypes.POINTER(BsimUpdate), _u64,
                                          ctypes.POINTER(ctypes.POINTER(BsimResult))]),
    "bsim_state_graph": (ctypes.c_int, [_p, ctypes.POINTER(BsimGraph)]),
    "bsim_state_device_graph": (ctypes.c_int, [_p, ctypes.POINTER(BsimGraph)]),
    "bsim_host_free": (None, [_p]),
    "bsim_state_free": (None, [_p]),
    "bsim_state_save": (ctypes.c_int, [_p, ctypes.c_char_p]),
    "bsim_state_load": (ctypes.c_int, [_p, ctypes.c_char_p, ctypes.POINTER(_p),
                                       ctypes.POINTER(ctypes.POINTER(BsimResult))]),
    "bsim_server_create": (ctypes.c_int, [ctypes.c_int, _u64, _u32, ctypes.POINTER(_p)]),
    "bsim_server_submit": (ctypes.c_int, [_p, ctypes.POINTER(BsimRequest), ctypes.POINTER(_u64)]),
    "bsim_server_poll": (ctypes.c_int, [_p, _u64, ctypes.c_int, ctypes.POINTER(ctypes.POINTER(BsimResult)),
                                        ctypes.POINTER(_p)]),
    "bsim_server_stats_get": (ctypes.c_int, [_p, ctypes.POINTER(BsimServerStats)]),
    "bsim_server_set_option": (ctypes.c_int, [_p, ctypes.c_char_p, ctypes.c_int64]),
    "bsim_server_release_state": (ctypes.c_int, [_p, _p]),
    "bsim_server_free": (None, [_p]),
    "bsim_probe_gather": (ctypes.c_int, [_p, _p, _u64, _p, _u32, _u32, ctypes.POINTER(ctypes.c_float)]),
    "bsim_probe_copy": (ctypes.c_int, [_p, _u64, _u32, ctypes.POINTER(ctypes.c_float)]),
    "bsim_noalloc_scratch_bytes": (_u64, []),
    "bsim_summarize_noalloc": (ctypes.c_int, [_p, ctypes.POINTER(BsimGraph), ctypes.POINTER(BsimParams),
                                              ctypes.POINTER(BsimNoallocOut)]),
    "bsim_batch_summarize": (ctypes.c_int, [_p, ctypes.POINTER(BsimGraph), _u32,
                                            ctypes.POINTER(BsimParams),
                                            ctypes.POINTER(ctypes.POINTER(BsimResult))]),
}

_lib = None


def lib() -> ctypes.CDLL:
    """Load libbsim.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError("libbsim.so is not built; run `python -m paper_2111_12493_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in EXPORTS.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


class BsimError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__("%s (%d): %s" % (lib().bsim_status_string(status).decode(), status, msg))
        self.status = status


def _torch():
    import torch
    return torch


class Context:
    """A library context bound to one device and one HIP stream."""

    def __init__(self, device: int = 0, stream=None):
        torch = _torch()
        if stream is None:
            stream = torch.cuda.current_stream(device)
        self.stream = stream
        self.device = device
        h = _p()
        rc = lib().bsim_ctx_create(device, _p(stream.cuda_stream), ctypes.byref(h))
        if rc != OK:
            raise BsimError(rc, "context creation failed")
        self.handle = h

    def close(self):
        if self.handle:
            lib().bsim_ctx_free(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def last_error(self) -> str:
        return lib().bsim_last_error(self.handle).decode()

    def check(self, rc: int):
        if rc != OK:
            raise BsimError(rc, self.last_error())

    def set_option(self, name: str, value: int):
        self.check(lib().bsim_ctx_set_option(self.handle, name.encode(), int(value)))

    def get_option(self, name: str) -> int:
        v = ctypes.c_int64()
        self.check(lib().bsim_ctx_get_option(self.handle, name.encode(), ctypes.byref(v)))
        return int(v.value)


class PackedGraph:
    """Keeps a graph's bsim_graph struct packed once, so that a call over
    thousands of graphs marshals each with one bytes copy.  Assigning any
    attribute of the graph drops the packed copy (the arrays' addresses are
    read again on the next call); subclasses build the struct in
    _make_struct."""

    def __setattr__(self, name, value):
        object.__setattr__(self, name, value)
        if name != "_packed":
            object.__setattr__(self, "_packed", None)

    def packed(self) -> bytes:
        p = getattr(self, "_packed", None)
        if p is None:
            p = bytes(self._make_struct())
            object.__setattr__(self, "_packed", p)
        return p

    def struct(self) -> BsimGraph:
        return BsimGraph.from_buffer_copy(self.packed())


def pack_graphs(graphs: Sequence) -> ctypes.Array:
    """A bsim_graph array (at least one entry) for the given graphs."""
    G = len(graphs)
    raw = b"".join(g.packed() if isinstance(g, PackedGraph) else bytes(g.struct()) for g in graphs)
    if G == 0:
        return (BsimGraph * 1)()
    return (BsimGraph * G).from_buffer_copy(raw)


class DeviceGraph(PackedGraph):
    """A graph whose CSR arrays are torch tensors on the GPU (bit-preserving
    signed views of the unsigned arrays)."""

    def __init__(self, g, device: str = "cuda"):
        torch = _torch()
        self.n = int(g.n)
        self.m = int(g.m)
        lab = np.ascontiguousarray(g.lab)
        self.label_bytes = 2 if lab.dtype == np.uint16 else 4

        def up(a, dt):
            a = np.ascontiguousarray(a)
            if a.size == 0:
                a = np.zeros(1, dtype=a.dtype)
            return torch.from_numpy(a.view(dt)).to(device)

        self.row_off = up(np.asarray(g.row_off, dtype=np.uint32), np.int32)
        self.tgt = up(np.asarray(g.tgt, dtype=np.uint32), np.int32)
        self.lab = up(lab if self.label_bytes == 2 else lab.astype(np.uint32),
                      np.int16 if self.label_bytes == 2 else np.int32)
        self.type_off = up(np.asarray(g.typ_off, dtype=np.uint32), np.int32)
        self.typ = up(np.asarray(g.typ, dtype=np.uint32), np.int32)
        self.alive = None if g.alive is None else up(np.asarray(g.alive, dtype=np.uint8), np.uint8)

    def _make_struct(self) -> BsimGraph:
        return BsimGraph(self.n, self.label_bytes, self.m, self.row_off.data_ptr(), self.tgt.data_ptr(),
                         self.lab.data_ptr(), self.type_off.data_ptr(), self.typ.data_ptr(),
                         self.alive.data_ptr() if self.alive is not None else None, MEM_DEVICE, 0)


class HostGraph(PackedGraph):
    """A graph given as host numpy arrays (the library copies it)."""

    def __init__(self, g):
        self.n = int(g.n)
        self.m = int(g.m)
        lab = np.ascontiguousarray(g.lab)
        self.label_bytes = 2 if lab.dtype == np.uint16 else 4
        self.row_off = np.ascontiguousarray(g.row_off, dtype=np.uint32)
        self.tgt = np.ascontiguousarray(g.tgt, dtype=np.uint32)
        self.lab = lab if self.label_bytes == 2 else np.ascontiguousarray(lab, dtype=np.uint32)
        self.type_off = np.ascontiguousarray(g.typ_off, dtype=np.uint32)
        self.typ = np.ascontiguousarray(g.typ, dtype=np.uint32)
        if self.typ.size == 0:
            self.typ = np.zeros(1, dtype=np.uint32)
        self.alive = None if g.alive is None else np.ascontiguousarray(g.alive, dtype=np.uint8)

    def _make_struct(self) -> BsimGraph:
        def ptr(a):
            return None if a is None else a.ctypes.data

        return BsimGraph(self.n, self.label_bytes, self.m, ptr(self.row_off), ptr(self.tgt),
                         ptr(self.lab), ptr(self.type_off), ptr(self.typ), ptr(self.alive),
                         MEM_HOST, 0)


class Result:
    """Owner of a bsim_result; arrays are fetched to numpy on demand."""

    FIELDS = {"hashes": np.uint64, "block_ids": np.uint32, "block_sizes": np.uint32,
              "se_src": np.uint32, "se_label": np.uint32, "se_dst": np.uint32}

    SCALARS = ("n_vertices", "k_done", "fixpoint", "n_blocks", "n_summary_edges", "n_iter_launches", "mem_kind",
               "ms_stage", "ms_iterate", "ms_finalize", "ms_total", "ms_iter_kernels", "ms_hub_kernels",
               "n_timed_launches", "n_split_launches", "ms_resolve")

    def __init__(self, ptr):
        # the struct's fields are read on first use (a batched call returns
        # thousands of results, most of which are never looked at)
        self.ptr = ptr

    def __getattr__(self, name):
        if name in Result.SCALARS or name == "blocks_per_iter":
            if not self.__dict__.get("ptr"):
                raise AttributeError("%s of a result freed before it was read" % name)
            self._load()
            return self.__dict__[name]
        raise AttributeError(name)

    def _load(self):
        r = self.ptr.contents
        d = self.__dict__
        for f in Result.SCALARS:
            d[f] = getattr(r, f)
        k = r.k_done + 1
        d["blocks_per_iter"] = (np.ctypeslib.as_array(r.blocks_per_iter, shape=(k,)).astype(np.uint32)
                                if r.blocks_per_iter else np.zeros(0, dtype=np.uint32))

    def _len(self, field):
        if field in ("hashes", "block_ids"):
            return self.n_vertices
        if field == "block_sizes":
            return self.n_blocks
        return self.n_summary_edges

    def fetch(self, field: str) -> np.ndarray:
        out = np.zeros(max(self._len(field), 1), dtype=self.FIELDS[field])
        rc = lib().bsim_result_copy(self.ptr, field.encode(), out.ctypes.data, MEM_HOST)
        if rc != OK:
            raise BsimError(rc, "result copy of " + field)
        return out[:self._len(field)]

    def fetch_device(self, field: str):
        """The field copied into a new torch tensor on the current GPU
        (int64 / int32 views of the unsigned arrays)."""
        torch = _torch()
        dt = torch.int64 if self.FIELDS[field] == np.uint64 else torch.int32
        out = torch.zeros(max(self._len(field), 1), dtype=dt, device="cuda")
        rc = lib().bsim_result_copy(self.ptr, field.encode(), out.data_ptr(), MEM_DEVICE)
        if rc != OK:
            raise BsimError(rc, "result copy of " + field)
        torch.cuda.synchronize()
        return out[:self._len(field)]

    def to_dict(self) -> Dict:
        d = dict(k_done=self.k_done, fixpoint=self.fixpoint, n_blocks=self.n_blocks,
                 blocks_per_iter=self.blocks_per_iter)
        for f in self.FIELDS:
            key = {"se_label": "se_label"}.get(f, f)
            d[key] = self.fetch(f)
        return d

    def free(self):
        if self.__dict__.get("ptr"):
            if "k_done" not in self.__dict__:
                self._load()  # the fields stay readable after the free
            lib().bsim_result_free(self.ptr)
            self.ptr = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def summarize(ctx: Context, graph, k_max: int = K_UNBOUNDED, stop_at_fixpoint: bool = True,
              untyped: bool = False, summary_edges: bool = True, result_on_host: bool = False,
              direction: str = "out", labels=None, prev_level_edges: bool = False) -> Result:
    """bsim_summarize on a DeviceGraph or HostGraph; with ``labels`` (the
    kept label set) bsim_summarize_labels.  ``direction`` is "out", "in"
    (BSIM_BACKWARD) or "both" (BSIM_BOTH_DIRECTIONS); ``prev_level_edges``
    sets BSIM_PREV_LEVEL_EDGES (summary edges into the targets'
    (k_done-1)-classes)."""
    flags = (STOP_AT_FIXPOINT if stop_at_fixpoint else 0) | (UNTYPED if untyped else 0) | \
            (0 if summary_edges else NO_SUMMARY_EDGES) | (RESULT_ON_HOST if result_on_host else 0) | \
            DIRECTION_FLAGS[direction] | (PREV_LEVEL_EDGES if prev_level_edges else 0)
    gs = graph.struct()
    params = BsimParams(int(k_max), flags)
    out = ctypes.POINTER(BsimResult)()
    if labels is None:
        ctx.check(lib().bsim_summarize(ctx.handle, ctypes.byref(gs), ctypes.byref(params), None,
                                       ctypes.byref(out)))
    else:
        ids = np.ascontiguousarray(np.asarray(list(labels), dtype=np.uint32).reshape(-1))
        ctx.check(lib().bsim_summarize_labels(ctx.handle, ctypes.byref(gs), ctypes.byref(params),
                                              ids.ctypes.data_as(_p) if ids.size else None, ids.size,
                                              ctypes.byref(out)))
    return Result(out)


def summarize_noalloc(ctx: Context, graph: "DeviceGraph", k_max: int = K_UNBOUNDED, stop_at_fixpoint: bool = True,
                      untyped: bool = False, summary_edges: bool = True) -> dict:
    """bsim_summarize_noalloc on a DeviceGraph: the outputs are torch device
    tensors allocated here (the call itself allocates no device memory);
    returns the result as a dict like Result.to_dict, plus scratch_used."""
    torch = _torch()
    n, m = graph.n, graph.m
    dev = graph.tgt.device
    hashes = torch.zeros(max(n, 1), dtype=torch.int64, device=dev)
    bids = torch.zeros(max(n, 1), dtype=torch.int32, device=dev)
    bsz = torch.zeros(max(n, 1), dtype=torch.int32, device=dev)
    se = [torch.zeros(max(m, 1), dtype=torch.int32, device=dev) for _ in range(3)] if summary_edges else None
    k_bound = min(int(k_max), n + 1) if stop_at_fixpoint else int(k_max)
    bpi = np.zeros(k_bound + 1, dtype=np.uint32)
    o = BsimNoallocOut()
    o.hashes, o.block_ids, o.block_sizes = hashes.data_ptr(), bids.data_ptr(), bsz.data_ptr()
    if se is not None:
        o.se_src, o.se_label, o.se_dst = (t.data_ptr() for t in se)
    o.blocks_per_iter = bpi.ctypes.data
    o.blocks_per_iter_cap = bpi.size
    flags = (STOP_AT_FIXPOINT if stop_at_fixpoint else 0) | (UNTYPED if untyped else 0) | \
            (0 if summary_edges else NO_SUMMARY_EDGES)
    gs = graph.struct()
    params = BsimParams(int(k_max), flags)
    ctx.check(lib().bsim_summarize_noalloc(ctx.handle, ctypes.byref(gs), ctypes.byref(params), ctypes.byref(o)))
    nb, ns = int(o.n_blocks), int(o.n_summary_edges)

    def host(t, count, dt):
        return t[:count].cpu().numpy().view(dt) if count else np.zeros(0, dtype=dt)

    d = dict(k_done=int(o.k_done), fixpoint=int(o.fixpoint), n_blocks=nb,
             blocks_per_iter=bpi[:int(o.k_done) + 1].copy(), hashes=host(hashes, n, np.uint64),
             block_ids=host(bids, n, np.uint32), block_sizes=host(bsz, nb, np.uint32),
             scratch_used=int(o.scratch_used))
    if se is not None:
        d["se_src"], d["se_label"], d["se_dst"] = (host(t, ns, np.uint32) for t in se)
    return d


def probe_gather(ctx: Context, graph: "DeviceGraph", h, reps: int = 10) -> float:
    """ms per pass of the gather probe over graph's targets, gathering from
    the device tensor h (int64, at least graph.n entries)."""
    ms = ctypes.c_float()
    ctx.check(lib().bsim_probe_gather(ctx.handle, graph.tgt.data_ptr(), graph.m, h.data_ptr(), graph.n, reps,
                                      ctypes.byref(ms)))
    return ms.value


def probe_copy(ctx: Context, nbytes: int, reps: int = 10) -> float:
    """ms per pass of a STREAM-style copy of nbytes bytes."""
    ms = ctypes.c_float()
    ctx.check(lib().bsim_probe_copy(ctx.handle, int(nbytes), reps, ctypes.byref(ms)))
    return ms.value


def diff_snapshots(ctx: Context, before, after, as_tuples: bool = True):
    """bsim_diff_snapshots on two snapshots (DeviceGraph, HostGraph or a
    BsimGraph such as State.device_graph()): the
    ordered batch as tuples, ("add_v", types), ("mod_v", u, types),
    ("del_e", u, l, w), ("add_e", u, l, w), ("del_v", u); with as_tuples
    False only the number of operations."""
    gb = before if isinstance(before, BsimGraph) else before.struct()
    ga = after if isinstance(after, BsimGraph) else after.struct()
    ops = ctypes.POINTER(BsimUpdate)()
    n = _u64()
    ctx.check(lib().bsim_diff_snapshots(ctx.handle, ctypes.byref(gb), ctypes.byref(ga), ctypes.byref(ops),
                                        ctypes.byref(n)))
    out = []
    try:
        if not as_tuples:
            return n.value
        for i in range(n.value):
            o = ops[i]
            types = [int(o.types[j]) for j in range(o.n_types)]
            if o.op == OP_ADD_V:
                out.append(("add_v", types))
            elif o.op == OP_MOD_V:
                out.append(("mod_v", int(o.u), types))
            elif o.op == OP_DEL_V:
                out.append(("del_v", int(o.u)))
            elif o.op == OP_DEL_E:
                out.append(("del_e", int(o.u), int(o.label), int(o.w)))
            else:
                out.append(("add_e", int(o.u), int(o.label), int(o.w)))
    finally:
        if ops:
            lib().bsim_updates_free(ops)
    return out


def source_payload(ctx: Context, result: "Result", source_labels):
    """bsim_source_payload with host arrays: the distinct (block, source
    label) pairs of a result, sorted, as two numpy uint32 arrays."""
    n = result.n_vertices
    lab = np.ascontiguousarray(np.asarray(source_labels, dtype=np.uint32).reshape(-1))
    if lab.size != n:
        raise ValueError("one source label per vertex")
    ob = np.zeros(max(n, 1), dtype=np.uint32)
    ol = np.zeros(max(n, 1), dtype=np.uint32)
    cnt = _u64()
    ctx.check(lib().bsim_source_payload(ctx.handle, result.ptr, lab.ctypes.data_as(_p), MEM_HOST,
                                        ob.ctypes.data_as(_p), ol.ctypes.data_as(_p), ctypes.byref(cnt)))
    return ob[:cnt.value].copy(), ol[:cnt.value].copy()


# The summary models of the paper's experiments as parameters of the same
# refinement (no stop test, exact k):
#   class collection      vertices with the same type set (k = 0);
#   attribute collection  vertices with the same set of outgoing edge labels
#                         (untyped, k = 1);
#   SchemEX               the same type set and the same (edge label,
#                         neighbour type set) pairs (typed, k = 1).
SUMMARY_MODELS = {
    "class_collection": dict(k_max=0, untyped=False),
    "attribute_collection": dict(k_max=1, untyped=True),
    "schemex": dict(k_max=1, untyped=False),
}


def summarize_model(ctx: Context, graph, model: str, **kw) -> Result:
    """bsim_summarize with the parameters of one of SUMMARY_MODELS."""
    return summarize(ctx, graph, stop_at_fixpoint=False, **SUMMARY_MODELS[model], **kw)


# ---------------------------------------------------------------- update batches

UPDATE_DTYPE = np.dtype({"names": ["op", "u", "w", "label", "new_label", "n_types", "types"],
                         "formats": [np.uint32] * 6 + [np.uint64],
                         "offsets": [0, 4, 8, 12, 16, 20, 24], "itemsize": 32})
assert UPDATE_DTYPE.itemsize == ctypes.sizeof(BsimUpdate)

OP_CODES = {"add_v": OP_ADD_V, "mod_v": OP_MOD_V, "del_v": OP_DEL_V, "add_e": OP_ADD_E,
            "mod_e": OP_MOD_E, "del_e": OP_DEL_E}


class UpdateBatch:
    """An ordered batch of update operations laid out as bsim_update[].

    Built from tuples: ("add_v", types), ("mod_v", u, types), ("del_v", u),
    ("add_e", u, label, w), ("mod_e", u, label, w, new_label), ("del_e", u, label, w).
    """

    def __init__(self, ops: Sequence[tuple]):
        n = len(ops)
        self.arr = np.zeros(max(n, 1), dtype=UPDATE_DTYPE)[:n]
        lists = []
        for i, o in enumerate(ops):
            kind = o[0]
            rec = self.arr[i]
            rec["op"] = OP_CODES[kind]
            if kind == "add_v":
                lists.append((i, o[1]))
            elif kind in ("mod_v", "del_v"):
                rec["u"] = o[1]
                if kind == "mod_v":
                    lists.append((i, o[2]))
            else:
                rec["u"], rec["label"], rec["w"] = o[1], o[2], o[3]
                if kind == "mod_e":
                    rec["new_label"] = o[4]
        sizes = [len(t) for _, t in lists]
        self.types = np.zeros(max(sum(sizes), 1), dtype=np.uint32)
        pos = 0
        for (i, t), c in zip(lists, sizes):
            self.types[pos:pos + c] = np.asarray(t, dtype=np.uint32)
            self.arr[i]["n_types"] = c
            self.arr[i]["types"] = self.types.ctypes.data + 4 * pos
            pos += c

    @classmethod
    def from_op_arrays(cls, d: dict) -> "UpdateBatch":
        """From the arrays of graphgen.update_ops (op, u, w, label, new_label, t_off, t_ids)."""
        n = len(d["op"])
        arr = np.zeros(max(n, 1), dtype=UPDATE_DTYPE)[:n]
        for f in ("op", "u", "w", "label", "new_label"):
            arr[f] = d[f]
        types = np.ascontiguousarray(d["t_ids"], dtype=np.uint32)
        if types.size == 0:
            types = np.zeros(1, dtype=np.uint32)
        t_off = np.asarray(d["t_off"], dtype=np.uint64)
        arr["n_types"] = np.diff(t_off).astype(np.uint32)
        arr["types"] = np.uint64(types.ctypes.data) + 4 * t_off[:-1]
        return cls.from_arrays(arr, types)

    @classmethod
    def from_arrays(cls, arr: np.ndarray, types: np.ndarray) -> "UpdateBatch":
        """Wrap a prepared UPDATE_DTYPE array whose type pointers index `types`."""
        b = cls.__new__(cls)
        b.arr, b.types = arr, types
        return b

    def __len__(self):
        return len(self.arr)


class State:
    """A resident incremental state (bsim_summarize with state_out), with its
    first result in ``self.result``."""

    def __init__(self, ctx: Context, graph, k_max: int, stop_at_fixpoint: bool = False,
                 untyped: bool = False, summary_edges: bool = True):
        flags = (STOP_AT_FIXPOINT if stop_at_fixpoint else 0) | (UNTYPED if untyped else 0) | \
                (0 if summary_edges else NO_SUMMARY_EDGES)
        self.ctx = ctx
        gs = graph.struct()
        params = BsimParams(int(k_max), flags)
        out = ctypes.POINTER(BsimResult)()
        h = _p()
        ctx.check(lib().bsim_summarize(ctx.handle, ctypes.byref(gs), ctypes.byref(params), ctypes.byref(h),
                                       ctypes.byref(out)))
        self.handle = h
        self.result = Result(out)

    def apply(self, batch: UpdateBatch) -> Result:
        out = ctypes.POINTER(BsimResult)()
        ptr = batch.arr.ctypes.data_as(ctypes.POINTER(BsimUpdate)) if len(batch) else None
        self.ctx.check(lib().bsim_apply_updates(self.handle, ptr, len(batch), ctypes.byref(out)))
        return Result(out)

    def graph(self):
        """The state's current graph as a host graphgen.Graph."""
        from . import graphgen as gg
        g = BsimGraph()
        self.ctx.check(lib().bsim_state_graph(self.handle, ctypes.byref(g)))
        n, m = g.n_vertices, g.n_edges

        def take(ptr, count, dt):
            a = np.ctypeslib.as_array(ctypes.cast(ptr, ctypes.POINTER(np.ctypeslib.as_ctypes_type(dt))),
                                      shape=(max(count, 1),))[:count].copy()
            return a

        try:
            row_off = take(g.row_off, n + 1, np.uint32).astype(np.uint64)
            tgt = take(g.targets, m, np.uint32)
            lab = take(g.labels, m, np.uint16 if g.label_bytes == 2 else np.uint32)
            typ_off = take(g.type_off, n + 1, np.uint32).astype(np.uint64)
            typ = take(g.type_ids, int(typ_off[-1]) if n + 1 else 0, np.uint32)
            alive = take(g.alive, n, np.uint8)
        finally:
            for p in (g.row_off, g.targets, g.labels, g.type_off, g.type_ids, g.alive):
                lib().bsim_host_free(p)
        return gg.Graph(n=n, row_off=row_off, tgt=tgt, lab=lab, typ_off=typ_off, typ=typ, alive=alive)

    def save(self, path) -> None:
        """bsim_state_save: the state's graph, parameters and levels to a host file."""
        self.ctx.check(lib().bsim_state_save(self.handle, os.fsencode(path)))

    @classmethod
    def load(cls, ctx: Context, path) -> "State":
        """bsim_state_load: a state read back from a file written by save();
        its summary is in ``result``."""
        out = ctypes.POINTER(BsimResult)()
        h = _p()
        ctx.check(lib().bsim_state_load(ctx.handle, os.fsencode(path), ctypes.byref(h), ctypes.byref(out)))
        st = cls.__new__(cls)
        st.ctx, st.handle, st.result = ctx, h, Result(out)
        return st

    def device_graph(self) -> BsimGraph:
        g = BsimGraph()
        self.ctx.check(lib().bsim_state_device_graph(self.handle, ctypes.byref(g)))
        return g

    def free(self):
        if getattr(self, "handle", None):
            self.result.free()
            lib().bsim_state_free(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


class _Borrowed:
    """A bsim_graph struct passed through as is (e.g. a state's device view)."""

    def __init__(self, gs: BsimGraph):
        self.gs = gs

    def struct(self) -> BsimGraph:
        return self.gs


def batch_summarize(ctx: Context, graphs: Sequence, k_max: int = K_UNBOUNDED, stop_at_fixpoint: bool = True,
                    untyped: bool = False, summary_edges: bool = True,
                    result_on_host: bool = False, direction: str = "out") -> List[Result]:
    """bsim_batch_summarize: one refinement run over many graphs (all
    DeviceGraph or all HostGraph, same label width); one Result per graph."""
    flags = (STOP_AT_FIXPOINT if stop_at_fixpoint else 0) | (UNTYPED if untyped else 0) | \
            (0 if summary_edges else NO_SUMMARY_EDGES) | (RESULT_ON_HOST if result_on_host else 0) | \
            DIRECTION_FLAGS[direction]
    G = len(graphs)
    arr = pack_graphs(graphs)
    outs = (ctypes.POINTER(BsimResult) * max(G, 1))()
    params = BsimParams(int(k_max), flags)
    ctx.check(lib().bsim_batch_summarize(ctx.handle, arr, G, ctypes.byref(params), outs))
    return [Result(outs[i]) for i in range(G)]



def _check(rc: int, what: str):
    if rc != OK:
        raise BsimError(rc, what)


class Server:
    """bsim_server: continuous batching of summarize and update requests."""

    def __init__(self, device: int = 0, mem_budget: int = 0, workers: int = 4):
        h = _p()
        _check(lib().bsim_server_create(device, int(mem_budget), int(workers), ctypes.byref(h)), "server create")
        self.handle = h
        self._keep = {}

    def submit_summarize(self, graph, k_max: int = K_UNBOUNDED, stop_at_fixpoint: bool = True,
                         untyped: bool = False, summary_edges: bool = True, keep_state: bool = False,
                         direction: str = "out", prev_level_edges: bool = False) -> int:
        flags = (STOP_AT_FIXPOINT if stop_at_fixpoint else 0) | (UNTYPED if untyped else 0) | \
                (0 if summary_edges else NO_SUMMARY_EDGES) | DIRECTION_FLAGS[direction] | \
                (PREV_LEVEL_EDGES if prev_level_edges else 0)
        gs = graph.struct()
        req = BsimRequest(REQ_SUMMARIZE, 1 if keep_state else 0, ctypes.pointer(gs), BsimParams(int(k_max), flags),
                          None, None, 0)
        t = _u64()
        _check(lib().bsim_server_submit(self.handle, ctypes.byref(req), ctypes.byref(t)), "submit")
        if graph.struct().mem_kind == MEM_DEVICE:
            self._keep[t.value] = graph  # device arrays are borrowed until completion
        return t.value

    def submit_update(self, state, batch: "UpdateBatch") -> int:
        ptr = batch.arr.ctypes.data_as(ctypes.POINTER(BsimUpdate)) if len(batch) else None
        req = BsimRequest(REQ_UPDATE, 0, None, BsimParams(0, 0), state, ptr, len(batch))
        t = _u64()
        _check(lib().bsim_server_submit(self.handle, ctypes.byref(req), ctypes.byref(t)), "submit")
        return t.value

    def poll(self, ticket: int, wait: bool = True):
        """(Result, state handle or None); raises BsimError for a failed request."""
        out = ctypes.POINTER(BsimResult)()
        st = _p()
        rc = lib().bsim_server_poll(self.handle, ticket, 1 if wait else 0, ctypes.byref(out), ctypes.byref(st))
        self._keep.pop(ticket, None)
        _check(rc, "request %d" % ticket)
        return Result(out), (st.value or None)

    def stats(self) -> dict:
        s = BsimServerStats()
        _check(lib().bsim_server_stats_get(self.handle, ctypes.byref(s)), "stats")
        return dict(submitted=s.submitted, completed=s.completed, failed=s.failed,
                    bytes_in_use=s.bytes_in_use, bytes_budget=s.bytes_budget,
                    p50_ms=list(s.p50_ms), p99_ms=list(s.p99_ms), busy_ms=s.busy_ms)

    def set_option(self, name: str, value: int):
        _check(lib().bsim_server_set_option(self.handle, name.encode(), int(value)), "server option " + name)

    def release_state(self, state):
        _check(lib().bsim_server_release_state(self.handle, state), "release state")

    def free(self):
        if getattr(self, "handle", None):
            lib().bsim_server_free(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def state_graph(state_handle):
    """Host copy of any state's graph (as graphgen.Graph)."""
    s = State.__new__(State)
    s.handle = state_handle

    class _C:
        @staticmethod
        def check(rc):
            _check(rc, "state graph")

    s.ctx = _C()
    g = s.graph()
    s.handle = None
    return g
