"""Python binding of the C ABI in ``include/mayura.h`` (argument marshalling
only: graph ingest, tree construction and counting all run in ``libmayura.so``,
the search itself in its HIP kernels).

PyTorch supplies device memory (its caching allocator is registered through
``mg_set_allocator``) and the stream (the current torch stream by default).
There is no fallback: without the built library every call raises.
"""
from __future__ import annotations

import atexit
import ctypes
import os
import sys

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmayura.so")

MODE_COMINE = 0
MODE_PER_MOTIF = 1
SORTED_BY_T = 1

_STATUS = {0: "MG_OK", -1: "MG_EINVAL", -2: "MG_ENOMEM", -3: "MG_EDEVICE",
           -4: "MG_EUNSUPPORTED", -5: "MG_EINTERNAL"}


class MayuraError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("%s: %s" % (_STATUS.get(status, status), msg))
        self.status = status


class GraphInfo(ctypes.Structure):
    _fields_ = [("n_edges", ctypes.c_int64), ("n_nodes", ctypes.c_int32),
                ("self_loops", ctypes.c_int64), ("t_min", ctypes.c_int64),
                ("t_max", ctypes.c_int64), ("time_bytes", ctypes.c_int32),
                ("device_bytes", ctypes.c_int64)]


class TreeInfo(ctypes.Structure):
    _fields_ = [("n_motifs", ctypes.c_int32), ("n_distinct", ctypes.c_int32),
                ("n_prefixes", ctypes.c_int32), ("n_nodes", ctypes.c_int32),
                ("depth", ctypes.c_int32), ("root_edges", ctypes.c_int32),
                ("similarity", ctypes.c_double), ("delta", ctypes.c_int64)]


class CountOpts(ctypes.Structure):
    _fields_ = [("mode", ctypes.c_int32), ("blocks", ctypes.c_int32),
                ("chunk", ctypes.c_int32), ("queues", ctypes.c_int32),
                ("stream", ctypes.c_void_p), ("roots", ctypes.c_void_p),
                ("n_roots", ctypes.c_int64),
                ("elapsed_ms", ctypes.POINTER(ctypes.c_float)),
                ("stats", ctypes.c_void_p), ("root_cost", ctypes.c_void_p)]


STAT_NAMES = ("win_list", "win_all", "ent_list", "ent_all", "push", "credit", "roots")


_ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p,
                             ctypes.c_void_p)
_RELEASE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p)

_lib = None
_callbacks = None
# Handles still alive at interpreter exit are left to the process end:
# releasing them would call back into a torch that is being torn down.  The
# flag is a list so that objects keep a reference to it after module globals
# are cleared during finalisation.
_EXIT = [False]


@atexit.register
def _mark_exit():
    _EXIT[0] = True


def _exiting(flag=_EXIT):
    return flag[0] or sys.is_finalizing()


def lib():
    """The loaded ``libmayura.so``; raises if it was not built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError("libmayura.so is not built (run `python -m "
                              "paper_2507_14813_amd.build`): %s" % LIB_PATH)
        L = ctypes.CDLL(LIB_PATH)
        p, i32, i64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
        L.mg_set_allocator.argtypes = [_ALLOC_FN, _RELEASE_FN, p]
        L.mg_graph_create.argtypes = [p, p, p, i64, i32, ctypes.c_uint32, p,
                                      ctypes.POINTER(p)]
        L.mg_graph_info.argtypes = [p, ctypes.POINTER(GraphInfo)]
        L.mg_graph_destroy.argtypes = [p]
        L.mg_graph_destroy.restype = None
        L.mg_tree_create.argtypes = [p, p, i32, i64, ctypes.POINTER(p)]
        L.mg_tree_info.argtypes = [p, ctypes.POINTER(TreeInfo)]
        L.mg_tree_destroy.argtypes = [p]
        L.mg_tree_destroy.restype = None
        L.mg_count_opts_init.argtypes = [ctypes.POINTER(CountOpts)]
        L.mg_count_opts_init.restype = None
        L.mg_count.argtypes = [p, p, ctypes.POINTER(CountOpts), p]
        L.mg_last_error.restype = ctypes.c_char_p
        for f in ("mg_set_allocator", "mg_graph_create", "mg_graph_info",
                  "mg_tree_create", "mg_tree_info", "mg_count"):
            getattr(L, f).restype = ctypes.c_int
        _lib = L
    return _lib


def _check(rc):
    if rc != 0:
        raise MayuraError(rc, lib().mg_last_error().decode(errors="replace"))


def use_torch_allocator():
    """Route the library's device allocations through torch's caching allocator."""
    global _callbacks
    if _callbacks is not None:
        return
    import torch

    def _alloc(nbytes, stream, ctx):
        try:
            return int(torch.cuda.caching_allocator_alloc(
                int(nbytes), torch.cuda.current_device(),
                int(stream or 0)))
        except Exception:
            return None

    def _release(ptr, stream, ctx, _done=_exiting):
        if not _done():
            torch.cuda.caching_allocator_delete(int(ptr))

    cbs = (_ALLOC_FN(_alloc), _RELEASE_FN(_release))
    _check(lib().mg_set_allocator(cbs[0], cbs[1], None))
    _callbacks = cbs


def _default_stream(stream):
    if stream is not None:
        return int(stream)
    try:
        import torch
        if torch.cuda.is_available():
            return int(torch.cuda.current_stream().cuda_stream)
    except Exception:
        pass
    return 0


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p)


class Graph:
    """A temporal graph resident on the current GPU (``mg_graph_create``)."""

    def __init__(self, src, dst, t, n_nodes, sorted_by_t=False, stream=None,
                 torch_allocator=True):
        L = lib()
        if torch_allocator:
            use_torch_allocator()
        self._src = np.ascontiguousarray(src, dtype=np.int32)
        self._dst = np.ascontiguousarray(dst, dtype=np.int32)
        self._t = np.ascontiguousarray(t, dtype=np.int64)
        h = ctypes.c_void_p()
        _check(L.mg_graph_create(_p(self._src), _p(self._dst), _p(self._t),
                                 len(self._src), int(n_nodes),
                                 SORTED_BY_T if sorted_by_t else 0,
                                 _default_stream(stream), ctypes.byref(h)))
        self._h = h
        self._L = L
        self._done = _exiting
        self.n_edges = len(self._src)
        del self._src, self._dst, self._t

    @property
    def handle(self):
        return self._h

    def info(self) -> dict:
        gi = GraphInfo()
        _check(lib().mg_graph_info(self._h, ctypes.byref(gi)))
        return {f: getattr(gi, f) for f, _ in GraphInfo._fields_}

    def close(self):
        if getattr(self, "_h", None) and not self._done():
            self._L.mg_graph_destroy(self._h)
        self._h = None

    __del__ = close


class Tree:
    """The MG-Tree of a motif group for a window delta (``mg_tree_create``)."""

    def __init__(self, motifs, delta):
        L = lib()
        ks = np.array([len(m) for m in motifs], dtype=np.int32)
        uv = np.array([x for m in motifs for e in m for x in e], dtype=np.int32)
        if uv.size == 0:
            uv = np.zeros(2, dtype=np.int32)
        h = ctypes.c_void_p()
        _check(L.mg_tree_create(_p(uv), _p(ks), len(ks), int(delta), ctypes.byref(h)))
        self._h = h
        self._L = L
        self._done = _exiting
        self.n_motifs = len(ks)

    @property
    def handle(self):
        return self._h

    def info(self) -> dict:
        ti = TreeInfo()
        _check(lib().mg_tree_info(self._h, ctypes.byref(ti)))
        return {f: getattr(ti, f) for f, _ in TreeInfo._fields_}

    def close(self):
        if getattr(self, "_h", None) and not self._done():
            self._L.mg_tree_destroy(self._h)
        self._h = None

    __del__ = close


def count(graph: Graph, tree: Tree, mode="comine", roots=None, blocks=0, chunk=0,
          queues=0, stream=None, timed=False, stats=False, root_cost=False):
    """Exact count per motif (``mg_count``), in the tree's motif order.

    ``mode``: "comine" (one search over the MG-Tree) or "per_motif" (one search
    per motif).  ``roots``: optional root positions (time order).  Returns a
    uint64 array; with ``timed`` also the device milliseconds; with ``stats``
    also a dict of search statistics; with ``root_cost`` also the per-root
    cost log (uint64 per edge; both run instrumented kernels).
    """
    L = lib()
    o = CountOpts()
    L.mg_count_opts_init(ctypes.byref(o))
    o.mode = {"comine": MODE_COMINE, "per_motif": MODE_PER_MOTIF}[mode]
    o.blocks = int(blocks)
    o.chunk = int(chunk)
    o.queues = int(queues)
    o.stream = _default_stream(stream)
    r = None
    if roots is not None:
        r = np.ascontiguousarray(roots, dtype=np.int64)
        o.roots = r.ctypes.data if r.size else _p(np.zeros(1, np.int64)).value
        o.n_roots = r.size
    ms = ctypes.c_float(0.0)
    if timed:
        o.elapsed_ms = ctypes.pointer(ms)
    st = np.zeros(len(STAT_NAMES), dtype=np.uint64)
    if stats:
        o.stats = st.ctypes.data
    rcost = None
    if root_cost:
        rcost = np.zeros(max(1, graph.n_edges), dtype=np.uint64)
        o.root_cost = rcost.ctypes.data
    out = np.zeros(tree.n_motifs, dtype=np.uint64)
    _check(L.mg_count(graph.handle, tree.handle, ctypes.byref(o), _p(out)))
    res = [out]
    if timed:
        res.append(float(ms.value))
    if stats:
        res.append({k: int(v) for k, v in zip(STAT_NAMES, st)})
    if root_cost:
        res.append(rcost[:graph.n_edges])
    return res[0] if len(res) == 1 else tuple(res)
