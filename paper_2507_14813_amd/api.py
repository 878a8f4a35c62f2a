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
DEVICE_INPUT = 2
HOST_ONLY = 4

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
                ("similarity", ctypes.c_double), ("delta", ctypes.c_int64),
                ("n_deltas", ctypes.c_int32)]


class CountOpts(ctypes.Structure):
    _fields_ = [("mode", ctypes.c_int32), ("blocks", ctypes.c_int32),
                ("chunk", ctypes.c_int32), ("queues", ctypes.c_int32),
                ("stream", ctypes.c_void_p), ("roots", ctypes.c_void_p),
                ("n_roots", ctypes.c_int64),
                ("elapsed_ms", ctypes.POINTER(ctypes.c_float)),
                ("stats", ctypes.c_void_p), ("sched", ctypes.c_int32),
                ("leaf_scan", ctypes.c_int32), ("model", ctypes.c_void_p),
                ("root_cost", ctypes.c_void_p), ("sample", ctypes.c_int32),
                ("stop", ctypes.c_void_p), ("max_chunks", ctypes.c_int64),
                ("cursor", ctypes.c_void_p), ("wave_clock", ctypes.c_void_p),
                ("wave_clock_len", ctypes.c_int64), ("epoch_idle", ctypes.c_int32),
                ("max_epochs", ctypes.c_int32), ("epoch_contexts", ctypes.c_void_p)]


class TuneResult(ctypes.Structure):
    _fields_ = [("blocks", ctypes.c_int32), ("chunk", ctypes.c_int32),
                ("queues", ctypes.c_int32), ("leaf_scan", ctypes.c_int32),
                ("ms", ctypes.c_float), ("default_ms", ctypes.c_float),
                ("from_cache", ctypes.c_int32), ("trials", ctypes.c_int32)]


class CpuOpts(ctypes.Structure):
    _fields_ = [("mode", ctypes.c_int32), ("threads", ctypes.c_int32),
                ("codegen", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("roots", ctypes.c_void_p), ("n_roots", ctypes.c_int64),
                ("elapsed_ms", ctypes.POINTER(ctypes.c_double))]


class Advice(ctypes.Structure):
    _fields_ = [("co_mine", ctypes.c_int32), ("bipartite", ctypes.c_int32),
                ("similarity", ctypes.c_double), ("threshold", ctypes.c_double)]


class Cursor(ctypes.Structure):
    """Resume point of a stopped count (``mg_cursor``)."""
    _fields_ = [("head", ctypes.c_uint64 * 8), ("n_roots", ctypes.c_int64),
                ("chunk", ctypes.c_int32), ("queues", ctypes.c_int32),
                ("started", ctypes.c_int32), ("done", ctypes.c_int32)]

    def __init__(self):
        super().__init__()
        lib().mg_cursor_init(ctypes.byref(self))


STAT_NAMES = ("win_list", "win_all", "ent_list", "ent_all", "push", "credit", "roots")


class BatchOpts(ctypes.Structure):
    _fields_ = [("blocks", ctypes.c_int32), ("item_roots", ctypes.c_int32),
                ("use_graph", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("stream", ctypes.c_void_p), ("model", ctypes.c_void_p)]


class BatchInfo(ctypes.Structure):
    _fields_ = [("n_jobs", ctypes.c_int32), ("total_motifs", ctypes.c_int32),
                ("total_roots", ctypes.c_int64), ("n_items", ctypes.c_int64),
                ("item_roots", ctypes.c_int32), ("blocks", ctypes.c_int32),
                ("graph_captured", ctypes.c_int32), ("depth", ctypes.c_int32),
                ("tuned_ms", ctypes.c_float), ("learned", ctypes.c_int32),
                ("predict_ms", ctypes.c_float)]


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
        L.mg_tree_create_multi.argtypes = [p, p, i32, p, i32, ctypes.POINTER(p)]
        L.mg_tree_info.argtypes = [p, ctypes.POINTER(TreeInfo)]
        L.mg_tree_destroy.argtypes = [p]
        L.mg_tree_destroy.restype = None
        L.mg_count_opts_init.argtypes = [ctypes.POINTER(CountOpts)]
        L.mg_count_opts_init.restype = None
        L.mg_count.argtypes = [p, p, ctypes.POINTER(CountOpts), p]
        L.mg_cursor_init.argtypes = [p]
        L.mg_cursor_init.restype = None
        L.mg_count_noalloc.argtypes = [p, p, ctypes.POINTER(CountOpts), p]
        L.mg_tune.argtypes = [p, p, ctypes.c_char_p, p, ctypes.POINTER(TuneResult)]
        L.mg_enumerate.argtypes = [p, p, p, p, i64, ctypes.POINTER(i64)]
        L.mg_cpu_opts_init.argtypes = [ctypes.POINTER(CpuOpts)]
        L.mg_cpu_opts_init.restype = None
        L.mg_count_cpu.argtypes = [p, p, ctypes.POINTER(CpuOpts), p]
        L.mg_comine_advice.argtypes = [p, p, i32, ctypes.POINTER(Advice)]
        L.mg_last_error.restype = ctypes.c_char_p
        L.mg_model_create.argtypes = [ctypes.c_uint64, ctypes.POINTER(p)]
        L.mg_model_get_weights.argtypes = [p, p]
        L.mg_model_set_weights.argtypes = [p, p]
        L.mg_model_get_moments.argtypes = [p, p, p]
        L.mg_model_destroy.argtypes = [p]
        L.mg_model_destroy.restype = None
        L.mg_root_features.argtypes = [p, p, p, i64, p]
        L.mg_model_predict.argtypes = [p, p, i64, p]
        L.mg_model_train.argtypes = [p, p, p, i64, i32, ctypes.c_float, ctypes.c_uint64, p]
        L.mg_batch_opts_init.argtypes = [ctypes.POINTER(BatchOpts)]
        L.mg_batch_opts_init.restype = None
        L.mg_batch_create.argtypes = [p, p, i32, ctypes.POINTER(BatchOpts), ctypes.POINTER(p)]
        L.mg_batch_count.argtypes = [p, p, ctypes.POINTER(ctypes.c_float)]
        L.mg_batch_info.argtypes = [p, ctypes.POINTER(BatchInfo)]
        L.mg_batch_destroy.argtypes = [p]
        L.mg_batch_destroy.restype = None
        L.mg_count_batch.argtypes = [p, p, i32, ctypes.POINTER(BatchOpts), p]
        for f in ("mg_set_allocator", "mg_graph_create", "mg_graph_info",
                  "mg_tree_create", "mg_tree_create_multi", "mg_tree_info", "mg_count", "mg_count_noalloc", "mg_tune", "mg_enumerate", "mg_count_cpu",
                  "mg_comine_advice", "mg_batch_create",
                  "mg_batch_count", "mg_batch_info", "mg_count_batch", "mg_model_create", "mg_model_get_weights",
                  "mg_model_set_weights", "mg_model_get_moments", "mg_root_features", "mg_model_predict",
                  "mg_model_train"):
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
                 torch_allocator=True, host_only=False):
        L = lib()
        if torch_allocator and not host_only:
            use_torch_allocator()
        flags = (SORTED_BY_T if sorted_by_t else 0) | (HOST_ONLY if host_only else 0)
        if all(hasattr(x, "is_cuda") and x.is_cuda for x in (src, dst, t)):
            # torch tensors on the GPU: handed over as device pointers
            import torch
            self._src = src.to(torch.int32).contiguous()
            self._dst = dst.to(torch.int32).contiguous()
            self._t = t.to(torch.int64).contiguous()
            ptrs = [x.data_ptr() for x in (self._src, self._dst, self._t)]
            flags |= DEVICE_INPUT
        else:
            self._src = np.ascontiguousarray(src, dtype=np.int32)
            self._dst = np.ascontiguousarray(dst, dtype=np.int32)
            self._t = np.ascontiguousarray(t, dtype=np.int64)
            ptrs = [_p(x).value for x in (self._src, self._dst, self._t)]
        h = ctypes.c_void_p()
        _check(L.mg_graph_create(ptrs[0], ptrs[1], ptrs[2], len(self._src), int(n_nodes), flags,
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
    """The MG-Tree of a motif group for a window delta (``mg_tree_create``),
    or for several windows counted in one search when ``delta`` is a list
    (``mg_tree_create_multi``; counts then come as one row per window)."""

    def __init__(self, motifs, delta):
        L = lib()
        ks = np.array([len(m) for m in motifs], dtype=np.int32)
        uv = np.array([x for m in motifs for e in m for x in e], dtype=np.int32)
        if uv.size == 0:
            uv = np.zeros(2, dtype=np.int32)
        h = ctypes.c_void_p()
        self.multi = isinstance(delta, (list, tuple, np.ndarray))
        if self.multi:
            ds = np.ascontiguousarray(delta, dtype=np.int64)
            _check(L.mg_tree_create_multi(_p(uv), _p(ks), len(ks), _p(ds), len(ds),
                                          ctypes.byref(h)))
            self.n_deltas = len(ds)
        else:
            _check(L.mg_tree_create(_p(uv), _p(ks), len(ks), int(delta), ctypes.byref(h)))
            self.n_deltas = 1
        self._h = h
        self._L = L
        self._done = _exiting
        self.n_motifs = len(ks)

    def shape_counts(self, flat):
        """Counts as mg_count returns them -> 1-D per motif, or windows x motifs."""
        return flat.reshape(self.n_deltas, self.n_motifs) if self.multi else flat

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
          queues=0, stream=None, timed=False, stats=False, root_cost=False, model=None,
          leaf_scan=0, sample=0, stop=None, max_chunks=0, cursor=None, wave_clock=None,
          epoch_idle=0, max_epochs=0, epoch_contexts=None):
    """Exact count per motif (``mg_count``), in the tree's motif order.

    ``mode``: "comine" (one search over the MG-Tree) or "per_motif" (one search
    per motif).  ``roots``: optional root positions (time order).  ``model``:
    a ``Model`` selects the learned schedule (``sample``: it scores one root in
    that many per 64-root segment, 0 = default).  Returns a
    uint64 array; with ``timed`` also the device milliseconds; with ``stats``
    also a dict of search statistics; with ``root_cost`` also the per-root
    cost log (uint64 per edge; both run instrumented kernels).
    ``stop`` (address of an int32 flag in pinned host or device memory),
    ``max_chunks`` and ``cursor`` (a ``Cursor``, updated in place) stop a
    count early and resume it; the counts are then those of this call.
    ``wave_clock`` (a uint64 array, filled in place) receives every wave's
    start and end ticks.  ``epoch_idle`` (percent of the waves) turns on
    epochs: a launch ends once that many waves are idle and the next one
    spreads the root-level candidates left over across all waves;
    ``max_epochs`` bounds the launches and ``epoch_contexts`` (an int64 array
    of that length, filled in place) receives the contexts each one left.
    """
    L = lib()
    o = CountOpts()
    L.mg_count_opts_init(ctypes.byref(o))
    o.mode = {"comine": MODE_COMINE, "per_motif": MODE_PER_MOTIF, "auto": 2}[mode]
    o.blocks = int(blocks)
    o.chunk = int(chunk)
    o.queues = int(queues)
    o.leaf_scan = int(leaf_scan)
    o.sample = int(sample)
    if model is not None:
        o.sched = 1
        o.model = model.handle.value
    o.stream = _default_stream(stream)
    if stop is not None:
        o.stop = int(stop)
    o.max_chunks = int(max_chunks)
    if cursor is not None:
        o.cursor = ctypes.addressof(cursor)
    if wave_clock is not None:
        assert wave_clock.dtype == np.uint64 and wave_clock.flags.c_contiguous
        o.wave_clock = wave_clock.ctypes.data
        o.wave_clock_len = wave_clock.size
    o.epoch_idle = int(epoch_idle)
    o.max_epochs = int(max_epochs)
    if epoch_contexts is not None:
        assert epoch_contexts.dtype == np.int64 and epoch_contexts.flags.c_contiguous
        assert epoch_contexts.size >= (max_epochs if max_epochs > 0 else 16)
        o.epoch_contexts = epoch_contexts.ctypes.data
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
    out = np.zeros(tree.n_motifs * tree.n_deltas, dtype=np.uint64)
    _check(L.mg_count(graph.handle, tree.handle, ctypes.byref(o), _p(out)))
    res = [tree.shape_counts(out)]
    if timed:
        res.append(float(ms.value))
    if stats:
        res.append({k: int(v) for k, v in zip(STAT_NAMES, st)})
    if root_cost:
        res.append(rcost[:graph.n_edges])
    return res[0] if len(res) == 1 else tuple(res)


def count_cpu(graph: Graph, tree: Tree, mode="comine", threads=0, codegen=True, roots=None,
              timed=False):
    """``mg_count_cpu``: the CPU backend (generated and compiled nested loops
    per trie level, or the interpreted trie with ``codegen=False``).  Counts
    as ``count``; with ``timed`` also the wall milliseconds of the search."""
    L = lib()
    o = CpuOpts()
    L.mg_cpu_opts_init(ctypes.byref(o))
    o.mode = {"comine": MODE_COMINE, "per_motif": MODE_PER_MOTIF}[mode]
    o.threads = int(threads)
    o.codegen = 1 if codegen else 0
    r = None
    if roots is not None:
        r = np.ascontiguousarray(roots, dtype=np.int64)
        o.roots = r.ctypes.data if r.size else _p(np.zeros(1, np.int64)).value
        o.n_roots = r.size
    ms = ctypes.c_double(0.0)
    if timed:
        o.elapsed_ms = ctypes.pointer(ms)
    out = np.zeros(tree.n_motifs * tree.n_deltas, dtype=np.uint64)
    _check(L.mg_count_cpu(graph.handle, tree.handle, ctypes.byref(o), _p(out)))
    out = tree.shape_counts(out)
    return (out, float(ms.value)) if timed else out


def comine_advice(graph: Graph, tree: Tree, platform="gpu"):
    """``mg_comine_advice``: the paper's heuristic for whether co-mining pays."""
    a = Advice()
    _check(lib().mg_comine_advice(graph.handle, tree.handle,
                                  {"gpu": 0, "cpu": 1}[platform], ctypes.byref(a)))
    return {f: getattr(a, f) for f, _ in Advice._fields_}


def enumerate_matches(graph: Graph, tree: Tree, stream=None):
    """``mg_enumerate``: every match, as (motif index array, edges array of
    shape n x 5 with -1 past each motif's length), in no particular order;
    edges are indices into the arrays the graph was created from."""
    L = lib()
    n = ctypes.c_int64(0)
    st = _default_stream(stream)
    _check(L.mg_enumerate(graph.handle, tree.handle, st, None, 0, ctypes.byref(n)))
    rec = np.zeros((max(1, n.value), 6), dtype=np.int32)
    _check(L.mg_enumerate(graph.handle, tree.handle, st, _p(rec), n.value, ctypes.byref(n)))
    rec = rec[:n.value]
    return rec[:, 0].copy(), rec[:, 1:].copy()


def tune(graph: Graph, tree: Tree, cache=None, stream=None):
    """``mg_tune``: launch settings for ``count`` (a dict with blocks, chunk,
    queues, leaf_scan), plus the timings, read from or appended to the JSON
    lines file ``cache`` when given."""
    r = TuneResult()
    _check(lib().mg_tune(graph.handle, tree.handle,
                         None if cache is None else os.fsencode(cache),
                         _default_stream(stream), ctypes.byref(r)))
    return {f: getattr(r, f) for f, _ in TuneResult._fields_}


def count_noalloc(graph: Graph, tree: Tree, blocks=0, chunk=0, queues=0, stream=None,
                  stats=False, leaf_scan=0, stop=None, max_chunks=0):
    """``mg_count_noalloc``: co-mining over every root with the library's
    static device scratch (no device allocation).  The tree must have been
    counted on this device before.  Returns the uint64 counts, with ``stats``
    also the statistics dict."""
    L = lib()
    o = CountOpts()
    L.mg_count_opts_init(ctypes.byref(o))
    o.blocks, o.chunk, o.queues = int(blocks), int(chunk), int(queues)
    o.leaf_scan = int(leaf_scan)
    o.stream = _default_stream(stream)
    if stop is not None:
        o.stop = int(stop)
    o.max_chunks = int(max_chunks)
    st = np.zeros(len(STAT_NAMES), dtype=np.uint64)
    if stats:
        o.stats = st.ctypes.data
    out = np.zeros(tree.n_motifs * tree.n_deltas, dtype=np.uint64)
    _check(L.mg_count_noalloc(graph.handle, tree.handle, ctypes.byref(o), _p(out)))
    out = tree.shape_counts(out)
    if stats:
        return out, {k: int(v) for k, v in zip(STAT_NAMES, st)}
    return out


NFEATURES = 16
MODEL_PARAMS = 10497


class Model:
    """Root-cost MLP (``mg_model_*``): BF16 weights, FP32 accumulation."""

    def __init__(self, seed=0, weights=None):
        L = lib()
        h = ctypes.c_void_p()
        _check(L.mg_model_create(int(seed), ctypes.byref(h)))
        self._h, self._L, self._done = h, L, _exiting
        if weights is not None:
            self.set_weights(weights)

    @property
    def handle(self):
        return self._h

    def weights(self):
        w = np.zeros(MODEL_PARAMS, dtype=np.float32)
        _check(self._L.mg_model_get_weights(self._h, _p(w)))
        return w

    def set_weights(self, w):
        w = np.ascontiguousarray(w, dtype=np.float32)
        assert w.size == MODEL_PARAMS
        _check(self._L.mg_model_set_weights(self._h, _p(w)))

    def moments(self):
        """Adam's first and second moments, in the parameter layout."""
        m1 = np.zeros(MODEL_PARAMS, dtype=np.float32)
        m2 = np.zeros(MODEL_PARAMS, dtype=np.float32)
        _check(self._L.mg_model_get_moments(self._h, _p(m1), _p(m2)))
        return m1, m2

    def predict(self, feats):
        f = np.ascontiguousarray(feats, dtype=np.float32).reshape(-1, NFEATURES)
        out = np.zeros(len(f), dtype=np.float32)
        _check(self._L.mg_model_predict(self._h, _p(f), len(f), _p(out)))
        return out

    def train(self, feats, labels, epochs=5, lr=1e-3, seed=0):
        f = np.ascontiguousarray(feats, dtype=np.float32).reshape(-1, NFEATURES)
        y = np.ascontiguousarray(labels, dtype=np.float32)
        assert len(y) == len(f)
        loss = np.zeros(max(1, epochs), dtype=np.float32)
        _check(self._L.mg_model_train(self._h, _p(f), _p(y), len(f), int(epochs), float(lr),
                                      int(seed), _p(loss)))
        return loss[:epochs]

    def close(self):
        if getattr(self, "_h", None) and not self._done():
            self._L.mg_model_destroy(self._h)
        self._h = None

    __del__ = close


def root_features(graph: Graph, tree: Tree, roots=None):
    """Per-root features (n x 16) the cost model reads (``mg_root_features``)."""
    L = lib()
    if roots is None:
        n, rp = graph.n_edges, None
    else:
        r = np.ascontiguousarray(roots, dtype=np.int64)
        n, rp = len(r), (_p(r) if len(r) else _p(np.zeros(1, np.int64)))
    out = np.zeros((max(1, n), NFEATURES), dtype=np.float32)
    _check(L.mg_root_features(graph.handle, tree.handle, rp, n, _p(out)))
    return out[:n]


def count_batch(graphs, trees, item_roots=0, blocks=0, stream=None, model=None):
    """``mg_count_batch``: a batch planned, counted once and released in one
    call.  Returns the counts per job, as ``Batch.count``."""
    L = lib()
    assert len(graphs) == len(trees) and len(graphs) > 0
    o = BatchOpts()
    L.mg_batch_opts_init(ctypes.byref(o))
    o.item_roots, o.blocks = int(item_roots), int(blocks)
    o.stream = _default_stream(stream)
    if model is not None:
        o.model = model.handle.value
    gh = (ctypes.c_void_p * len(graphs))(*[g.handle.value for g in graphs])
    th = (ctypes.c_void_p * len(trees))(*[t.handle.value for t in trees])
    sizes = [t.n_motifs * t.n_deltas for t in trees]
    out = np.zeros(sum(sizes), dtype=np.uint64)
    _check(L.mg_count_batch(gh, th, len(graphs), ctypes.byref(o), _p(out)))
    parts, k = [], 0
    for n, t in zip(sizes, trees):
        parts.append(t.shape_counts(out[k:k + n]))
        k += n
    return parts


class Batch:
    """Many (graph, tree) jobs counted by one persistent launch, replayed as a
    captured HIP graph (``mg_batch_*``).  Keeps its graphs and trees alive."""

    def __init__(self, graphs, trees, item_roots=0, blocks=0, use_graph=True, stream=None,
                 model=None):
        L = lib()
        assert len(graphs) == len(trees) and len(graphs) > 0
        self._graphs, self._trees = list(graphs), list(trees)
        o = BatchOpts()
        L.mg_batch_opts_init(ctypes.byref(o))
        o.item_roots = int(item_roots)
        o.blocks = int(blocks)
        o.use_graph = 1 if use_graph else 0
        o.stream = _default_stream(stream)
        if model is not None:
            o.model = model.handle.value
            self._model = model
        gh = (ctypes.c_void_p * len(graphs))(*[g.handle.value for g in graphs])
        th = (ctypes.c_void_p * len(trees))(*[t.handle.value for t in trees])
        h = ctypes.c_void_p()
        _check(L.mg_batch_create(gh, th, len(graphs), ctypes.byref(o), ctypes.byref(h)))
        self._h = h
        self._L = L
        self._done = _exiting
        self.sizes = [t.n_motifs * t.n_deltas for t in trees]

    def info(self) -> dict:
        bi = BatchInfo()
        _check(self._L.mg_batch_info(self._h, ctypes.byref(bi)))
        return {f: getattr(bi, f) for f, _ in BatchInfo._fields_}

    def count(self, timed=False):
        """Counts per job (list of uint64 arrays), plus device ms when timed."""
        out = np.zeros(sum(self.sizes), dtype=np.uint64)
        ms = ctypes.c_float(0.0)
        _check(self._L.mg_batch_count(self._h, _p(out), ctypes.byref(ms) if timed else None))
        parts, k = [], 0
        for n, t in zip(self.sizes, self._trees):
            parts.append(t.shape_counts(out[k:k + n]))
            k += n
        return (parts, float(ms.value)) if timed else parts

    def close(self):
        if getattr(self, "_h", None) and not self._done():
            self._L.mg_batch_destroy(self._h)
        self._h = None

    __del__ = close
