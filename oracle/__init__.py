"""CPU oracle for delta-temporal motif counts -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, the smoke check in ``__graft_entry__`` and the benchmark's
CPU-baseline leg may import this package.  It shares no code with the HIP path
and imports nothing from it.

* ``count`` (``oracle.c``): plain per-motif depth-first matching (the paper's
  Algorithm 1 with the readings listed in ``oracle.c``), OpenMP over roots.
* ``brute.count`` (``brute.py``): the definition itself, enumerating every
  time-increasing k-tuple of edges; tiny inputs only.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "liboracle.so")
_lib = None
_mutants = {}


def build(force: bool = True, mutant: int = 0) -> str:
    """Compile ``oracle.c`` with gcc into ``liboracle.so`` (next to it).

    ``mutant`` > 0 builds a library with a planted mistake (tests only)."""
    so = _SO if mutant == 0 else os.path.join(_HERE, "liboracle_mut%d.so" % mutant)
    if force or not os.path.exists(so):
        tmp = so + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-shared", "-fPIC",
                               "-std=c99", "-Wall", "-DORACLE_MUTANT=%d" % mutant,
                               os.path.join(_HERE, "oracle.c"), "-o", tmp])
        os.replace(tmp, so)
    return so


def _load(mutant: int = 0):
    global _lib
    if mutant:
        if mutant not in _mutants:
            _mutants[mutant] = _bind(ctypes.CDLL(build(force=True, mutant=mutant)))
        return _mutants[mutant]
    if _lib is None:
        if not os.path.exists(_SO):
            build()
        _lib = _bind(ctypes.CDLL(_SO))
    return _lib


def _bind(lib):
    p = ctypes.c_void_p
    lib.oracle_count.argtypes = [ctypes.c_int64, p, p, p, ctypes.c_int32,
                                 ctypes.c_int32, p, ctypes.c_int64, p,
                                 ctypes.c_int64, p, p, ctypes.c_int32, p]
    lib.oracle_count.restype = ctypes.c_int
    lib.oracle_max_threads.restype = ctypes.c_int
    lib.oracle_graph_new.argtypes = [ctypes.c_int64, p, p, p, ctypes.c_int32]
    lib.oracle_graph_new.restype = p
    lib.oracle_graph_free.argtypes = [p]
    lib.oracle_graph_free.restype = None
    lib.oracle_graph_count.argtypes = [p, ctypes.c_int32, p, ctypes.c_int64, p,
                                       ctypes.c_int64, p, p, p, p, ctypes.c_int32, p]
    lib.oracle_graph_count.restype = ctypes.c_int
    return lib


def max_threads() -> int:
    return int(_load().oracle_max_threads())


def _ptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def count(src, dst, t, n_nodes, motif, delta, roots=None, per_root=False,
          level=False, threads=0, mutant=0):
    """Count one motif (sequence of (u, v) pairs).

    ``roots`` are positions in the stably time-sorted edge list.  Returns the
    total, or ``(total, per_root, level)`` when either log is asked for
    (``level[r, j]`` = partial matches of the first j+1 motif edges from root
    r).
    """
    src = np.ascontiguousarray(src, dtype=np.int32)
    dst = np.ascontiguousarray(dst, dtype=np.int32)
    t = np.ascontiguousarray(t, dtype=np.int64)
    uv = np.ascontiguousarray(np.asarray(motif, dtype=np.int32).reshape(-1))
    k = len(uv) // 2
    n = len(src)
    r = None if roots is None else np.ascontiguousarray(roots, dtype=np.int64)
    nr = n if r is None else len(r)
    pr = np.zeros(nr, dtype=np.uint64) if per_root else None
    lv = np.zeros((nr, k), dtype=np.uint64) if level else None
    tot = np.zeros(1, dtype=np.uint64)
    rc = _load(mutant).oracle_count(n, _ptr(src), _ptr(dst), _ptr(t),
                                    int(n_nodes), k, _ptr(uv), int(delta), _ptr(r),
                                    nr, _ptr(pr), _ptr(lv), int(threads), _ptr(tot))
    if rc != 0:
        raise ValueError("oracle_count failed with status %d" % rc)
    if per_root or level:
        return int(tot[0]), pr, lv
    return int(tot[0])


def count_many(src, dst, t, n_nodes, motifs, delta, roots=None, threads=0):
    """Per-motif counts (list of ints), one oracle pass per motif."""
    return [count(src, dst, t, n_nodes, m, delta, roots=roots, threads=threads)
            for m in motifs]


class OracleGraph:
    """A graph loaded (sorted, adjacency built) once for many oracle counts.

    ``mutant`` > 0 loads a library with a planted mistake (tests only)."""

    def __init__(self, src, dst, t, n_nodes, mutant=0):
        src = np.ascontiguousarray(src, dtype=np.int32)
        dst = np.ascontiguousarray(dst, dtype=np.int32)
        t = np.ascontiguousarray(t, dtype=np.int64)
        self._lib = _load(mutant)
        self._h = self._lib.oracle_graph_new(len(src), _ptr(src), _ptr(dst), _ptr(t),
                                             int(n_nodes))
        if not self._h:
            raise ValueError("oracle_graph_new failed (bad ids or out of memory)")
        self.n_edges = len(src)

    def count(self, motif, delta, roots=None, per_root=False, level=False,
              windows=False, windows_per_root=False, threads=0):
        """Like ``count``; ``windows`` adds the per-edge window-entry totals,
        ``windows_per_root`` the same per root (n_roots x k)."""
        uv = np.ascontiguousarray(np.asarray(motif, dtype=np.int32).reshape(-1))
        k = len(uv) // 2
        r = None if roots is None else np.ascontiguousarray(roots, dtype=np.int64)
        nr = self.n_edges if r is None else len(r)
        pr = np.zeros(nr, dtype=np.uint64) if per_root else None
        lv = np.zeros((nr, k), dtype=np.uint64) if level else None
        wn = np.zeros(k, dtype=np.uint64) if windows else None
        wr = np.zeros((nr, k), dtype=np.uint64) if windows_per_root else None
        tot = np.zeros(1, dtype=np.uint64)
        rc = self._lib.oracle_graph_count(self._h, k, _ptr(uv), int(delta), _ptr(r), nr,
                                          _ptr(pr), _ptr(lv), _ptr(wn), _ptr(wr),
                                          int(threads), _ptr(tot))
        if rc != 0:
            raise ValueError("oracle_graph_count failed with status %d" % rc)
        if not (per_root or level or windows or windows_per_root):
            return int(tot[0])
        out = [int(tot[0])]
        if per_root:
            out.append(pr)
        if level:
            out.append(lv)
        if windows:
            out.append(wn)
        if windows_per_root:
            out.append(wr)
        return tuple(out)

    def close(self):
        if getattr(self, "_h", None):
            self._lib.oracle_graph_free(self._h)
            self._h = None

    __del__ = close
