"""CPU oracle for frequent subgraph mining -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, the smoke check and the benchmark's CPU-baseline leg may
import this package.  It wraps ``liboracle.so`` (plain single-thread C written
from the MNI-support definition, Section 2.2) and a pure-Python brute force for
tiny graphs (``oracle.brute``).  It shares no code with the device library.

Results are lists of ``(size, labels, adj, support)`` sorted by size, then by
the canonical label sequence, then by the canonical adjacency bit sequence;
``labels`` is a tuple of ``size`` canonical vertex labels and ``adj`` has bit
``k`` set when the k-th pair (i<j), counted in row-major upper-triangle order,
is an edge of the canonical form.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

from . import build as _build

_lib = None
MAXN = 9


def _load():
    global _lib
    if _lib is not None:
        return _lib
    # FSM_ORACLE_LIB: another build of the same source (the sanitized one)
    path = os.environ.get("FSM_ORACLE_LIB") or _build.LIB
    if path == _build.LIB and (not os.path.exists(path) or
                               os.path.getmtime(path) < os.path.getmtime(_build.SRC)):
        _build.build()
    lib = ctypes.CDLL(path)
    i32p = ctypes.POINTER(ctypes.c_int32)
    i64p = ctypes.POINTER(ctypes.c_int64)
    u64p = ctypes.POINTER(ctypes.c_uint64)
    lib.oracle_mine.argtypes = [ctypes.c_int64, ctypes.c_int64, i32p, i32p, i32p,
                                ctypes.c_int64, ctypes.c_int32,
                                ctypes.POINTER(ctypes.c_void_p)]
    lib.oracle_mine.restype = ctypes.c_int
    lib.oracle_result_count.argtypes = [ctypes.c_void_p]
    lib.oracle_result_count.restype = ctypes.c_int64
    lib.oracle_result_get.argtypes = [ctypes.c_void_p, i32p, i32p, u64p, i64p]
    lib.oracle_result_get.restype = ctypes.c_int
    lib.oracle_result_levels.argtypes = [ctypes.c_void_p, i64p, i64p]
    lib.oracle_result_levels.restype = ctypes.c_int
    lib.oracle_result_free.argtypes = [ctypes.c_void_p]
    lib.oracle_result_free.restype = None
    lib.oracle_canonical.argtypes = [ctypes.c_int32, i32p, ctypes.c_uint64, i32p, u64p]
    lib.oracle_canonical.restype = ctypes.c_int
    lib.oracle_pattern_support.argtypes = [ctypes.c_int64, ctypes.c_int64, i32p, i32p,
                                           i32p, ctypes.c_int32, i32p, ctypes.c_uint64]
    lib.oracle_pattern_support.restype = ctypes.c_int64
    lib.oracle_mine_ex.argtypes = lib.oracle_mine.argtypes[:7] + [ctypes.c_int32,
                                                                 lib.oracle_mine.argtypes[7]]
    lib.oracle_mine_ex.restype = ctypes.c_int
    lib.oracle_pattern_support_ex.argtypes = lib.oracle_pattern_support.argtypes + [ctypes.c_int32]
    lib.oracle_pattern_support_ex.restype = ctypes.c_int64
    lib.oracle_count_connected.argtypes = [ctypes.c_int64, ctypes.c_int64, i32p, i32p,
                                           i32p, ctypes.c_int32]
    lib.oracle_count_connected.restype = ctypes.c_int64
    lib.oracle_graph_new.argtypes = [ctypes.c_int64, ctypes.c_int64, i32p, i32p, i32p]
    lib.oracle_graph_new.restype = ctypes.c_void_p
    lib.oracle_graph_support.argtypes = [ctypes.c_void_p, ctypes.c_int32, i32p, ctypes.c_uint64,
                                         ctypes.c_int64, ctypes.c_int32]
    lib.oracle_graph_support.restype = ctypes.c_int64
    lib.oracle_graph_free.argtypes = [ctypes.c_void_p]
    lib.oracle_graph_free.restype = None
    _lib = lib
    return lib


def _arr(a):
    a = np.ascontiguousarray(a, dtype=np.int32)
    return a, a.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))


def mine(n_vertices, src, dst, labels, support, max_size, induced=False):
    """Exact frequent patterns of sizes 2..max_size (see module doc);
    ``induced`` selects vertex-induced embeddings."""
    lib = _load()
    s, sp = _arr(src)
    d, dp = _arr(dst)
    lab, lp = _arr(labels)
    h = ctypes.c_void_p()
    rc = lib.oracle_mine_ex(int(n_vertices), int(s.size), sp, dp, lp, int(support),
                            int(max_size), 1 if induced else 0, ctypes.byref(h))
    if rc != 0:
        raise ValueError("oracle_mine rejected its input")
    try:
        cnt = lib.oracle_result_count(h)
        sizes = np.zeros(cnt, np.int32)
        labs = np.zeros((cnt, MAXN), np.int32)
        adj = np.zeros(cnt, np.uint64)
        sup = np.zeros(cnt, np.int64)
        if cnt:
            lib.oracle_result_get(
                h, sizes.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                labs.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                adj.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)),
                sup.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)))
    finally:
        lib.oracle_result_free(h)
    return [(int(sizes[i]), tuple(int(x) for x in labs[i, :sizes[i]]),
             int(adj[i]), int(sup[i])) for i in range(cnt)]


def canonical(labels, adj):
    """Canonical (labels, adj) of one pattern given in any vertex order."""
    lib = _load()
    n = len(labels)
    lab, lp = _arr(labels)
    out = np.zeros(MAXN, np.int32)
    oadj = ctypes.c_uint64()
    rc = lib.oracle_canonical(n, lp, ctypes.c_uint64(adj),
                              out.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                              ctypes.byref(oadj))
    if rc != 0:
        raise ValueError("bad pattern")
    return tuple(int(x) for x in out[:n]), int(oadj.value)


def pattern_support(n_vertices, src, dst, labels, plabels, padj, induced=False):
    """Exact MNI support of one connected pattern."""
    lib = _load()
    s, sp = _arr(src)
    d, dp = _arr(dst)
    lab, lp = _arr(labels)
    pl, plp = _arr(plabels)
    r = lib.oracle_pattern_support_ex(int(n_vertices), int(s.size), sp, dp, lp,
                                      len(plabels), plp, ctypes.c_uint64(padj),
                                      1 if induced else 0)
    if r < 0:
        raise ValueError("bad pattern")
    return int(r)


def count_connected(n_vertices, src, dst, size):
    """Number of connected edge-induced subgraphs with ``size`` vertices."""
    lib = _load()
    s, sp = _arr(src)
    d, dp = _arr(dst)
    lab, lp = _arr(np.zeros(int(n_vertices), np.int32))
    r = lib.oracle_count_connected(int(n_vertices), int(s.size), sp, dp, lp, int(size))
    if r < 0:
        raise ValueError("bad input")
    return int(r)


def pair_index(i, j, n):
    """Bit position of the unordered pair (i<j), row-major upper triangle."""
    return i * n - i * (i + 1) // 2 + (j - i - 1)


class Graph:
    """A normalised input graph kept for many exact support queries."""

    def __init__(self, n_vertices, src, dst, labels):
        lib = _load()
        s, sp = _arr(src)
        d, dp = _arr(dst)
        lab, lp = _arr(labels)
        self._h = lib.oracle_graph_new(int(n_vertices), int(s.size), sp, dp, lp)
        if not self._h:
            raise ValueError("oracle_graph_new rejected its input")

    def support(self, plabels, padj, t=0, induced=False):
        """Exact MNI support of one connected pattern; with t > 0, -1 when
        it is below t (the search stops early)."""
        pl, plp = _arr(plabels)
        r = _load().oracle_graph_support(self._h, len(plabels), plp, ctypes.c_uint64(padj),
                                         int(t), 1 if induced else 0)
        if r == -2:
            raise ValueError("bad pattern")
        return int(r)

    def close(self):
        if self._h:
            _load().oracle_graph_free(self._h)
            self._h = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
