"""Python binding of the MI355X two-vertex-exploration frequent subgraph
miner (``include/fsm.h``).

Argument marshalling only: every step of mining runs in ``libfsm.so``.  The
library must have been built (``paper_2101_07690_amd.build.build()``);
importing this package without it raises, there is no fallback.

Results are lists of ``(size, labels, adj, support)`` ordered by size, then
canonical label sequence, then canonical pair-bit sequence; ``labels`` is a
tuple of the caller's label values of the canonical vertices and ``adj`` has
bit ``k`` set when the k-th vertex pair (i<j), in row-major upper-triangle
order, is an edge.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libfsm.so")

FSM_PLAIN = 0
FSM_BATCHED = 1
FSM_LEARNED = 2
FSM_SAMPLED = 4
FSM_INDUCED = 8
FSM_SINGLE = 16
FSM_SCHEDULE_QUEUE = 0
FSM_SCHEDULE_STATIC = 1
FEATURE_LABELS = 16
FEATURES = 6 + 2 * FEATURE_LABELS
MAX_SIZE = 7

STATUS = {0: "FSM_OK", -1: "FSM_EINVAL", -2: "FSM_ENOMEM", -3: "FSM_EDEVICE",
          -4: "FSM_EOVERFLOW", -5: "FSM_EUNSUPPORTED"}


class FsmError(RuntimeError):
    def __init__(self, code, message):
        super().__init__(f"{STATUS.get(code, code)}: {message}")
        self.code = code


class Code(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("label", ctypes.c_int32 * MAX_SIZE),
                ("adj", ctypes.c_uint32)]


class LevelStats(ctypes.Structure):
    _fields_ = [("parents", ctypes.c_int64), ("work_items", ctypes.c_int64),
                ("candidates", ctypes.c_int64), ("emitted", ctypes.c_int64),
                ("quick_patterns", ctypes.c_int64), ("patterns", ctypes.c_int64),
                ("frequent", ctypes.c_int64), ("stored", ctypes.c_int64),
                ("algorithmic_bytes", ctypes.c_int64),
                ("kernel_ms", ctypes.c_double), ("join_ms", ctypes.c_double),
                ("domain_passes", ctypes.c_int64), ("qp_capacity", ctypes.c_int64),
                ("qp_predicted", ctypes.c_int64), ("rank_slices", ctypes.c_int64),
                ("hash_bytes", ctypes.c_int64), ("canonical_forms", ctypes.c_int64)]


class Stats(ctypes.Structure):
    _fields_ = [("max_size", ctypes.c_int32), ("frequent_labels", ctypes.c_int32),
                ("dropped_self_loops", ctypes.c_int64),
                ("dropped_duplicates", ctypes.c_int64),
                ("filtered_edges", ctypes.c_int64),
                ("level", LevelStats * (MAX_SIZE + 1)),
                ("total_ms", ctypes.c_double), ("batch_chunk", ctypes.c_int32),
                ("batch_chunks", ctypes.c_int32), ("batch_splits", ctypes.c_int32),
                ("captured_levels", ctypes.c_int32), ("captured_graphs", ctypes.c_int32),
                ("level_fallbacks", ctypes.c_int32), ("host_syncs", ctypes.c_int64)]


TUNE_MAX = 16


class Tuning(ctypes.Structure):
    _fields_ = [("chunk_vertices", ctypes.c_int64), ("tiles_per_wave", ctypes.c_int32),
                ("configs", ctypes.c_int32), ("cand_chunk", ctypes.c_int64 * TUNE_MAX),
                ("cand_tiles", ctypes.c_int32 * TUNE_MAX), ("cand_ms", ctypes.c_double * TUNE_MAX)]


class BatchOptions(ctypes.Structure):
    _fields_ = [("max_size", ctypes.c_int32), ("mode", ctypes.c_uint32),
                ("chunk_vertices", ctypes.c_int64), ("disable_pruning", ctypes.c_int32),
                ("tiles_per_wave", ctypes.c_int32), ("hash_capacity_min", ctypes.c_int64),
                ("pattern_capacity_min", ctypes.c_int64), ("model", ctypes.c_void_p),
                ("learn", ctypes.c_int32), ("train_steps", ctypes.c_int32),
                ("lr", ctypes.c_float), ("eager_levels", ctypes.c_int32),
                ("pool_budget_mib", ctypes.c_int64)]


class Options(ctypes.Structure):
    _fields_ = [("support", ctypes.c_int64), ("max_size", ctypes.c_int32),
                ("mode", ctypes.c_uint32), ("disable_pruning", ctypes.c_int32),
                ("schedule", ctypes.c_int32), ("sampling_rate", ctypes.c_double),
                ("seed", ctypes.c_uint64), ("hash_capacity_min", ctypes.c_int64),
                ("pattern_capacity_min", ctypes.c_int64), ("model", ctypes.c_void_p),
                ("record", ctypes.c_int32), ("tiles_per_wave", ctypes.c_int32),
                ("pool_budget_mib", ctypes.c_int64), ("join_threshold", ctypes.c_int64),
                ("match_threshold", ctypes.c_int64), ("force_overflow", ctypes.c_int32),
                ("reserved2", ctypes.c_int32)]


_ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)
_RELEASE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p)

_lib = None


def lib():
    """The loaded library; raises when it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with "
                          "paper_2101_07690_amd.build.build()")
    # One HIP runtime per process: PyTorch ships its own libamdhip64 (same
    # soname).  Loading torch first makes the dynamic loader bind this
    # library to that runtime, so torch streams and allocations are valid
    # here; loading ours first would give torch a second runtime.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    L = ctypes.CDLL(LIB_PATH)
    vp = ctypes.c_void_p
    i32p = ctypes.POINTER(ctypes.c_int32)
    i64p = ctypes.POINTER(ctypes.c_int64)
    L.fsm_set_allocator.argtypes = [_ALLOC_FN, _RELEASE_FN, vp]
    L.fsm_set_allocator.restype = ctypes.c_int
    L.fsm_set_stream.argtypes = [vp]
    L.fsm_set_stream.restype = ctypes.c_int
    L.fsm_build_graph.argtypes = [ctypes.c_int64, ctypes.c_int64, i32p, i32p, i32p,
                                  ctypes.POINTER(vp)]
    L.fsm_build_graph.restype = ctypes.c_int
    L.fsm_graph_vertices.argtypes = [vp]
    L.fsm_graph_vertices.restype = ctypes.c_int64
    L.fsm_graph_edges.argtypes = [vp]
    L.fsm_graph_edges.restype = ctypes.c_int64
    L.fsm_mine.argtypes = [vp, ctypes.c_int64, ctypes.c_int32, ctypes.c_uint32,
                           ctypes.POINTER(vp)]
    L.fsm_mine.restype = ctypes.c_int
    L.fsm_mine_ex.argtypes = [vp, ctypes.POINTER(Options), ctypes.POINTER(vp)]
    L.fsm_mine_ex.restype = ctypes.c_int
    L.fsm_mine_noalloc.argtypes = [vp, ctypes.POINTER(Options), ctypes.c_int64, i32p,
                                   ctypes.POINTER(Code), i64p, i64p, ctypes.POINTER(Stats)]
    L.fsm_mine_noalloc.restype = ctypes.c_int
    L.fsm_mine_batch.argtypes = [ctypes.POINTER(vp), ctypes.c_int32, i64p, ctypes.c_int32,
                                 ctypes.c_uint32, ctypes.POINTER(vp)]
    L.fsm_mine_batch.restype = ctypes.c_int
    L.fsm_mine_batch_ex.argtypes = [ctypes.POINTER(vp), ctypes.c_int32, i64p,
                                    ctypes.POINTER(BatchOptions), ctypes.POINTER(vp)]
    L.fsm_mine_batch_ex.restype = ctypes.c_int
    L.fsm_tune_batch.argtypes = [ctypes.POINTER(vp), ctypes.c_int32, i64p, ctypes.c_int32,
                                 ctypes.POINTER(Tuning)]
    L.fsm_tune_batch.restype = ctypes.c_int
    L.fsm_reset_tuning.argtypes = []
    L.fsm_reset_tuning.restype = ctypes.c_int
    L.fsm_result_count.argtypes = [vp]
    L.fsm_result_count.restype = ctypes.c_int64
    L.fsm_result_training_count.argtypes = [vp]
    L.fsm_result_training_count.restype = ctypes.c_int64
    L.fsm_result_training_rows.argtypes = [vp, ctypes.POINTER(ctypes.c_float),
                                           ctypes.POINTER(ctypes.c_float), i32p]
    L.fsm_result_training_rows.restype = ctypes.c_int
    L.fsm_result_patterns.argtypes = [vp, i32p, i32p, ctypes.POINTER(Code), i64p]
    L.fsm_result_patterns.restype = ctypes.c_int
    L.fsm_result_stats.argtypes = [vp, ctypes.POINTER(Stats)]
    L.fsm_result_stats.restype = ctypes.c_int
    L.fsm_graph_free.argtypes = [vp]
    L.fsm_graph_free.restype = None
    L.fsm_result_free.argtypes = [vp]
    L.fsm_result_free.restype = None
    L.fsm_last_error.argtypes = []
    L.fsm_last_error.restype = ctypes.c_char_p
    L.fsm_dissect.argtypes = [ctypes.c_int32, i32p, ctypes.c_uint32,
                              ctypes.POINTER(ctypes.c_uint32), i32p]
    L.fsm_dissect.restype = ctypes.c_int
    L.fsm_proposal_thresholds.argtypes = [ctypes.POINTER(ctypes.c_float), ctypes.c_int64,
                                          ctypes.c_double, ctypes.POINTER(ctypes.c_uint64)]
    L.fsm_proposal_thresholds.restype = ctypes.c_int
    L.fsm_key_graph.argtypes = [ctypes.c_uint64, ctypes.c_int32, ctypes.c_int32, i32p]
    L.fsm_key_graph.restype = ctypes.c_int
    f32p = ctypes.POINTER(ctypes.c_float)
    L.fsm_model_param_count.argtypes = [ctypes.c_int32]
    L.fsm_model_param_count.restype = ctypes.c_int64
    L.fsm_model_create.argtypes = [ctypes.c_int32, f32p, ctypes.c_uint64, ctypes.POINTER(vp)]
    L.fsm_model_create.restype = ctypes.c_int
    L.fsm_model_in_dim.argtypes = [vp]
    L.fsm_model_in_dim.restype = ctypes.c_int32
    L.fsm_model_params.argtypes = [vp, f32p]
    L.fsm_model_params.restype = ctypes.c_int
    L.fsm_model_gradient.argtypes = [vp, f32p, f32p, ctypes.c_int64, f32p,
                                     ctypes.POINTER(ctypes.c_double)]
    L.fsm_model_gradient.restype = ctypes.c_int
    L.fsm_model_train.argtypes = [vp, f32p, f32p, ctypes.c_int64, ctypes.c_int32, ctypes.c_float,
                                  ctypes.POINTER(ctypes.c_double)]
    L.fsm_model_train.restype = ctypes.c_int
    L.fsm_model_predict.argtypes = [vp, f32p, ctypes.c_int64, f32p]
    L.fsm_model_predict.restype = ctypes.c_int
    L.fsm_model_free.argtypes = [vp]
    L.fsm_model_free.restype = None
    _lib = L
    return L


def _check(rc):
    if rc != 0:
        msg = lib().fsm_last_error()
        raise FsmError(rc, msg.decode() if msg else "")


def _i32(a):
    a = np.ascontiguousarray(a, dtype=np.int32)
    return a, a.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))


_torch_hooks = None


def use_torch_allocator(enable: bool = True):
    """Route the library's device allocations through PyTorch's caching
    allocator (on the current device and stream), or back to hipMalloc."""
    global _torch_hooks
    L = lib()
    if not enable:
        _check(L.fsm_set_allocator(_ALLOC_FN(), _RELEASE_FN(), None))
        _torch_hooks = None
        return
    import torch

    def _alloc(nbytes, _ctx):
        try:
            return torch.cuda.caching_allocator_alloc(int(nbytes))
        except Exception:   # out of memory -> NULL, reported as FSM_ENOMEM
            return None

    def _release(ptr, _ctx):
        torch.cuda.caching_allocator_delete(ptr)

    hooks = (_ALLOC_FN(_alloc), _RELEASE_FN(_release))
    _check(L.fsm_set_allocator(hooks[0], hooks[1], None))
    _torch_hooks = hooks


def set_stream(stream=None):
    """Use a torch.cuda.Stream (or a raw hipStream_t int; None = null stream)."""
    if stream is None:
        ptr = None
    elif isinstance(stream, int):
        ptr = stream
    else:
        ptr = stream.cuda_stream
    _check(lib().fsm_set_stream(ptr))


class Graph:
    """Device-resident CSR of a labelled undirected graph (fsm_build_graph)."""

    def __init__(self, n_vertices, src, dst, labels):
        L = lib()
        s, sp = _i32(src)
        d, dp = _i32(dst)
        lab, lp = _i32(labels)
        if s.shape != d.shape:
            raise ValueError("src and dst differ in length")
        if lab.size != n_vertices:
            raise ValueError("labels must have n_vertices entries")
        h = ctypes.c_void_p()
        _check(L.fsm_build_graph(int(n_vertices), int(s.size), sp, dp, lp, ctypes.byref(h)))
        self._h = h

    @property
    def handle(self):
        return self._h

    @property
    def n_vertices(self):
        return int(lib().fsm_graph_vertices(self._h))

    @property
    def n_edges(self):
        return int(lib().fsm_graph_edges(self._h))

    def close(self):
        if self._h:
            lib().fsm_graph_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


class Result:
    """Host copy of one mining result.  ``sizes``, ``codes`` (rows of the
    36-byte fsm_code: n, label[7], adj) and ``supports`` are numpy arrays;
    ``patterns`` is the list of ``(size, labels, adj, support)`` built from
    them on first use; ``stats`` holds the call's counters."""

    def __init__(self, handle):
        L = lib()
        try:
            cnt = L.fsm_result_count(handle)
            self.sizes = np.zeros(max(cnt, 1), np.int32)
            self.supports = np.zeros(max(cnt, 1), np.int64)
            self.codes = np.zeros((max(cnt, 1), 2 + MAX_SIZE), np.int32)
            _check(L.fsm_result_patterns(
                handle, None, self.sizes.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                self.codes.ctypes.data_as(ctypes.POINTER(Code)),
                self.supports.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))))
            self.sizes, self.supports, self.codes = self.sizes[:cnt], self.supports[:cnt], self.codes[:cnt]
            st = Stats()
            _check(L.fsm_result_stats(handle, ctypes.byref(st)))
            nrow = L.fsm_result_training_count(handle)
            self.train_x = np.zeros((nrow, FEATURES), np.float32)
            self.train_t = np.zeros((nrow, 2), np.float32)
            self.train_level = np.zeros(nrow, np.int32)
            if nrow > 0:
                _check(L.fsm_result_training_rows(
                    handle, self.train_x.ctypes.data_as(ctypes.POINTER(ctypes.c_float)),
                    self.train_t.ctypes.data_as(ctypes.POINTER(ctypes.c_float)),
                    self.train_level.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))))
        finally:
            L.fsm_result_free(handle)
        self.stats = _stats_dict(st)
        self._patterns = None

    def __len__(self):
        return len(self.sizes)

    @property
    def patterns(self):
        if self._patterns is None:
            adj = self.codes.view(np.uint32)[:, 1 + MAX_SIZE].tolist()
            labs = self.codes[:, 1:1 + MAX_SIZE].tolist()
            self._patterns = [(n, tuple(lab[:n]), a, s) for n, lab, a, s in
                              zip(self.sizes.tolist(), labs, adj, self.supports.tolist())]
        return self._patterns


def _stats_dict(st):
    levels = {}
    for n in range(2, st.max_size + 1):
        lv = st.level[n]
        levels[n] = {f: getattr(lv, f) for f, _ in LevelStats._fields_}
    return {"max_size": st.max_size, "frequent_labels": st.frequent_labels,
            "dropped_self_loops": st.dropped_self_loops,
            "dropped_duplicates": st.dropped_duplicates,
            "filtered_edges": st.filtered_edges, "levels": levels,
            "total_ms": st.total_ms, "batch_chunk": st.batch_chunk,
            "batch_chunks": st.batch_chunks, "batch_splits": st.batch_splits,
            "captured_levels": st.captured_levels, "captured_graphs": st.captured_graphs,
            "level_fallbacks": st.level_fallbacks, "host_syncs": st.host_syncs}


def mine(graph: Graph, support: int, max_size: int, mode: int = FSM_PLAIN, *,
         sampling_rate: float = 1.0, seed: int = 0, disable_pruning: bool = False,
         hash_capacity_min: int = 0, pattern_capacity_min: int = 0, model=None,
         record: bool = False, schedule: int = FSM_SCHEDULE_QUEUE,
         tiles_per_wave: int = 0, pool_budget_mib: int = 0, join_threshold: int = 0,
         match_threshold: int = 0, force_overflow: bool = False) -> Result:
    """Frequent patterns of sizes 2..max_size with MNI support >= support.
    ``model`` (a Model with FEATURES inputs) sizes the join tables when
    ``mode`` has FSM_LEARNED; ``record`` keeps the join work-item rows.
    ``join_threshold`` x samples x^2 size-3 subgraphs per key group at every
    join (and x edges at the size-4 join), ``match_threshold`` t keeps t
    size-3 subgraphs per vertex in matching (Section 5, seeded by ``seed``)."""
    o = Options()
    o.join_threshold = int(join_threshold)
    o.match_threshold = int(match_threshold)
    o.force_overflow = 1 if force_overflow else 0
    o.model = model.handle.value if model is not None else None
    o.record = 1 if record else 0
    o.schedule = int(schedule)
    o.tiles_per_wave = int(tiles_per_wave)
    o.pool_budget_mib = int(pool_budget_mib)
    o.support = int(support)
    o.max_size = int(max_size)
    o.mode = int(mode)
    o.disable_pruning = 1 if disable_pruning else 0
    o.sampling_rate = float(sampling_rate)
    o.seed = int(seed) & ((1 << 64) - 1)
    o.hash_capacity_min = int(hash_capacity_min)
    o.pattern_capacity_min = int(pattern_capacity_min)
    h = ctypes.c_void_p()
    _check(lib().fsm_mine_ex(graph.handle, ctypes.byref(o), ctypes.byref(h)))
    return Result(h)


NOALLOC_SCRATCH_MIB = 256


def mine_noalloc(graph: Graph, support: int, max_size: int, mode: int = FSM_PLAIN, *,
                 capacity: int = 1 << 16, sampling_rate: float = 1.0, seed: int = 0,
                 join_threshold: int = 0, match_threshold: int = 0, model=None):
    """fsm_mine_noalloc: the same mining call with no device allocation
    (buffers come from the library's fixed scratch array).  Returns
    ``(patterns, stats)`` with patterns as ``Result.patterns``."""
    o = Options()
    o.support = int(support)
    o.max_size = int(max_size)
    o.mode = int(mode)
    o.sampling_rate = float(sampling_rate)
    o.seed = int(seed) & ((1 << 64) - 1)
    o.join_threshold = int(join_threshold)
    o.match_threshold = int(match_threshold)
    o.model = model.handle.value if model is not None else None
    cap = int(capacity)
    sizes = np.zeros(max(cap, 1), np.int32)
    codes = np.zeros((max(cap, 1), 2 + MAX_SIZE), np.int32)
    sups = np.zeros(max(cap, 1), np.int64)
    cnt = ctypes.c_int64()
    st = Stats()
    _check(lib().fsm_mine_noalloc(
        graph.handle, ctypes.byref(o), cap, sizes.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
        codes.ctypes.data_as(ctypes.POINTER(Code)),
        sups.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), ctypes.byref(cnt), ctypes.byref(st)))
    n = cnt.value
    adj = codes.view(np.uint32)[:n, 1 + MAX_SIZE].tolist()
    labs = codes[:n, 1:1 + MAX_SIZE].tolist()
    pats = [(k, tuple(lab[:k]), a, s) for k, lab, a, s in
            zip(sizes[:n].tolist(), labs, adj, sups[:n].tolist())]
    return pats, _stats_dict(st)


def mine_batch(graphs, supports, max_size: int, mode: int = FSM_BATCHED, *,
               chunk_vertices: int = 0, disable_pruning: bool = False,
               hash_capacity_min: int = 0, pattern_capacity_min: int = 0, model=None,
               learn: bool = False, train_steps: int = 0, lr: float = 0.0,
               tiles_per_wave: int = 0, pool_budget_mib: int = 0, eager_levels: bool = False):
    """Mine several graphs in union passes of at most ``chunk_vertices``
    vertices (0: the library default); one Result per graph.  With a
    ``model``, FSM_LEARNED in ``mode`` sizes every chunk's join tables from
    it, and ``learn`` trains it on each chunk's work items."""
    n = len(graphs)
    if len(supports) != n:
        raise ValueError("one support per graph")
    hs = (ctypes.c_void_p * n)(*[g.handle for g in graphs])
    sup = np.ascontiguousarray(supports, dtype=np.int64)
    outs = (ctypes.c_void_p * n)()
    o = BatchOptions()
    o.max_size = int(max_size)
    o.mode = int(mode)
    o.chunk_vertices = int(chunk_vertices)
    o.tiles_per_wave = int(tiles_per_wave)
    o.pool_budget_mib = int(pool_budget_mib)
    o.disable_pruning = 1 if disable_pruning else 0
    o.hash_capacity_min = int(hash_capacity_min)
    o.pattern_capacity_min = int(pattern_capacity_min)
    o.model = model.handle.value if model is not None else None
    o.learn = 1 if learn else 0
    o.eager_levels = 1 if eager_levels else 0
    o.train_steps = int(train_steps)
    o.lr = float(lr)
    _check(lib().fsm_mine_batch_ex(hs, n, sup.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                                   ctypes.byref(o), outs))
    return [Result(ctypes.c_void_p(outs[i])) for i in range(n)]


def tune_batch(graphs, supports, max_size: int):
    """Time the candidate batch shapes on these graphs and keep the fastest
    as the library's defaults; returns (winner, [(chunk, tiles, ms), ...])."""
    n = len(graphs)
    hs = (ctypes.c_void_p * n)(*[g.handle for g in graphs])
    sup = np.ascontiguousarray(supports, dtype=np.int64)
    t = Tuning()
    _check(lib().fsm_tune_batch(hs, n, sup.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                                int(max_size), ctypes.byref(t)))
    cands = [(int(t.cand_chunk[i]), int(t.cand_tiles[i]), float(t.cand_ms[i]))
             for i in range(t.configs)]
    return {"chunk_vertices": int(t.chunk_vertices), "tiles_per_wave": int(t.tiles_per_wave)}, cands


def reset_tuning():
    _check(lib().fsm_reset_tuning())


def _f32(a, cols=None):
    a = np.ascontiguousarray(a, dtype=np.float32)
    if cols is not None and (a.ndim != 2 or a.shape[1] != cols):
        raise ValueError(f"expected a (rows, {cols}) array")
    return a, a.ctypes.data_as(ctypes.POINTER(ctypes.c_float))


class Model:
    """Join cost model on the device (two-layer perceptron, bfloat16
    weights, float32 accumulation); see ``fsm_model_*`` in include/fsm.h."""

    HIDDEN = 64
    OUT = 2

    def __init__(self, in_dim: int, params=None, seed: int = 0):
        L = lib()
        self.in_dim = int(in_dim)
        self.count = int(L.fsm_model_param_count(self.in_dim))
        pp = None
        if params is not None:
            self._init, pp = _f32(params)
            if self._init.size != self.count:
                raise ValueError(f"expected {self.count} parameters")
        h = ctypes.c_void_p()
        _check(L.fsm_model_create(self.in_dim, pp, int(seed) & ((1 << 64) - 1), ctypes.byref(h)))
        self.handle = h

    def params(self):
        out = np.empty(self.count, np.float32)
        _check(lib().fsm_model_params(self.handle, out.ctypes.data_as(ctypes.POINTER(ctypes.c_float))))
        return out

    def gradient(self, x, t):
        x, xp = _f32(x, self.in_dim)
        t, tp = _f32(t, self.OUT)
        g = np.empty(self.count, np.float32)
        loss = ctypes.c_double()
        _check(lib().fsm_model_gradient(self.handle, xp, tp, len(x),
                                        g.ctypes.data_as(ctypes.POINTER(ctypes.c_float)),
                                        ctypes.byref(loss)))
        return g, loss.value

    def train(self, x, t, steps: int, lr: float) -> float:
        x, xp = _f32(x, self.in_dim)
        t, tp = _f32(t, self.OUT)
        loss = ctypes.c_double()
        _check(lib().fsm_model_train(self.handle, xp, tp, len(x), int(steps), float(lr),
                                     ctypes.byref(loss)))
        return loss.value

    def predict(self, x):
        x, xp = _f32(x, self.in_dim)
        y = np.empty((len(x), self.OUT), np.float32)
        _check(lib().fsm_model_predict(self.handle, xp, len(x),
                                       y.ctypes.data_as(ctypes.POINTER(ctypes.c_float))))
        return y

    def close(self):
        if getattr(self, "handle", None):
            lib().fsm_model_free(self.handle)
            self.handle = None

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def score_sampled(exact, sampled):
    """Score a sampled mining result against the exact one (lists of
    ``(size, labels, adj, support)``).  Sampled embeddings are a subset of
    the exact ones, so every sampled support is a lower bound of the exact
    support and every reported pattern is truly frequent; the score states
    how much of the exact answer the sample recovers:

    ``recall``          found / exact frequent patterns
    ``precision``       reported patterns that are exactly frequent
    ``support_ratio``   mean of estimated / exact support over found patterns
    ``lower_bound``     True when no estimate exceeds its exact support
    ``by_size``         recall per pattern size
    """
    ex = {(p[0], tuple(p[1]), p[2]): p[3] for p in exact}
    sm = {(p[0], tuple(p[1]), p[2]): p[3] for p in sampled}
    found = [k for k in sm if k in ex]
    ratios = [sm[k] / ex[k] for k in found]
    sizes = sorted({k[0] for k in ex})
    by_size = {}
    for n in sizes:
        tot = sum(1 for k in ex if k[0] == n)
        by_size[n] = sum(1 for k in found if k[0] == n) / tot if tot else 1.0
    return {"exact": len(ex), "reported": len(sm), "found": len(found),
            "recall": len(found) / len(ex) if ex else 1.0,
            "precision": len(found) / len(sm) if sm else 1.0,
            "support_ratio": float(np.mean(ratios)) if ratios else 0.0,
            "lower_bound": all(sm[k] <= ex[k] for k in found),
            "by_size": by_size}


def dissect(ids, adj):
    """Host instance of the join's dissection rule: (l_mask, shared position)."""
    n = len(ids)
    a, ap = _i32(ids)
    lm = ctypes.c_uint32()
    sh = ctypes.c_int32()
    _check(lib().fsm_dissect(n, ap, ctypes.c_uint32(adj), ctypes.byref(lm), ctypes.byref(sh)))
    return int(lm.value), int(sh.value)


def proposal_thresholds(pred, rate: float):
    """Keep thresholds of the learned sampling proposal for per-item
    predictions ``pred`` (log1p of predicted children), as the miner
    computes them (fsm_proposal_thresholds)."""
    p = np.ascontiguousarray(pred, dtype=np.float32).ravel()
    out = np.zeros(max(p.size, 1), np.uint64)
    _check(lib().fsm_proposal_thresholds(
        p.ctypes.data_as(ctypes.POINTER(ctypes.c_float)), p.size, float(rate),
        out.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64))))
    return out[:p.size]


def key_graph(key: int, size: int, graphs: int) -> int:
    """Graph id a batched pattern key carries, checked (fsm_key_graph)."""
    g = ctypes.c_int32()
    _check(lib().fsm_key_graph(ctypes.c_uint64(key), int(size), int(graphs), ctypes.byref(g)))
    return int(g.value)
