"""ctypes binding of libgapbfs.so (include/gapbfs.h).

Argument marshalling only: every step of the search runs in the library's
HIP kernels.  Device buffers are torch tensors (int32, on the graph's
device); streams are torch streams (their ``cuda_stream`` handle).  If the
library is not built, every call raises: there is no CPU fallback.
"""
from __future__ import annotations

import atexit
import ctypes
import os
import threading
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libgapbfs.so")
_lib = None
_lock = threading.Lock()

GAP_OK, GAP_EINVAL, GAP_ENOMEM, GAP_EDEVICE, GAP_EBUSY, GAP_EINTERNAL, GAP_ETIMEOUT = 0, -1, -2, -3, -4, -5, -6
MODE_PERSISTENT, MODE_LEVELS, MODE_GRAPH = 0, 1, 2
DIR_AUTO, DIR_TOPDOWN, DIR_BOTTOMUP = 0, 1, 2


class GapError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"gapbfs status {status}: {msg}")
        self.status = status


class _Params(ctypes.Structure):
    _fields_ = [("mode", ctypes.c_int32), ("direction", ctypes.c_int32),
                ("alpha", ctypes.c_int32), ("beta", ctypes.c_int32),
                ("block", ctypes.c_int32), ("blocks_per_cu", ctypes.c_int32),
                ("hub_degree", ctypes.c_int32), ("chunk_edges", ctypes.c_int32),
                ("graph_chunk", ctypes.c_int32), ("batch_mode", ctypes.c_int32),
                ("batch_alpha", ctypes.c_int32), ("batch_beta", ctypes.c_int32),
                ("grid_split", ctypes.c_int32), ("small_frontier", ctypes.c_int32),
                ("lds_bitmap", ctypes.c_int32), ("wait_limit_us", ctypes.c_int32),
                ("bu_mapping", ctypes.c_int32), ("batch_words", ctypes.c_int32),
                ("serve_window_us", ctypes.c_int32), ("td_plain", ctypes.c_int32),
                ("coop_launch", ctypes.c_int32)]


PARAM_NAMES = [f[0] for f in _Params._fields_]


class LevelStat(ctypes.Structure):
    _fields_ = [("level", ctypes.c_int32), ("direction", ctypes.c_int32),
                ("frontier", ctypes.c_int64), ("frontier_edges", ctypes.c_int64),
                ("claimed", ctypes.c_int64), ("scanned", ctypes.c_int64),
                ("unvisited", ctypes.c_int64), ("time_ns", ctypes.c_int64)]


class DeviceInfo(ctypes.Structure):
    _fields_ = [("device", ctypes.c_int32), ("compute_units", ctypes.c_int32),
                ("lds_per_cu", ctypes.c_int32), ("l2_bytes", ctypes.c_int32),
                ("wave_size", ctypes.c_int32), ("clock_khz", ctypes.c_int32),
                ("total_mem", ctypes.c_int64), ("arch", ctypes.c_char * 64)]


EXPORTED = ["gap_build_csr", "gap_graph_info", "gap_graph_directed", "gap_graph_export",
            "gap_graph_export_in", "gap_bfs", "gap_bfs_batch",
            "gap_free", "gap_last_error", "gap_set_params", "gap_get_params", "gap_bfs_ex",
            "gap_device_query", "gap_stream_copy", "gap_bc", "gap_build_csr_weighted",
            "gap_graph_export_weights", "gap_sssp", "gap_sssp_ex", "gap_cc", "gap_stream_status",
            "gap_shutdown", "gap_bfs_noalloc", "gap_bfs_batch_ex", "gap_serve_open", "gap_serve_submit",
            "gap_serve_poll", "gap_serve_close"]


def library_path() -> str:
    return _LIB_PATH


def load():
    """Load libgapbfs.so; raises if it has not been built."""
    global _lib
    with _lock:
        if _lib is not None:
            return _lib
        if not os.path.exists(_LIB_PATH):
            raise ImportError(f"{_LIB_PATH} is not built (run __graft_entry__.build() or "
                              "python -m paper_1508_03619_amd.build)")
        # torch ships its own HIP runtime.  Loading torch first makes this
        # library bind to that same runtime; loading the library first puts a
        # second runtime in the process and one of the two then finds no device.
        import torch  # noqa: F401
        L = ctypes.CDLL(_LIB_PATH)
        vp, i32, i64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
        i32p = ctypes.POINTER(ctypes.c_int32)
        i64p = ctypes.POINTER(ctypes.c_int64)
        L.gap_build_csr.argtypes = [i64, i64, i32p, i32p, ctypes.c_uint32, vp, ctypes.POINTER(vp)]
        L.gap_graph_info.argtypes = [vp, i64p, i64p]
        L.gap_graph_export.argtypes = [vp, i64p, i32p]
        L.gap_graph_export_in.argtypes = [vp, i64p, i32p]
        L.gap_graph_directed.argtypes = [vp]
        L.gap_bfs.argtypes = [vp, i32, vp, vp, vp]
        L.gap_bfs_noalloc.argtypes = [vp, i32, vp, vp, vp]
        L.gap_serve_open.argtypes = [i64, i64, vp, ctypes.POINTER(vp)]
        L.gap_serve_submit.argtypes = [vp, vp, i64, i32, vp, vp]
        L.gap_serve_poll.argtypes = [vp, i64p, i32, i32p]
        L.gap_serve_close.argtypes = [vp]
        L.gap_bfs_ex.argtypes = [vp, i32, vp, vp, vp, ctypes.POINTER(_Params),
                                 ctypes.POINTER(LevelStat), i32, i32p]
        L.gap_bfs_batch.argtypes = [ctypes.POINTER(vp), i32, i32p, i32p, i32,
                                    ctypes.POINTER(vp), ctypes.POINTER(vp), vp]
        L.gap_bfs_batch_ex.argtypes = [ctypes.POINTER(vp), i32, i32p, i32p, i32,
                                       ctypes.POINTER(vp), ctypes.POINTER(vp), vp,
                                       ctypes.POINTER(LevelStat), i32, i32p]
        L.gap_free.argtypes = [vp]
        L.gap_free.restype = None
        L.gap_last_error.argtypes = []
        L.gap_last_error.restype = ctypes.c_char_p
        L.gap_set_params.argtypes = [ctypes.POINTER(_Params)]
        L.gap_get_params.argtypes = [ctypes.POINTER(_Params)]
        L.gap_device_query.argtypes = [ctypes.POINTER(DeviceInfo)]
        L.gap_stream_copy.argtypes = [vp, vp, i64, vp]
        L.gap_bc.argtypes = [vp, i32p, i32, vp, ctypes.c_uint32, vp]
        L.gap_build_csr_weighted.argtypes = [i64, i64, i32p, i32p, i32p, ctypes.c_uint32, vp,
                                             ctypes.POINTER(vp)]
        L.gap_graph_export_weights.argtypes = [vp, i32p]
        L.gap_sssp.argtypes = [vp, i32, vp, ctypes.c_uint32, vp]
        L.gap_sssp_ex.argtypes = [vp, i32, vp, ctypes.c_uint32, vp, i32p]
        L.gap_cc.argtypes = [vp, vp, vp]
        L.gap_stream_status.argtypes = [vp]
        L.gap_shutdown.argtypes = []
        L.gap_shutdown.restype = None
        for name in ("gap_build_csr", "gap_graph_info", "gap_graph_export", "gap_graph_export_in",
                     "gap_graph_directed", "gap_bfs", "gap_bfs_ex", "gap_bfs_noalloc", "gap_bfs_batch_ex",
                     "gap_bfs_batch", "gap_set_params", "gap_get_params", "gap_device_query",
                     "gap_stream_copy", "gap_bc", "gap_build_csr_weighted",
                     "gap_graph_export_weights", "gap_sssp", "gap_sssp_ex", "gap_cc",
                     "gap_stream_status", "gap_serve_open", "gap_serve_submit", "gap_serve_poll",
                     "gap_serve_close"):
            getattr(L, name).restype = ctypes.c_int32
        _lib = L
        # release the library's scratch, events and captured graphs before
        # the HIP runtime and any attached profiler tear down
        atexit.register(L.gap_shutdown)
        _apply_tuned(L)
        return L


_defaults: dict = {}
_tuned: Optional[tuple] = None


def _apply_tuned(L):
    """Remember the library's built-in parameters, then apply the tuned set
    for this GPU model if one exists (``tuned/<arch>_<CUs>cu.json``, written
    by ``autotune``).  GAPBFS_TUNED=0 keeps the built-in set."""
    global _tuned
    p = _Params()
    if L.gap_get_params(ctypes.byref(p)) != GAP_OK:
        raise GapError(GAP_EINTERNAL, "gap_get_params failed")
    _defaults.update({k: int(getattr(p, k)) for k in PARAM_NAMES})
    if os.environ.get("GAPBFS_TUNED", "1") == "0":
        return
    import torch
    if not torch.cuda.is_available():
        return
    info = DeviceInfo()
    if L.gap_device_query(ctypes.byref(info)) != GAP_OK:
        return  # no device visible: nothing to tune for
    from .autotune import read_tuned, tuned_path
    path = tuned_path(info.arch.decode(), info.compute_units)
    if not os.path.exists(path):
        return
    tuned = read_tuned(path)
    for k, v in tuned.items():
        if k not in PARAM_NAMES:
            raise KeyError(f"{path}: unknown parameter {k}")
        setattr(p, k, int(v))
    if L.gap_set_params(ctypes.byref(p)) != GAP_OK:
        raise GapError(GAP_EINVAL, f"{path}: {L.gap_last_error().decode()}")
    _tuned = (path, dict(tuned))


def library_defaults() -> dict:
    """The library's built-in parameter set (before any tuned file)."""
    load()
    return dict(_defaults)


def tuned_params() -> Optional[tuple]:
    """(path, params) of the tuned file applied at load, or None."""
    load()
    return _tuned


def _check(status: int):
    if status != GAP_OK:
        msg = load().gap_last_error()
        raise GapError(status, msg.decode() if msg else "")


def _stream_handle(stream) -> Optional[int]:
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


def _i32p(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))


BUILD_DIRECTED = 1  # gap_build_csr flag


class Graph:
    """A CSR graph resident in device memory (owns its gap_graph handle)."""

    def __init__(self, handle: int, n: int, nnz: int, directed: bool = False,
                 weighted: bool = False):
        self.handle = ctypes.c_void_p(handle)
        self.n = n
        self.nnz = nnz
        self.directed = directed
        self.weighted = weighted

    def free(self):
        if self.handle and self.handle.value:
            load().gap_free(self.handle)
            self.handle = ctypes.c_void_p(None)

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass

    def _export(self, fn, with_col=True):
        row_ptr = np.empty(self.n + 1, np.int64)
        col = np.empty(max(self.nnz, 1), np.int32) if with_col else None
        _check(fn(self.handle, row_ptr.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                  _i32p(col) if with_col else None))
        return row_ptr, (col[:self.nnz] if with_col else None)

    def export(self):
        """(row_ptr int64[n+1], col int32[nnz]) copied to the host: the
        out-lists of a directed graph."""
        return self._export(load().gap_graph_export)

    def export_in(self):
        """The in-lists (the transpose), as ``export``."""
        return self._export(load().gap_graph_export_in)

    def export_weights(self) -> np.ndarray:
        """Out-list weights (int32[nnz]) in ``export`` order."""
        w = np.empty(max(self.nnz, 1), np.int32)
        _check(load().gap_graph_export_weights(self.handle, _i32p(w)))
        return w[:self.nnz]

    def degrees(self) -> np.ndarray:
        rp, _ = self.export_row_ptr()
        return np.diff(rp)

    def export_row_ptr(self):
        return self._export(load().gap_graph_export, with_col=False)


def build_csr(n: int, src: np.ndarray, dst: np.ndarray, stream=None, directed: bool = False,
              weights: Optional[np.ndarray] = None) -> Graph:
    """Build the device CSR from raw pairs (copied).  ``directed`` keeps
    src[i] -> dst[i] as a one-way edge; otherwise every pair is undirected.
    ``weights`` (int32 per pair, >= 1) are kept for shortest paths."""
    L = load()
    src = np.ascontiguousarray(src, dtype=np.int32)
    dst = np.ascontiguousarray(dst, dtype=np.int32)
    out = ctypes.c_void_p()
    flags = BUILD_DIRECTED if directed else 0
    if weights is None:
        _check(L.gap_build_csr(int(n), int(src.shape[0]), _i32p(src), _i32p(dst), flags,
                               _stream_handle(stream), ctypes.byref(out)))
    else:
        w = np.ascontiguousarray(weights, dtype=np.int32)
        if w.shape[0] != src.shape[0]:
            raise ValueError("one weight per pair")
        _check(L.gap_build_csr_weighted(int(n), int(src.shape[0]), _i32p(src), _i32p(dst), _i32p(w),
                                        flags, _stream_handle(stream), ctypes.byref(out)))
    nn, nnz = ctypes.c_int64(), ctypes.c_int64()
    _check(L.gap_graph_info(out, ctypes.byref(nn), ctypes.byref(nnz)))
    dflag = L.gap_graph_directed(out)
    if dflag < 0:
        _check(dflag)
    return Graph(out.value, nn.value, nnz.value, directed=bool(dflag), weighted=weights is not None)


def graph_info(g: Graph):
    return g.n, g.nnz


def free(g: Graph):
    g.free()


def _params_struct(d: dict) -> _Params:
    p = _Params()
    _check(load().gap_get_params(ctypes.byref(p)))
    for k, v in d.items():
        if k not in PARAM_NAMES:
            raise KeyError(k)
        setattr(p, k, int(v))
    return p


def get_params() -> dict:
    p = _Params()
    _check(load().gap_get_params(ctypes.byref(p)))
    return {k: int(getattr(p, k)) for k in PARAM_NAMES}


def set_params(**kw):
    p = _params_struct(kw)
    _check(load().gap_set_params(ctypes.byref(p)))


_last_stats: list = []


def last_stats() -> list:
    return list(_last_stats)


def _ptr(t) -> Optional[int]:
    if t is None:
        return None
    import torch
    if t.dtype != torch.int32 or not t.is_cuda or not t.is_contiguous():
        raise ValueError("output buffers must be contiguous int32 device tensors")
    return t.data_ptr()


def bfs(g: Graph, source: int, parent, depth=None, stream=None, params: Optional[dict] = None,
        stats: bool = False, max_levels: int = 1 << 16):
    """One search.  parent/depth: int32 device tensors of length n (depth may be None).
    With stats=True the call waits for the search and returns per-level records."""
    L = load()
    if parent.numel() < g.n or (depth is not None and depth.numel() < g.n):
        raise ValueError("output buffers shorter than n")
    if params is None and not stats:
        _check(L.gap_bfs(g.handle, int(source), _ptr(parent), _ptr(depth), _stream_handle(stream)))
        return None
    pp = ctypes.byref(_params_struct(params)) if params is not None else None
    if stats:
        recs = (LevelStat * max_levels)()
        nl = ctypes.c_int32(0)
        _check(L.gap_bfs_ex(g.handle, int(source), _ptr(parent), _ptr(depth), _stream_handle(stream),
                            pp, recs, int(max_levels), ctypes.byref(nl)))
        out = [{k: int(getattr(recs[i], k)) for k, _ in LevelStat._fields_}
               for i in range(min(nl.value, max_levels))]
        _last_stats[:] = out
        return out
    _check(L.gap_bfs_ex(g.handle, int(source), _ptr(parent), _ptr(depth), _stream_handle(stream),
                        pp, None, 0, None))
    return None


def bfs_noalloc(g: Graph, source: int, parent, depth=None, stream=None):
    """gap_bfs_noalloc: one search (persistent schedule) whose scratch is the
    library's per-device array; nothing is allocated.  Graphs whose scratch
    exceeds NOALLOC_SCRATCH_BYTES raise GapError (GAP_EINVAL)."""
    L = load()
    if parent.numel() < g.n or (depth is not None and depth.numel() < g.n):
        raise ValueError("output buffers shorter than n")
    _check(L.gap_bfs_noalloc(g.handle, int(source), _ptr(parent), _ptr(depth),
                             _stream_handle(stream)))


NOALLOC_SCRATCH_BYTES = 64 << 20  # GAP_NOALLOC_SCRATCH_BYTES

SERVE_RING = 256  # queries a server holds in flight at most


class Server:
    """gap_serve_*: continuous batching of single-source queries on one graph
    at a time.  ``submit`` returns False when the server cannot take the
    query now (GAP_EBUSY: its ring is full, or it still holds queries on
    another graph); ``poll`` returns the ids of completed queries, whose
    outputs are then final (read them on a stream other than the server's)."""

    def __init__(self, max_vertices: int, max_entries: int, stream=None):
        L = load()
        h = ctypes.c_void_p()
        _check(L.gap_serve_open(int(max_vertices), int(max_entries), _stream_handle(stream),
                                ctypes.byref(h)))
        self.handle = h
        self.max_vertices, self.max_entries = int(max_vertices), int(max_entries)
        self._buf = (ctypes.c_int64 * SERVE_RING)()

    def submit(self, g: Graph, qid: int, source: int, parent, depth=None) -> bool:
        if parent.numel() < g.n or (depth is not None and depth.numel() < g.n):
            raise ValueError("output buffers shorter than n")
        st = load().gap_serve_submit(self.handle, g.handle, int(qid), int(source), _ptr(parent),
                                     _ptr(depth))
        if st == GAP_EBUSY:
            return False
        _check(st)
        return True

    def poll(self) -> list:
        n = ctypes.c_int32(0)
        _check(load().gap_serve_poll(self.handle, self._buf, SERVE_RING, ctypes.byref(n)))
        return [int(self._buf[i]) for i in range(n.value)]

    def close(self):
        if self.handle:
            load().gap_serve_close(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def bfs_batch(graphs: Sequence[Graph], graph_of_source: Sequence[int], sources: Sequence[int],
              parents: Sequence, depths: Optional[Sequence] = None, stream=None,
              stats: bool = False, max_levels: int = 128):
    """Lane i searches graphs[graph_of_source[i]] from sources[i].  With
    stats=True the call waits for the batch and returns per-level records
    (gap_bfs_batch_ex)."""
    L = load()
    ng, ns = len(graphs), len(sources)
    gh = (ctypes.c_void_p * ng)(*[g.handle.value for g in graphs])
    gos = np.ascontiguousarray(graph_of_source, dtype=np.int32)
    src = np.ascontiguousarray(sources, dtype=np.int32)
    if len(gos) != ns or len(parents) != ns or (depths is not None and len(depths) != ns):
        raise ValueError("per-lane arrays must all have num_sources entries")
    for i in range(ns):
        n = graphs[int(gos[i])].n
        if parents[i].numel() < n or (depths is not None and depths[i] is not None and depths[i].numel() < n):
            raise ValueError(f"lane {i}: output buffer shorter than n")
    pa = (ctypes.c_void_p * ns)(*[_ptr(t) for t in parents])
    da = None
    if depths is not None:
        da = (ctypes.c_void_p * ns)(*[_ptr(t) for t in depths])
    if stats:
        recs = (LevelStat * max_levels)()
        nl = ctypes.c_int32(0)
        _check(L.gap_bfs_batch_ex(gh, ng, _i32p(gos), _i32p(src), ns, pa, da, _stream_handle(stream),
                                  recs, int(max_levels), ctypes.byref(nl)))
        return [{k: int(getattr(recs[i], k)) for k, _ in LevelStat._fields_}
                for i in range(min(nl.value, max_levels))]
    _check(L.gap_bfs_batch(gh, ng, _i32p(gos), _i32p(src), ns, pa, da, _stream_handle(stream)))
    return None


BC_RAW = 1  # gap_bc flag


def bc(g: Graph, sources: Sequence[int], scores, normalise: bool = True, stream=None):
    """Betweenness centrality from ``sources`` into ``scores`` (a contiguous
    float64 device tensor of at least n entries), divided by the largest
    score unless ``normalise`` is False."""
    import torch
    L = load()
    src = np.ascontiguousarray(sources, dtype=np.int32)
    if scores.dtype != torch.float64 or not scores.is_cuda or not scores.is_contiguous():
        raise ValueError("scores must be a contiguous float64 device tensor")
    if scores.numel() < g.n:
        raise ValueError("scores shorter than n")
    _check(L.gap_bc(g.handle, _i32p(src), int(src.shape[0]), scores.data_ptr(),
                    0 if normalise else BC_RAW, _stream_handle(stream)))


SSSP_UNREACHABLE = 0xFFFFFFFF


def sssp(g: Graph, source: int, dist, delta: int = 0, stream=None, stats: bool = False):
    """Shortest-path distances from ``source`` into ``dist`` (a contiguous
    4-byte-element device tensor of at least n entries, read back as
    uint32; 0xFFFFFFFF marks unreachable vertices).  With ``stats`` the call
    waits and returns the number of relaxation phases."""
    import torch
    L = load()
    if dist.element_size() != 4 or not dist.is_cuda or not dist.is_contiguous():
        raise ValueError("dist must be a contiguous 4-byte device tensor")
    if dist.numel() < g.n:
        raise ValueError("dist shorter than n")
    if stats:
        ph = ctypes.c_int32(0)
        _check(L.gap_sssp_ex(g.handle, int(source), dist.data_ptr(), int(delta) & 0xFFFFFFFF,
                             _stream_handle(stream), ctypes.byref(ph)))
        return int(ph.value)
    _check(L.gap_sssp(g.handle, int(source), dist.data_ptr(), int(delta) & 0xFFFFFFFF,
                      _stream_handle(stream)))
    return None


def cc(g: Graph, labels, stream=None):
    """Connected-component labels (the smallest vertex of each component)
    into ``labels``, a contiguous int32 device tensor of at least n entries."""
    L = load()
    if labels.numel() < g.n:
        raise ValueError("labels shorter than n")
    _check(L.gap_cc(g.handle, _ptr(labels), _stream_handle(stream)))


def stream_status(stream=None):
    """Wait for ``stream`` and raise GapError if a search queued on it failed
    on the device since the last check (gap_stream_status)."""
    _check(load().gap_stream_status(_stream_handle(stream)))


def shutdown():
    """Release the library's per-stream scratch, events and captured graphs
    (gap_shutdown); later calls allocate them again."""
    load().gap_shutdown()


def device_query() -> dict:
    info = DeviceInfo()
    _check(load().gap_device_query(ctypes.byref(info)))
    d = {k: getattr(info, k) for k, _ in DeviceInfo._fields_}
    d["arch"] = info.arch.decode()
    return d


def stream_copy(dst, src, nbytes: int, stream=None):
    _check(load().gap_stream_copy(dst.data_ptr(), src.data_ptr(), int(nbytes), _stream_handle(stream)))
