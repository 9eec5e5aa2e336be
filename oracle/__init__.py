"""CPU oracle for breadth-first search and betweenness centrality -- TEST
INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the benchmark's
``cpu_baseline`` leg may import this package.  The GPU library never calls it,
and it shares no code with the GPU path: it takes the raw generated edge list
and builds its own adjacency.

Definitions followed (the paper, arXiv 1508.03619):
  * BFS output (Section 2.1): parent[source] = source; parent[v] = -1 when v
    is unreachable; otherwise an edge joins parent[v] to v and
    depth[v] = depth[parent[v]] + 1.  Depth is the hop distance, -1 when
    unreachable.
  * Graph clean-up (Section 2.3): duplicate edges and self-loops may be
    removed, neighbours may be reordered.  Kron and Urand are undirected, so
    the raw pairs are symmetrised.
  * Verification (Section 3, BFS verifier): a trivial serial BFS gives the
    reference depths; results are checked by properties, not by equality of
    parents, because several parent arrays are correct.
  * Betweenness centrality (Section 2.1): score[v] sums sigma_st(v)/sigma_st
    over the given sources s and all targets t, normalised so the largest
    score is one; Brandes' method without recorded successors (the paper's
    verifier for this kernel is also a serial Brandes, Section 3).
  * Shortest paths (Section 2.1): dist[source] = 0, unreachable vertices
    get the sentinel (-1 here), otherwise the least total weight of a path;
    Dijkstra's algorithm, the paper's verifier for this kernel (Section 3).
  * Connected components (Section 2.1): ``components`` labels every vertex
    with the smallest vertex of its (weak) component by union-find over the
    raw pairs; ``Adjacency.cc_check`` is the paper's verifier (Section 3)
    for any labelling.

The C implementation is ``oracle.c``; ``build()`` compiles it with gcc.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_libs: dict = {}

CHECK_NAMES = {
    0: "ok",
    1: "depth differs from the reference",
    2: "parent[source] != source",
    3: "reachability / negative-value mismatch",
    4: "parent is not a neighbour",
    5: "parent is not one level above",
    -1: "bad arguments",
}


def build(force: bool = False, out: str | None = None, defines: tuple = ()) -> str:
    """Compile the oracle (gcc, serial).  ``defines`` is for mutation tests."""
    target = out or _LIB
    if force or out or not os.path.exists(target) or os.path.getmtime(target) < os.path.getmtime(_SRC):
        tmp = target + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O2", "-fPIC", "-shared", "-std=c11", "-Wall", "-Wextra",
               *["-D" + d for d in defines], "-o", tmp, _SRC]
        subprocess.run(cmd, check=True)
        os.replace(tmp, target)
    return target


def _bind(path: str):
    lib = ctypes.CDLL(path)
    i32p = ctypes.POINTER(ctypes.c_int32)
    i64p = ctypes.POINTER(ctypes.c_int64)
    lib.oracle_build_adjacency.argtypes = [ctypes.c_int64, ctypes.c_int64, i32p, i32p, i64p, i32p]
    lib.oracle_build_adjacency.restype = ctypes.c_int64
    lib.oracle_build_out_adjacency.argtypes = [ctypes.c_int64, ctypes.c_int64, i32p, i32p, i64p, i32p]
    lib.oracle_build_out_adjacency.restype = ctypes.c_int64
    lib.oracle_bfs.argtypes = [ctypes.c_int64, i64p, i32p, ctypes.c_int32, i32p, i32p]
    lib.oracle_bfs.restype = ctypes.c_int64
    lib.oracle_check.argtypes = [ctypes.c_int64, i64p, i32p, ctypes.c_int32, i32p, i32p, i32p, i64p]
    lib.oracle_check.restype = ctypes.c_int
    lib.oracle_components.argtypes = [ctypes.c_int64, ctypes.c_int64, i32p, i32p, i32p]
    lib.oracle_components.restype = ctypes.c_int
    lib.oracle_bc.argtypes = [ctypes.c_int64, i64p, i32p, ctypes.c_int32, i32p, ctypes.c_int,
                              ctypes.POINTER(ctypes.c_double)]
    lib.oracle_bc.restype = ctypes.c_int
    lib.oracle_build_weighted_adjacency.argtypes = [ctypes.c_int64, ctypes.c_int64, i32p, i32p, i32p,
                                                    ctypes.c_int, i64p, i32p, i32p]
    lib.oracle_build_weighted_adjacency.restype = ctypes.c_int64
    lib.oracle_sssp.argtypes = [ctypes.c_int64, i64p, i32p, i32p, ctypes.c_int32, i64p]
    lib.oracle_sssp.restype = ctypes.c_int64
    lib.oracle_cc_check.argtypes = [ctypes.c_int64, i64p, i32p, i32p, i64p]
    lib.oracle_cc_check.restype = ctypes.c_int
    return lib


def lib(path: str | None = None):
    key = path or _LIB
    if key not in _libs:
        if path is None and not os.path.exists(_LIB):
            build()
        _libs[key] = _bind(key)
    return _libs[key]


def _i32(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))


def _i64(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))


class Adjacency:
    """Cleaned adjacency built by the oracle from raw pairs: symmetrised
    (undirected, the default) or out-lists only (``directed=True``)."""

    def __init__(self, n: int, src: np.ndarray, dst: np.ndarray, _lib=None, directed: bool = False):
        L = _lib or lib()
        src = np.ascontiguousarray(src, dtype=np.int32)
        dst = np.ascontiguousarray(dst, dtype=np.int32)
        m = int(src.shape[0])
        self.n = int(n)
        self.directed = bool(directed)
        self.offsets = np.zeros(self.n + 1, dtype=np.int64)
        adj = np.empty(max(2 * m, 1), dtype=np.int32)
        build = L.oracle_build_out_adjacency if self.directed else L.oracle_build_adjacency
        nnz = build(self.n, m, _i32(src), _i32(dst), _i64(self.offsets), _i32(adj))
        if nnz < 0:
            raise ValueError("oracle_build_adjacency: bad input")
        self.adj = adj[:nnz].copy()
        self._lib = L

    @property
    def nnz(self) -> int:
        return int(self.adj.shape[0])

    def degree(self) -> np.ndarray:
        return np.diff(self.offsets)

    def bfs(self, source: int):
        """(depth, parent) from a serial FIFO search."""
        depth = np.empty(self.n, dtype=np.int32)
        parent = np.empty(self.n, dtype=np.int32)
        r = self._lib.oracle_bfs(self.n, _i64(self.offsets), _i32(self.adj), int(source),
                                 _i32(depth), _i32(parent))
        if r < 0:
            raise ValueError("oracle_bfs: bad input")
        return depth, parent

    def check(self, source: int, depth_ref: np.ndarray, parent: np.ndarray,
              depth: np.ndarray | None = None):
        """(code, bad_vertex); code 0 means the result is a correct BFS."""
        bad = ctypes.c_int64(-1)
        parent = np.ascontiguousarray(parent, dtype=np.int32)
        dptr = None
        if depth is not None:
            depth = np.ascontiguousarray(depth, dtype=np.int32)
            dptr = _i32(depth)
        code = self._lib.oracle_check(self.n, _i64(self.offsets), _i32(self.adj), int(source),
                                      _i32(np.ascontiguousarray(depth_ref, dtype=np.int32)),
                                      _i32(parent), dptr, ctypes.byref(bad))
        return int(code), int(bad.value)

    def bc(self, sources, normalise: bool = True) -> np.ndarray:
        """Betweenness scores (float64[n]) from the given sources."""
        srcs = np.ascontiguousarray(sources, dtype=np.int32)
        out = np.empty(self.n, dtype=np.float64)
        r = self._lib.oracle_bc(self.n, _i64(self.offsets), _i32(self.adj), int(srcs.shape[0]),
                                _i32(srcs), 1 if normalise else 0,
                                out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
        if r != 0:
            raise ValueError("oracle_bc: bad input")
        return out

    def cc_check(self, label) -> tuple:
        """(code, bad_vertex) of the paper's component verifier; code 0 means
        the labelling is valid (this adjacency must be the undirected one)."""
        bad = ctypes.c_int64(-1)
        lab = np.ascontiguousarray(label, dtype=np.int32)
        code = self._lib.oracle_cc_check(self.n, _i64(self.offsets), _i32(self.adj), _i32(lab),
                                         ctypes.byref(bad))
        return int(code), int(bad.value)

    def component_edges(self, depth: np.ndarray) -> int:
        """Undirected edges inside the reached set: half the degree sum."""
        deg = self.degree()
        return int(deg[np.asarray(depth) >= 0].sum()) // 2


class WeightedAdjacency:
    """Weighted adjacency built by the oracle from raw (src, dst, weight)
    triples: undirected by default, out-lists with ``directed=True``; a
    repeated pair keeps its smallest weight."""

    def __init__(self, n: int, src, dst, w, _lib=None, directed: bool = False):
        L = _lib or lib()
        src = np.ascontiguousarray(src, dtype=np.int32)
        dst = np.ascontiguousarray(dst, dtype=np.int32)
        w = np.ascontiguousarray(w, dtype=np.int32)
        m = int(src.shape[0])
        self.n = int(n)
        self.offsets = np.zeros(self.n + 1, dtype=np.int64)
        cap = max((m if directed else 2 * m), 1)
        adj = np.empty(cap, dtype=np.int32)
        wadj = np.empty(cap, dtype=np.int32)
        nnz = L.oracle_build_weighted_adjacency(self.n, m, _i32(src), _i32(dst), _i32(w),
                                                1 if directed else 0, _i64(self.offsets),
                                                _i32(adj), _i32(wadj))
        if nnz < 0:
            raise ValueError("oracle_build_weighted_adjacency: bad input")
        self.adj = adj[:nnz].copy()
        self.wadj = wadj[:nnz].copy()
        self._lib = L

    def sssp(self, source: int) -> np.ndarray:
        """int64 distances, -1 when unreachable (Dijkstra)."""
        dist = np.empty(self.n, dtype=np.int64)
        if self._lib.oracle_sssp(self.n, _i64(self.offsets), _i32(self.adj), _i32(self.wadj),
                                 int(source), _i64(dist)) < 0:
            raise ValueError("oracle_sssp: bad input")
        return dist


def components(n: int, src: np.ndarray, dst: np.ndarray, _lib=None) -> np.ndarray:
    """Union-find component representative for every vertex (raw edges,
    taken as undirected): the smallest vertex of its component."""
    L = _lib or lib()
    src = np.ascontiguousarray(src, dtype=np.int32)
    dst = np.ascontiguousarray(dst, dtype=np.int32)
    label = np.empty(int(n), dtype=np.int32)
    if L.oracle_components(int(n), int(src.shape[0]), _i32(src), _i32(dst), _i32(label)) != 0:
        raise ValueError("oracle_components: bad input")
    return label
