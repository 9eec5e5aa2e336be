"""Seeded synthetic inputs: raw edge lists and trial sources.

Both the GPU library and the CPU oracle consume these edge lists; this module
contains no breadth-first-search arithmetic.  The graphs stand in for the
paper's Kron, Urand and Road inputs (Section 2.2); the trial sources follow
the measurement rules (Section 2.3: random non-zero-degree vertices).

The C generators live in ``gen.c`` and are built into ``libgapgen.so`` with
gcc/OpenMP.  Output is identical for any thread count (every draw is a pure
function of seed and counter).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "gen.c")
_LIB = os.path.join(_HERE, "libgapgen.so")
_lib = None

# Graph 500 / paper Section 2.2 Kron quadrant probabilities.
RMAT_A, RMAT_B, RMAT_C = 0.57, 0.19, 0.19


def build(force: bool = False) -> str:
    """Compile libgapgen.so with gcc (host only, OpenMP)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O3", "-march=x86-64-v2", "-fopenmp", "-fPIC", "-shared",
               "-std=c11", "-Wall", "-Wextra", "-o", tmp, _SRC]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        lib = ctypes.CDLL(_LIB)
        i32p = ctypes.POINTER(ctypes.c_int32)
        lib.gapgen_rmat.argtypes = [ctypes.c_int, ctypes.c_int64, ctypes.c_double,
                                    ctypes.c_double, ctypes.c_double, ctypes.c_uint64,
                                    ctypes.c_int, i32p, i32p]
        lib.gapgen_rmat.restype = ctypes.c_int64
        lib.gapgen_urand.argtypes = [ctypes.c_int64, ctypes.c_int64, ctypes.c_uint64, i32p, i32p]
        lib.gapgen_urand.restype = ctypes.c_int64
        lib.gapgen_grid.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_double,
                                    ctypes.c_int, ctypes.c_uint64, i32p, i32p, ctypes.c_int64]
        lib.gapgen_grid.restype = ctypes.c_int64
        lib.gapgen_grid_lattice_edges.argtypes = [ctypes.c_int, ctypes.c_int]
        lib.gapgen_grid_lattice_edges.restype = ctypes.c_int64
        lib.gapgen_grid_num_shortcuts.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_double]
        lib.gapgen_grid_num_shortcuts.restype = ctypes.c_int64
        lib.gapgen_pick_sources.argtypes = [ctypes.c_int64, ctypes.c_int64, i32p, i32p,
                                            ctypes.c_uint64, ctypes.c_int32, i32p]
        lib.gapgen_pick_sources.restype = ctypes.c_int32
        lib.gapgen_weights.argtypes = [ctypes.c_int64, i32p, i32p, ctypes.c_uint64, ctypes.c_int, i32p]
        lib.gapgen_weights.restype = ctypes.c_int
        lib.gapgen_pick_out_sources.argtypes = lib.gapgen_pick_sources.argtypes
        lib.gapgen_pick_out_sources.restype = ctypes.c_int32
        lib.gapgen_set_threads.argtypes = [ctypes.c_int]
        lib.gapgen_set_threads.restype = None
        lib.gapgen_max_threads.argtypes = []
        lib.gapgen_max_threads.restype = ctypes.c_int
        _lib = lib
    return _lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))


@dataclass
class EdgeList:
    """A raw generated edge list (may hold duplicates and self-loops)."""
    n: int
    src: np.ndarray  # int32[m]
    dst: np.ndarray  # int32[m]
    name: str = ""
    params: dict = field(default_factory=dict)

    @property
    def m(self) -> int:
        return int(self.src.shape[0])


def set_threads(t: int) -> None:
    _load().gapgen_set_threads(int(t))


def max_threads() -> int:
    return int(_load().gapgen_max_threads())


def rmat(scale: int, edge_factor: int = 16, seed: int = 1, permute: bool = True,
         a: float = RMAT_A, b: float = RMAT_B, c: float = RMAT_C) -> EdgeList:
    """R-MAT/Kronecker tuples: edge_factor * 2^scale raw pairs."""
    m = int(edge_factor) << int(scale)
    src = np.empty(m, dtype=np.int32)
    dst = np.empty(m, dtype=np.int32)
    got = _load().gapgen_rmat(int(scale), int(edge_factor), a, b, c, int(seed) & (2**64 - 1),
                              1 if permute else 0, _p(src), _p(dst))
    if got != m:
        raise ValueError("gapgen_rmat rejected its arguments")
    return EdgeList(1 << int(scale), src, dst, f"rmat{scale}",
                    dict(kind="rmat", scale=scale, edge_factor=edge_factor, seed=seed,
                         permute=permute, a=a, b=b, c=c))


def urand(n: int, m: int, seed: int = 1) -> EdgeList:
    """m uniform random endpoint pairs over n vertices."""
    src = np.empty(m, dtype=np.int32)
    dst = np.empty(m, dtype=np.int32)
    got = _load().gapgen_urand(int(n), int(m), int(seed) & (2**64 - 1), _p(src), _p(dst))
    if got != m:
        raise ValueError("gapgen_urand rejected its arguments")
    return EdgeList(int(n), src, dst, f"urand_n{n}", dict(kind="urand", n=n, m=m, seed=seed))


def urand_scale(scale: int, edge_factor: int = 16, seed: int = 1) -> EdgeList:
    e = urand(1 << scale, edge_factor << scale, seed)
    e.name = f"urand{scale}"
    e.params.update(scale=scale, edge_factor=edge_factor)
    return e


def grid(w: int, h: int, p_delete: float = 0.10, shortcut_frac: float = 0.01,
         max_offset: int = 3, seed: int = 1) -> EdgeList:
    """Road-like lattice with deletions and short diagonal shortcuts."""
    lib = _load()
    cap = int(lib.gapgen_grid_lattice_edges(w, h)) + int(lib.gapgen_grid_num_shortcuts(w, h, shortcut_frac))
    src = np.empty(max(cap, 1), dtype=np.int32)
    dst = np.empty(max(cap, 1), dtype=np.int32)
    got = lib.gapgen_grid(int(w), int(h), float(p_delete), float(shortcut_frac), int(max_offset),
                          int(seed) & (2**64 - 1), _p(src), _p(dst), cap)
    if got < 0:
        raise ValueError("gapgen_grid rejected its arguments")
    return EdgeList(int(w) * int(h), src[:got].copy(), dst[:got].copy(), f"grid{w}x{h}",
                    dict(kind="grid", w=w, h=h, p_delete=p_delete, shortcut_frac=shortcut_frac,
                         max_offset=max_offset, seed=seed))


def lattice_edge_count(w: int, h: int) -> int:
    return int(_load().gapgen_grid_lattice_edges(int(w), int(h)))


def shortcut_count(w: int, h: int, frac: float) -> int:
    return int(_load().gapgen_grid_num_shortcuts(int(w), int(h), float(frac)))


def pick_sources(el: EdgeList, k: int = 64, seed: int = 1, directed: bool = False) -> np.ndarray:
    """Up to k distinct uniform-random vertices with non-zero degree (with
    ``directed``, non-zero out-degree: pair e is the edge src[e] -> dst[e])."""
    out = np.empty(max(int(k), 1), dtype=np.int32)
    fn = _load().gapgen_pick_out_sources if directed else _load().gapgen_pick_sources
    got = fn(int(el.n), int(el.m), _p(el.src), _p(el.dst), int(seed) & (2**64 - 1), int(k), _p(out))
    if got < 0:
        raise ValueError("the source picker rejected its arguments")
    return out[:got].copy()


def weights(el: EdgeList, seed: int = 1, directed: bool = False) -> np.ndarray:
    """Integer weights 1..255 per raw pair (Section 2.2), a function of the
    pair's endpoints (unordered unless ``directed``) and the seed."""
    w = np.empty(max(el.m, 1), dtype=np.int32)
    if _load().gapgen_weights(int(el.m), _p(el.src), _p(el.dst), int(seed) & (2**64 - 1),
                              1 if directed else 0, _p(w)) != 0:
        raise ValueError("the weight generator rejected its arguments")
    return w[:el.m].copy()


# Named workloads (sizes and seeds of the measured configurations).
def workload(name: str) -> EdgeList:
    """Named synthetic workloads used by the tests and the benchmark."""
    if name == "rmat16":
        return rmat(16, 16, seed=16001)
    if name == "rmat22":
        return rmat(22, 16, seed=22001)
    if name == "rmat16d":  # the pairs taken as directed edges (skewed, like a social graph)
        return rmat(16, 16, seed=16003)
    if name == "rmat22d":
        return rmat(22, 16, seed=22003)
    if name == "urand22":
        e = urand_scale(22, 16, seed=22002)
        return e
    if name == "rmat24":
        return rmat(24, 16, seed=24001)
    if name == "grid4096":
        return grid(4096, 4096, seed=40960)
    raise KeyError(name)


SOURCE_SEEDS = {"rmat16": 1016001, "rmat22": 1022001, "urand22": 1022002,
                "rmat24": 1024001, "grid4096": 1040960, "rmat16d": 1016003, "rmat22d": 1022003}

# Seeds of the edge weights of the shortest-path workloads.
WEIGHT_SEEDS = {"rmat16": 2016001, "rmat22": 2022001, "urand22": 2022002, "grid4096": 2040960,
                "rmat16d": 2016003, "rmat22d": 2022003}

# Workloads whose pairs are directed edges (build with directed=True, pick
# sources with directed=True).
DIRECTED = {"rmat16d", "rmat22d"}
