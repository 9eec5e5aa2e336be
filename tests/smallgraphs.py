"""Small graph families with closed-form BFS depths, and the golden parser.

Each builder returns (n, src, dst) as raw int32 edge arrays, plus a function
giving the exact hop distance from a source (or -1) for every vertex.
"""
from __future__ import annotations

import os

import numpy as np

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _arr(pairs):
    if not pairs:
        return np.zeros(0, np.int32), np.zeros(0, np.int32)
    a = np.asarray(pairs, dtype=np.int32)
    return a[:, 0].copy(), a[:, 1].copy()


def path(k):
    s, d = _arr([(i, i + 1) for i in range(k - 1)])
    return k, s, d, lambda src: np.abs(np.arange(k) - src)


def cycle(k):
    s, d = _arr([(i, (i + 1) % k) for i in range(k)])

    def dist(src):
        t = np.abs(np.arange(k) - src)
        return np.minimum(t, k - t)
    return k, s, d, dist


def star(k):
    """Centre 0, leaves 1..k-1."""
    s, d = _arr([(0, i) for i in range(1, k)])

    def dist(src):
        if src == 0:
            r = np.ones(k, np.int64)
            r[0] = 0
            return r
        r = np.full(k, 2, np.int64)
        r[0] = 1
        r[src] = 0
        return r
    return k, s, d, dist


def complete(k):
    s, d = _arr([(i, j) for i in range(k) for j in range(i + 1, k)])

    def dist(src):
        r = np.ones(k, np.int64)
        r[src] = 0
        return r
    return k, s, d, dist


def bipartite(a, b):
    """K_{a,b}: side A = 0..a-1, side B = a..a+b-1."""
    s, d = _arr([(i, a + j) for i in range(a) for j in range(b)])
    k = a + b

    def dist(src):
        side = np.arange(k) >= a
        r = np.where(side == (src >= a), 2, 1).astype(np.int64)
        r[src] = 0
        return r
    return k, s, d, dist


def hypercube(dim):
    k = 1 << dim
    s, d = _arr([(v, v ^ (1 << i)) for v in range(k) for i in range(dim) if v < v ^ (1 << i)])

    def dist(src):
        x = np.arange(k) ^ src
        return np.array([bin(int(t)).count("1") for t in x], np.int64)
    return k, s, d, dist


def binary_tree(k):
    """Heap-indexed complete binary tree; closed form only from the root."""
    s, d = _arr([((i - 1) // 2, i) for i in range(1, k)])
    return k, s, d, lambda src: np.floor(np.log2(np.arange(k) + 1)).astype(np.int64)


def full_grid(w, h):
    pairs = []
    for y in range(h):
        for x in range(w):
            v = y * w + x
            if x + 1 < w:
                pairs.append((v, v + 1))
            if y + 1 < h:
                pairs.append((v, v + w))
    s, d = _arr(pairs)
    k = w * h

    def dist(src):
        xs, ys = np.arange(k) % w, np.arange(k) // w
        return np.abs(xs - src % w) + np.abs(ys - src // w)
    return k, s, d, dist


def disjoint_union(*parts):
    """Union of (n, src, dst, dist) parts; distance -1 across parts."""
    offs = np.cumsum([0] + [p[0] for p in parts])
    n = int(offs[-1])
    src = np.concatenate([p[1] + offs[i] for i, p in enumerate(parts)]).astype(np.int32)
    dst = np.concatenate([p[2] + offs[i] for i, p in enumerate(parts)]).astype(np.int32)

    def dist(s):
        r = np.full(n, -1, np.int64)
        i = int(np.searchsorted(offs, s, side="right") - 1)
        r[offs[i]:offs[i + 1]] = parts[i][3](s - offs[i])
        return r
    return n, src, dst, dist


def read_golden(name="tiny_graphs.txt"):
    """[(graph_name, n, src, dst, [(source, depths), ...]), ...]"""
    cases = []
    cur = None
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.split("#", 1)[0].strip()
            if not line:
                continue
            tok = line.split()
            if tok[0] == "graph":
                cur = [tok[1], int(tok[2]), None, None, []]
            elif tok[0] == "edges":
                pairs = [tuple(int(x) for x in t.split("-")) for t in tok[1:]]
                cur[2], cur[3] = _arr(pairs)
            elif tok[0] == "source":
                assert tok[2] == "depths"
                cur[4].append((int(tok[1]), np.array([int(x) for x in tok[3:]], np.int32)))
            elif tok[0] == "end":
                cases.append(tuple(cur))
                cur = None
    return cases


def floyd_warshall_batch(adjm: np.ndarray) -> np.ndarray:
    """All-pairs hop distances for a batch of 0/1 matrices (B, k, k); -1 = inf."""
    B, k, _ = adjm.shape
    INF = 10 ** 6
    d = np.where(adjm > 0, 1, INF).astype(np.int64)
    idx = np.arange(k)
    d[:, idx, idx] = 0
    for m in range(k):
        d = np.minimum(d, d[:, :, m:m + 1] + d[:, m:m + 1, :])
    return np.where(d >= INF, -1, d)


def matrix_power_depths(adjm: np.ndarray, s: int) -> np.ndarray:
    """depth[v] = min{t : (A^t)[s][v] != 0}, A^0 = I; -1 if never."""
    k = adjm.shape[0]
    a = (adjm > 0).astype(np.int64)
    reach = np.zeros(k, np.int64)
    reach[s] = 1
    depth = np.full(k, -1, np.int64)
    depth[s] = 0
    row = reach.copy()
    for t in range(1, k):
        row = (row @ a > 0).astype(np.int64)
        newly = (row > 0) & (depth < 0)
        depth[newly] = t
    return depth
