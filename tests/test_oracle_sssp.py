"""Pins of the shortest-path oracle (Section 2.1, "SSSP": dist[source] = 0,
the sentinel for unreachable vertices, otherwise the least total weight of a
path; Section 2.2: integer weights 1..255 for unweighted graphs).

Independent references: Floyd-Warshall (min-plus closure) on every graph of
4 vertices and every digraph of 3 vertices under several weightings;
scipy's Dijkstra on random graphs; unit weights against the BFS depths;
closed forms; and the two properties that define the answer on R-MAT: no
edge shortens a distance, and every reached vertex other than the source
has an edge that attains its distance."""
import itertools

import numpy as np
import pytest
import scipy.sparse as sp
from scipy.sparse import csgraph

import oracle
from tests import smallgraphs as sg


def wadj(n, s, d, w, L=None, directed=False):
    return oracle.WeightedAdjacency(n, np.asarray(s, np.int32), np.asarray(d, np.int32),
                                    np.asarray(w, np.int32), _lib=L, directed=directed)


def floyd_warshall(n, s, d, w, directed):
    INF = np.iinfo(np.int64).max // 4
    D = np.full((n, n), INF, np.int64)
    np.fill_diagonal(D, 0)
    for a, b, c in zip(s, d, w):
        if a == b:
            continue
        D[a, b] = min(D[a, b], c)
        if not directed:
            D[b, a] = min(D[b, a], c)
    for k in range(n):
        D = np.minimum(D, D[:, k:k + 1] + D[k:k + 1, :])
    return np.where(D >= INF, -1, D)


def min_reduced(n, s, d, w, directed):
    """Distinct pairs with their smallest weight (scipy would add repeats)."""
    s, d, w = np.asarray(s), np.asarray(d), np.asarray(w)
    keep = s != d
    s, d, w = s[keep], d[keep], w[keep]
    if not directed:
        s, d = np.concatenate([s, d]), np.concatenate([d, s])
        w = np.concatenate([w, w])
    order = np.lexsort((w, d, s))
    s, d, w = s[order], d[order], w[order]
    first = np.ones(len(s), bool)
    first[1:] = (s[1:] != s[:-1]) | (d[1:] != d[:-1])
    return s[first], d[first], w[first]


def test_all_four_vertex_graphs_vs_floyd_warshall(oracle_lib):
    k = 4
    pairs = list(itertools.combinations(range(k), 2))
    rng = np.random.default_rng(81)
    for mask in range(1 << len(pairs)):
        sel = [pairs[b] for b in range(len(pairs)) if (mask >> b) & 1]
        s = [p[0] for p in sel]
        d = [p[1] for p in sel]
        for _ in range(3):
            w = rng.integers(1, 4, len(sel))
            ref = floyd_warshall(k, s, d, w, False)
            A = wadj(k, s, d, w, oracle_lib)
            for src in range(k):
                assert A.sssp(src).tolist() == ref[src].tolist(), (mask, list(w), src)


def test_all_three_vertex_digraphs_vs_floyd_warshall(oracle_lib):
    k = 3
    offd = [(i, j) for i in range(k) for j in range(k) if i != j]
    rng = np.random.default_rng(82)
    for mask in range(1 << len(offd)):
        sel = [offd[b] for b in range(len(offd)) if (mask >> b) & 1]
        s = [p[0] for p in sel]
        d = [p[1] for p in sel]
        for _ in range(3):
            w = rng.integers(1, 5, len(sel))
            ref = floyd_warshall(k, s, d, w, True)
            A = wadj(k, s, d, w, oracle_lib, directed=True)
            for src in range(k):
                assert A.sssp(src).tolist() == ref[src].tolist(), (mask, list(w), src)


def test_random_graphs_vs_scipy_dijkstra(oracle_lib):
    rng = np.random.default_rng(83)
    for trial in range(60):
        n = int(rng.integers(2, 80))
        m = int(rng.integers(0, 4 * n))
        s = rng.integers(0, n, m).astype(np.int32)
        d = rng.integers(0, n, m).astype(np.int32)
        w = rng.integers(1, 256, m).astype(np.int32)
        if m:  # repeated pairs with other weights, and self-loops
            s = np.concatenate([s, s[: m // 3], d[:2]])
            d = np.concatenate([d, d[: m // 3], d[:2]])
            w = np.concatenate([w, rng.integers(1, 256, m // 3 + min(2, m)).astype(np.int32)])
        directed = bool(trial % 2)
        A = wadj(n, s, d, w, oracle_lib, directed)
        rs, rd, rw = min_reduced(n, s, d, w, directed)
        M = sp.csr_matrix((rw.astype(float), (rs, rd)), shape=(n, n))
        for src in rng.integers(0, n, 3):
            ref = csgraph.dijkstra(M, directed=True, indices=int(src))
            ref = np.where(np.isinf(ref), -1, ref).astype(np.int64)
            assert A.sssp(int(src)).tolist() == ref.tolist(), (trial, src)


def test_unit_weights_equal_bfs_depths(oracle_lib):
    from paper_1508_03619_amd import inputs
    for el in (inputs.rmat(12, 16, seed=84), inputs.grid(40, 30, seed=85)):
        A = wadj(el.n, el.src, el.dst, np.ones(el.m, np.int32), oracle_lib)
        B = oracle.Adjacency(el.n, el.src, el.dst, _lib=oracle_lib)
        for src in inputs.pick_sources(el, 4, seed=86):
            assert np.array_equal(A.sssp(int(src)), B.bfs(int(src))[0].astype(np.int64))


def test_closed_forms(oracle_lib):
    k = 9
    w = np.arange(1, k, dtype=np.int32) * 3
    A = wadj(k, range(k - 1), range(1, k), w, oracle_lib)
    pre = np.concatenate([[0], np.cumsum(w)])
    assert A.sssp(0).tolist() == pre.tolist()
    assert A.sssp(4).tolist() == np.abs(pre - pre[4]).tolist()
    # cycle: the shorter way round
    wc = np.array([5, 1, 1, 1, 1, 1, 1, 1, 1], np.int32)
    C = wadj(k, range(k), [(v + 1) % k for v in range(k)], wc, oracle_lib)
    fw = np.concatenate([[0], np.cumsum(wc)])[:k]
    bw = np.concatenate([[0], np.cumsum(wc[::-1])])[:k][::-1]
    bw = np.roll(bw, 1)
    assert C.sssp(0).tolist() == np.minimum(fw, bw).tolist()
    # star with centre 0: leaf to leaf through the centre
    ws = np.arange(1, k, dtype=np.int32)
    S = wadj(k, [0] * (k - 1), range(1, k), ws, oracle_lib)
    assert S.sssp(0).tolist() == [0] + ws.tolist()
    assert S.sssp(2).tolist() == [2, 3] + [0] + (ws[2:] + 2).tolist()
    # repeated pair keeps its smallest weight; self-loops ignored; isolated
    R = wadj(4, [0, 0, 1, 2, 3], [1, 1, 1, 2, 3], [9, 4, 7, 1, 1], oracle_lib)
    assert R.sssp(0).tolist() == [0, 4, -1, -1]
    with pytest.raises(ValueError):
        wadj(3, [0], [1], [0], oracle_lib)


def defining_properties_ok(L, n, s, d, w, sources, directed=False) -> bool:
    """dist[src] = 0; along every edge u -> v with u reached, v is reached
    and dist[v] <= dist[u] + w; every reached v != src has an in-edge with
    dist[u] + w == dist[v]."""
    A = wadj(n, s, d, w, L, directed)
    rows = np.repeat(np.arange(n), np.diff(A.offsets))
    for src in sources:
        dist = A.sssp(int(src))
        if dist[src] != 0:
            return False
        du, dv = dist[rows], dist[A.adj]
        ok = du >= 0
        if np.any(dv[ok] < 0) or np.any(dv[ok] > du[ok] + A.wadj[ok]):
            return False
        tight = np.zeros(n, bool)
        tight[A.adj[ok & (dv == du + A.wadj)]] = True
        reached = dist >= 0
        reached[src] = False
        if not np.all(tight[reached]):
            return False
    return True


def test_defining_properties_rmat(oracle_lib):
    from paper_1508_03619_amd import inputs
    el = inputs.rmat(12, 16, seed=87)
    w = inputs.weights(el, seed=88)
    assert w.min() >= 1 and w.max() <= 255
    assert defining_properties_ok(oracle_lib, el.n, el.src, el.dst, w, inputs.pick_sources(el, 4, seed=89))
    wd = inputs.weights(el, seed=88, directed=True)
    assert defining_properties_ok(oracle_lib, el.n, el.src, el.dst, wd,
                                  inputs.pick_sources(el, 4, seed=90, directed=True), directed=True)


def test_generated_weights_are_symmetric_and_uniform():
    from paper_1508_03619_amd import inputs
    el = inputs.urand(1 << 12, 1 << 17, seed=91)
    w = inputs.weights(el, seed=92)
    rev = inputs.weights(inputs.EdgeList(el.n, el.dst, el.src, "rev"), seed=92)
    assert np.array_equal(w, rev)
    counts = np.bincount(w, minlength=256)
    assert counts[0] == 0 and counts[1:].min() > 0.8 * len(w) / 255 and counts[1:].max() < 1.2 * len(w) / 255


# ---- pin function for the mutation tests ----------------------------------

def sssp_pins_ok(L) -> bool:
    try:
        k = 4
        pairs = list(itertools.combinations(range(k), 2))
        rng = np.random.default_rng(93)
        for mask in range(1 << len(pairs)):
            sel = [pairs[b] for b in range(len(pairs)) if (mask >> b) & 1]
            s = [p[0] for p in sel]
            d = [p[1] for p in sel]
            w = rng.integers(1, 4, len(sel))
            ref = floyd_warshall(k, s, d, w, False)
            A = wadj(k, s, d, w, L)
            for src in range(k):
                if A.sssp(src).tolist() != ref[src].tolist():
                    return False
        R = wadj(4, [0, 0, 1], [1, 1, 2], [9, 4, 1], L)
        if R.sssp(0).tolist() != [0, 4, 5, -1]:
            return False
        D = wadj(3, [0, 1], [1, 2], [2, 3], L, directed=True)
        if D.sssp(2).tolist() != [-1, -1, 0] or D.sssp(0).tolist() != [0, 2, 5]:
            return False
        from paper_1508_03619_amd import inputs
        el = inputs.rmat(9, 8, seed=94)
        return defining_properties_ok(L, el.n, el.src, el.dst, inputs.weights(el, seed=95),
                                      inputs.pick_sources(el, 2, seed=96))
    except Exception:
        return False


def test_sssp_pin_function_passes(oracle_lib):
    assert sssp_pins_ok(oracle_lib)
