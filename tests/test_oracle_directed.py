"""Pins of the directed oracle (out-lists; a search follows edge directions).

Section 2.1 defines the search output for a graph whose edges may be
directed (the paper's Twitter, Web and Road inputs are): parent[v] = u needs
an edge u -> v and depth[v] = depth[u] + 1.  The pins: every directed graph
on up to 4 vertices against Floyd-Warshall and boolean matrix powers,
random directed graphs against scipy's csgraph, closed forms, agreement
with the undirected oracle on symmetric inputs, invariants on R-MAT, and a
planted reversed parent edge."""

import numpy as np
import pytest
import scipy.sparse as sp
from scipy.sparse import csgraph

import oracle
from tests import smallgraphs as sg


def dadj(n, s, d, L=None):
    return oracle.Adjacency(n, np.asarray(s, np.int32), np.asarray(d, np.int32), _lib=L,
                            directed=True)


def pairs_of(mask, k):
    offd = [(i, j) for i in range(k) for j in range(k) if i != j]
    sel = [offd[b] for b in range(len(offd)) if (mask >> b) & 1]
    return ([p[0] for p in sel], [p[1] for p in sel])


@pytest.mark.parametrize("k", [1, 2, 3, 4])
def test_exhaustive_directed_vs_floyd_warshall(oracle_lib, k):
    offd = [(i, j) for i in range(k) for j in range(k) if i != j]
    masks = np.arange(1 << len(offd))
    mats = np.zeros((len(masks), k, k), np.int64)
    for b, (i, j) in enumerate(offd):
        mats[:, i, j] = (masks >> b) & 1
    fw = sg.floyd_warshall_batch(mats)
    for gi, mask in enumerate(masks):
        s, d = pairs_of(int(mask), k)
        A = dadj(k, s, d, oracle_lib)
        for src in range(k):
            depth, parent = A.bfs(src)
            assert depth.tolist() == fw[gi, src].tolist(), (mask, src)
            assert A.check(src, depth, parent, depth)[0] == 0


def test_random_k5_directed_vs_matrix_powers(oracle_lib):
    rng = np.random.default_rng(17)
    for _ in range(1500):
        k = 5
        mat = (rng.random((k, k)) < rng.uniform(0.1, 0.6)).astype(np.int64)
        np.fill_diagonal(mat, 0)
        s, d = np.nonzero(mat)
        A = dadj(k, s, d, oracle_lib)
        for src in range(k):
            depth, parent = A.bfs(src)
            assert depth.tolist() == sg.matrix_power_depths(mat, src).tolist()


def test_random_directed_vs_scipy(oracle_lib):
    rng = np.random.default_rng(23)
    for trial in range(60):
        n = int(rng.integers(2, 65))
        m = int(rng.integers(0, 4 * n))
        s = rng.integers(0, n, m).astype(np.int32)
        d = rng.integers(0, n, m).astype(np.int32)
        if m:  # repeats and self-loops on purpose
            s = np.concatenate([s, s[: m // 3], d[: 2]])
            d = np.concatenate([d, d[: m // 3], d[: 2]])
        A = dadj(n, s, d, oracle_lib)
        keep = s != d
        M = sp.coo_matrix((np.ones(int(keep.sum())), (s[keep], d[keep])), shape=(n, n)).tocsr()
        M.data[:] = 1.0
        dist = csgraph.shortest_path(M, directed=True, unweighted=True)
        for src in rng.integers(0, n, 3):
            depth, parent = A.bfs(int(src))
            ref = np.where(np.isinf(dist[src]), -1, dist[src]).astype(np.int64)
            assert depth.tolist() == ref.tolist(), (trial, src)
            assert A.check(int(src), depth, parent, depth)[0] == 0


def test_directed_closed_forms(oracle_lib):
    k = 9
    # directed path 0 -> 1 -> ... -> k-1
    A = dadj(k, range(k - 1), range(1, k), oracle_lib)
    for s in range(k):
        assert A.bfs(s)[0].tolist() == [v - s if v >= s else -1 for v in range(k)]
    # directed cycle
    A = dadj(k, range(k), [(v + 1) % k for v in range(k)], oracle_lib)
    for s in range(k):
        assert A.bfs(s)[0].tolist() == [(v - s) % k for v in range(k)]
    # out-star from 0 and in-star into 0
    out = dadj(k, [0] * (k - 1), range(1, k), oracle_lib)
    assert out.bfs(0)[0].tolist() == [0] + [1] * (k - 1)
    assert out.bfs(3)[0].tolist() == [-1, -1, -1, 0, -1, -1, -1, -1, -1]
    inn = dadj(k, range(1, k), [0] * (k - 1), oracle_lib)
    assert inn.bfs(0)[0].tolist() == [0] + [-1] * (k - 1)
    assert inn.bfs(4)[0].tolist() == [1, -1, -1, -1, 0, -1, -1, -1, -1]


def test_symmetric_directed_equals_undirected(oracle_lib):
    from paper_1508_03619_amd import inputs
    el = inputs.rmat(10, 8, seed=29)
    s = np.concatenate([el.src, el.dst])
    d = np.concatenate([el.dst, el.src])
    D = dadj(el.n, s, d, oracle_lib)
    U = oracle.Adjacency(el.n, el.src, el.dst, _lib=oracle_lib)
    assert np.array_equal(D.offsets, U.offsets) and np.array_equal(D.adj, U.adj)
    for src in inputs.pick_sources(el, 5, seed=30):
        assert np.array_equal(D.bfs(int(src))[0], U.bfs(int(src))[0])


def test_directed_invariants_rmat(oracle_lib):
    from paper_1508_03619_amd import inputs
    el = inputs.rmat(13, 16, seed=31)
    A = dadj(el.n, el.src, el.dst, oracle_lib)
    keep = el.src != el.dst
    M = sp.coo_matrix((np.ones(int(keep.sum())), (el.src[keep], el.dst[keep])),
                      shape=(el.n, el.n)).tocsr()
    rows = np.repeat(np.arange(el.n), np.diff(A.offsets))
    for src in inputs.pick_sources(el, 4, seed=32):
        depth, parent = A.bfs(int(src))
        assert depth[src] == 0 and parent[src] == src
        du, dv = depth[rows], depth[A.adj]
        reached = du >= 0
        assert np.all(dv[reached] >= 0)                 # closure along out-edges
        assert np.all(dv[reached] <= du[reached] + 1)   # no edge skips a level forward
        order = csgraph.breadth_first_order(M, int(src), directed=True, return_predecessors=False)
        assert int((depth >= 0).sum()) == len(order)
        assert A.check(int(src), depth, parent, depth)[0] == 0


def test_validator_rejects_reversed_parent_edge(oracle_lib):
    # 0 -> 1 -> 2 and 2 -> 3; also 3 -> 1 (so 1 has an in-neighbour 3 that is not its parent)
    A = dadj(4, [0, 1, 2, 3], [1, 2, 3, 1], oracle_lib)
    depth, parent = A.bfs(0)
    assert depth.tolist() == [0, 1, 2, 3]
    bad = parent.copy()
    bad[2] = 3  # 3 -> 2 is not an edge (2 -> 3 is)
    assert A.check(0, depth, bad, depth)[0] in (4, 5)
    bad = parent.copy()
    bad[3] = 1  # 1 -> 3 is not an edge
    assert A.check(0, depth, bad, depth)[0] == 4


# ---- pin functions for the mutation tests (return True when every pin holds)

def directed_pins_ok(L) -> bool:
    """Exhaustive k <= 3 against Floyd-Warshall, closed forms, agreement with
    the undirected oracle on symmetric input, and the reversed-edge check."""
    for k in (2, 3):
        offd = [(i, j) for i in range(k) for j in range(k) if i != j]
        masks = np.arange(1 << len(offd))
        mats = np.zeros((len(masks), k, k), np.int64)
        for b, (i, j) in enumerate(offd):
            mats[:, i, j] = (masks >> b) & 1
        fw = sg.floyd_warshall_batch(mats)
        for gi, mask in enumerate(masks):
            s, d = pairs_of(int(mask), k)
            A = dadj(k, s, d, L)
            for src in range(k):
                depth, parent = A.bfs(src)
                if depth.tolist() != fw[gi, src].tolist() or A.check(src, depth, parent, depth)[0]:
                    return False
    k = 7
    A = dadj(k, range(k - 1), range(1, k), L)
    if A.bfs(2)[0].tolist() != [v - 2 if v >= 2 else -1 for v in range(k)]:
        return False
    from paper_1508_03619_amd import inputs
    el = inputs.rmat(9, 8, seed=29)
    D = dadj(el.n, np.concatenate([el.src, el.dst]), np.concatenate([el.dst, el.src]), L)
    U = oracle.Adjacency(el.n, el.src, el.dst, _lib=L)
    if not (np.array_equal(D.offsets, U.offsets) and np.array_equal(D.adj, U.adj)):
        return False
    A = dadj(4, [0, 1, 2, 3], [1, 2, 3, 1], L)
    depth, parent = A.bfs(0)
    bad = parent.copy()
    bad[3] = 1
    return A.check(0, depth, bad, depth)[0] == 4


def test_directed_pin_function_passes(oracle_lib):
    assert directed_pins_ok(oracle_lib)


def test_directed_source_picker():
    """Sources of a directed workload have an out-edge, are distinct, and the
    picker is deterministic in its seed."""
    from paper_1508_03619_amd import inputs
    # 0 -> 1 only: vertex 1 has in-degree 1 but no out-edge
    el = inputs.EdgeList(4, np.array([0, 2, 3], np.int32), np.array([1, 2, 3], np.int32), "tiny")
    assert inputs.pick_sources(el, 8, seed=3, directed=True).tolist() == [0]
    assert sorted(inputs.pick_sources(el, 8, seed=3).tolist()) == [0, 1]
    el = inputs.workload("rmat16d")
    a = inputs.pick_sources(el, 64, seed=inputs.SOURCE_SEEDS["rmat16d"], directed=True)
    b = inputs.pick_sources(el, 64, seed=inputs.SOURCE_SEEDS["rmat16d"], directed=True)
    assert len(a) == 64 and len(set(a.tolist())) == 64 and np.array_equal(a, b)
    keep = el.src != el.dst
    outdeg = np.bincount(el.src[keep], minlength=el.n)
    assert (outdeg[a] > 0).all()
