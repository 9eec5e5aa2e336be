"""Pins for the CPU oracle: values that do not come from the oracle itself.

Every test here runs on the CPU.  The pins are chosen so that a plausible
mistake in the oracle (a dropped term, a wrong index, a missing direction,
LIFO instead of FIFO order, a wrong parent) fails at least one of them;
``test_oracle_mutants.py`` plants such mistakes and checks that they do.
"""
import itertools

import numpy as np
import pytest
import scipy.sparse as sp
from scipy.sparse import csgraph

import oracle
from tests import smallgraphs as sg


def _adj(n, s, d, L=None):
    return oracle.Adjacency(n, s, d, _lib=L)


# ---- 1. exhaustive small graphs: Floyd-Warshall and matrix powers --------

def exhaustive_depths_ok(L, k):
    pairs = list(itertools.combinations(range(k), 2))
    ng = 1 << len(pairs)
    mats = np.zeros((ng, k, k), np.int64)
    for gi in range(ng):
        for b, (u, v) in enumerate(pairs):
            if gi >> b & 1:
                mats[gi, u, v] = mats[gi, v, u] = 1
    fw = sg.floyd_warshall_batch(mats)
    for gi in range(ng):
        es = [pairs[b] for b in range(len(pairs)) if gi >> b & 1]
        s = np.array([e[0] for e in es], np.int32)
        d = np.array([e[1] for e in es], np.int32)
        A = _adj(k, s, d, L)
        for src in range(k):
            depth, parent = A.bfs(src)
            if not np.array_equal(depth, fw[gi, src]):
                return False
            if A.check(src, fw[gi, src].astype(np.int32), parent)[0] != 0:
                return False
    return True


@pytest.mark.parametrize("k", [1, 2, 3, 4, 5])
def test_exhaustive_vs_floyd_warshall(oracle_lib, k):
    assert exhaustive_depths_ok(oracle_lib, k)


def test_exhaustive_k6_vs_floyd_warshall(oracle_lib):
    """All 32,768 labelled simple graphs on 6 vertices, every source."""
    assert exhaustive_depths_ok(oracle_lib, 6)


def test_exhaustive_vs_matrix_powers(oracle_lib):
    k = 5
    pairs = list(itertools.combinations(range(k), 2))
    for gi in range(1 << len(pairs)):
        es = [pairs[b] for b in range(len(pairs)) if gi >> b & 1]
        m = np.zeros((k, k), np.int64)
        for u, v in es:
            m[u, v] = m[v, u] = 1
        s = np.array([e[0] for e in es], np.int32)
        d = np.array([e[1] for e in es], np.int32)
        A = _adj(k, s, d, oracle_lib)
        for src in range(k):
            assert np.array_equal(A.bfs(src)[0], sg.matrix_power_depths(m, src))


# ---- 2. random graphs with repeats and self-loops vs scipy ---------------

def _scipy_csr(n, s, d):
    m = sp.coo_matrix((np.ones(len(s)), (s, d)), shape=(n, n)).tocsr()
    m = m + m.T
    m.setdiag(0)
    m.eliminate_zeros()
    m.sort_indices()
    return m


def random_graph_ok(L, seed):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(1, 65))
    dens = rng.choice([0.0, 0.02, 0.05, 0.1, 0.3, 0.8])
    m = int(rng.binomial(n * n, dens)) if n > 1 else int(rng.integers(0, 3))
    s = rng.integers(0, n, m).astype(np.int32)
    d = rng.integers(0, n, m).astype(np.int32)
    if m:  # deliberate repeats and self-loops
        k = max(1, m // 8)
        s = np.concatenate([s, s[:k], d[:k]]).astype(np.int32)
        d = np.concatenate([d, d[:k], d[:k]]).astype(np.int32)
    A = _adj(n, s, d, L)
    ref = _scipy_csr(n, s, d)
    if not (np.array_equal(A.offsets, ref.indptr) and np.array_equal(A.adj, ref.indices)):
        return False
    dist = csgraph.shortest_path(ref, method="D", unweighted=True, directed=False)
    dist = np.where(np.isinf(dist), -1, dist).astype(np.int64)
    for src in range(n):
        depth, parent = A.bfs(src)
        if not np.array_equal(depth, dist[src]):
            return False
        if A.check(src, depth, parent, depth)[0] != 0:
            return False
    return True


def test_random_graphs_vs_scipy(oracle_lib):
    for seed in range(120):
        assert random_graph_ok(oracle_lib, seed), seed


# ---- 3. closed forms -----------------------------------------------------

CLOSED = [
    ("path1", lambda: sg.path(1)), ("path2", lambda: sg.path(2)), ("path17", lambda: sg.path(17)),
    ("cycle3", lambda: sg.cycle(3)), ("cycle10", lambda: sg.cycle(10)), ("cycle11", lambda: sg.cycle(11)),
    ("star9", lambda: sg.star(9)), ("K7", lambda: sg.complete(7)), ("K3,5", lambda: sg.bipartite(3, 5)),
    ("Q5", lambda: sg.hypercube(5)), ("grid7x5", lambda: sg.full_grid(7, 5)),
    ("grid1x9", lambda: sg.full_grid(1, 9)),
    ("union", lambda: sg.disjoint_union(sg.path(4), sg.cycle(5), sg.star(4), sg.path(1))),
]


def closed_forms_ok(L):
    for name, mk in CLOSED:
        n, s, d, dist = mk()
        A = _adj(n, s, d, L)
        for src in range(n):
            depth, parent = A.bfs(src)
            if not np.array_equal(depth, dist(src)):
                return False
            if A.check(src, depth, parent)[0] != 0:
                return False
    n, s, d, dist = sg.binary_tree(31)
    if not np.array_equal(_adj(n, s, d, L).bfs(0)[0], dist(0)):
        return False
    return True


def test_closed_forms(oracle_lib):
    assert closed_forms_ok(oracle_lib)


def test_isolated_source(oracle_lib):
    n, s, d, _ = sg.disjoint_union(sg.path(3), sg.path(1), sg.cycle(4))
    A = _adj(n, s, d, oracle_lib)
    depth, parent = A.bfs(3)
    assert depth[3] == 0 and parent[3] == 3
    assert (np.delete(depth, 3) == -1).all() and (np.delete(parent, 3) == -1).all()


def test_no_edges(oracle_lib):
    A = _adj(5, np.zeros(0, np.int32), np.zeros(0, np.int32), oracle_lib)
    assert A.nnz == 0
    depth, parent = A.bfs(2)
    assert depth.tolist() == [-1, -1, 0, -1, -1] and parent.tolist() == [-1, -1, 2, -1, -1]


def test_full_grid_large_closed_form(oracle_lib):
    """Undeleted 256x128 lattice: depth is the Manhattan distance."""
    n, s, d, dist = sg.full_grid(256, 128)
    A = _adj(n, s, d, oracle_lib)
    for src in (0, 255, 128 * 256 - 1, 64 * 256 + 100):
        assert np.array_equal(A.bfs(src)[0], dist(src))


# ---- golden, hand-worked ------------------------------------------------

def golden_ok(L):
    for name, n, s, d, cases in sg.read_golden():
        A = _adj(n, s, d, L)
        for src, want in cases:
            depth, parent = A.bfs(src)
            if not np.array_equal(depth, want):
                return False
            if A.check(src, want, parent)[0] != 0:
                return False
    return True


def test_golden_hand_worked(oracle_lib):
    assert golden_ok(oracle_lib)


# ---- 4. invariants on a generated R-MAT graph ---------------------------

def invariants_ok(L, el, sources):
    A = _adj(el.n, el.src, el.dst, L)
    comp = oracle.components(el.n, el.src, el.dst, _lib=L)
    rows = np.repeat(np.arange(el.n), np.diff(A.offsets))
    for src in sources:
        depth, parent = A.bfs(int(src))
        if depth[src] != 0:
            return False
        a, b = depth[rows], depth[A.adj]
        both = (a >= 0) & (b >= 0)
        if np.abs(a[both] - b[both]).max(initial=0) > 1:
            return False
        if ((a >= 0) != (b >= 0)).any():  # closure: no edge leaves the reached set
            return False
        if not np.array_equal(depth >= 0, comp == comp[src]):
            return False
        if A.check(int(src), depth, parent)[0] != 0:
            return False
    return True


def test_invariants_rmat(oracle_lib):
    from paper_1508_03619_amd import inputs
    el = inputs.rmat(12, 16, seed=7)
    srcs = inputs.pick_sources(el, 8, seed=8)
    assert len(srcs) == 8
    assert invariants_ok(oracle_lib, el, srcs)


@pytest.mark.slow
def test_invariants_rmat16_and_grid(oracle_lib):
    from paper_1508_03619_amd import inputs
    el = inputs.workload("rmat16")
    assert invariants_ok(oracle_lib, el, inputs.pick_sources(el, 4, seed=inputs.SOURCE_SEEDS["rmat16"]))
    g = inputs.grid(96, 80, seed=3)
    assert invariants_ok(oracle_lib, g, inputs.pick_sources(g, 4, seed=4))


# ---- 5. adjacency against scipy on a generated graph --------------------

def test_adjacency_matches_scipy_rmat(oracle_lib):
    from paper_1508_03619_amd import inputs
    el = inputs.rmat(13, 16, seed=11)
    A = _adj(el.n, el.src, el.dst, oracle_lib)
    ref = _scipy_csr(el.n, el.src, el.dst)
    assert np.array_equal(A.offsets, ref.indptr)
    assert np.array_equal(A.adj, ref.indices)


# ---- 6. validator sensitivity: planted mistakes are rejected -------------

def validator_ok(L):
    """True when the validator rejects every planted mistake with the right code."""
    n, s, d, dist = sg.disjoint_union(sg.full_grid(6, 5), sg.cycle(5), sg.path(1))
    # a diagonal 7-14 closes the triangle 7-8-14, so 8 and 14 are neighbours
    # on the same level when the search starts at 7
    s = np.append(s, np.int32(7)).astype(np.int32)
    d = np.append(d, np.int32(14)).astype(np.int32)
    A = _adj(n, s, d, L)
    src = 7
    depth, parent = A.bfs(src)
    if A.check(src, depth, parent, depth) != (0, -1):
        return False
    far = int(np.argmax(depth))          # a reached vertex at the largest depth
    unreached = int(np.flatnonzero(depth < 0)[0])
    tgt, nonadj = next((v, u) for v in range(30) for u in range(30)
                       if depth[v] >= 2 and depth[u] == depth[v] - 1
                       and u not in A.adj[A.offsets[v]:A.offsets[v + 1]])
    deep_v, deep_u = next((v, int(u)) for v in range(30) for u in A.adj[A.offsets[v]:A.offsets[v + 1]]
                          if depth[v] >= 1 and depth[u] == depth[v] + 1)
    planted = []
    p = parent.copy(); p[14] = 8; planted.append((p, None, 5))          # neighbour, same level
    p = parent.copy(); p[deep_v] = deep_u; planted.append((p, None, 5))  # neighbour, one level down
    p = parent.copy(); p[src] = -1; planted.append((p, None, 2))
    p = parent.copy(); p[unreached] = 0; planted.append((p, None, 3))
    p = parent.copy(); p[far] = -1; planted.append((p, None, 3))
    p = parent.copy(); p[far] = -5; planted.append((p, None, 3))      # leaked negative encoding
    p = parent.copy(); p[far] = n + 3; planted.append((p, None, 4))   # out of range
    p = parent.copy(); p[tgt] = nonadj; planted.append((p, None, 4))  # right level, not a neighbour
    dd = depth.copy(); dd[far] += 1; planted.append((parent, dd, 1))
    for p, dtest, code in planted:
        if A.check(src, depth, p, dtest)[0] != code:
            return False
    return True


def test_validator_rejects_planted_mistakes(oracle_lib):
    assert validator_ok(oracle_lib)


def test_validator_accepts_any_valid_parent(oracle_lib):
    """Several parent arrays are correct; the validator takes any of them."""
    n, s, d, _ = sg.cycle(4)
    A = _adj(n, s, d, oracle_lib)
    depth, parent = A.bfs(0)
    for p2 in (1, 3):
        p = parent.copy(); p[2] = p2
        assert A.check(0, depth, p)[0] == 0


# ---- union-find (reachability pin) against scipy ------------------------

def test_components_vs_scipy(oracle_lib):
    from paper_1508_03619_amd import inputs
    el = inputs.rmat(11, 4, seed=5)
    lab = oracle.components(el.n, el.src, el.dst, _lib=oracle_lib)
    k, ref = csgraph.connected_components(_scipy_csr(el.n, el.src, el.dst), directed=False)
    # same partition: labels map one-to-one
    pairs = set(zip(lab.tolist(), ref.tolist()))
    assert len(pairs) == len(set(lab.tolist())) == k
