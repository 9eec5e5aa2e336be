"""Pins of the betweenness-centrality oracle (Section 2.1, "Betweenness
Centrality": score[v] sums sigma_st(v) / sigma_st over the chosen sources s
and all targets t, then the scores are normalised to one).

The definition itself is evaluated on small graphs by listing every simple
path from each source and keeping the shortest ones per target (exact
rational arithmetic, no path counting recursion, no dependency recursion).
Also: closed forms on paths, stars, cycles, complete and complete bipartite
graphs; the identity that one source's dependencies add up to the sum of
(distance - 1) over the vertices it reaches; additivity over sources;
normalisation."""
from fractions import Fraction
import itertools

import numpy as np
import pytest

import oracle
from tests import smallgraphs as sg


def adj_lists(n, s, d, directed):
    out = [set() for _ in range(n)]
    for a, b in zip(s, d):
        a, b = int(a), int(b)
        if a == b:
            continue
        out[a].add(b)
        if not directed:
            out[b].add(a)
    return [sorted(x) for x in out]


def definition_bc(n, s, d, sources, directed=False):
    """sum_s sum_t sigma_st(v)/sigma_st from an explicit list of every
    shortest path (simple paths enumerated depth-first)."""
    out = adj_lists(n, s, d, directed)
    score = [Fraction(0)] * n
    for src in sources:
        best = {}      # target -> (length, [paths])
        stack = [(src, (src,))]
        while stack:
            u, path = stack.pop()
            t = path[-1]
            L = len(path) - 1
            if t != src:
                if t not in best or L < best[t][0]:
                    best[t] = (L, [path])
                elif L == best[t][0]:
                    best[t][1].append(path)
            for w in out[u]:
                if w not in path:
                    stack.append((w, path + (w,)))
        for t, (_, paths) in best.items():
            for v in range(n):
                if v in (src, t):
                    continue
                through = sum(1 for p in paths if v in p)
                if through:
                    score[v] += Fraction(through, len(paths))
    return score


def close(a, b, rtol=1e-12):
    a = np.asarray(a, float)
    b = np.asarray(b, float)
    return np.all(np.abs(a - b) <= rtol * np.maximum(1.0, np.abs(b)))


def obc(n, s, d, sources, L=None, directed=False, normalise=False):
    A = oracle.Adjacency(n, np.asarray(s, np.int32), np.asarray(d, np.int32), _lib=L,
                         directed=directed)
    return A.bc(sources, normalise=normalise)


def test_exhaustive_four_vertex_graphs_match_definition(oracle_lib):
    k = 4
    pairs = list(itertools.combinations(range(k), 2))
    for mask in range(1 << len(pairs)):
        sel = [pairs[b] for b in range(len(pairs)) if (mask >> b) & 1]
        s = [p[0] for p in sel]
        d = [p[1] for p in sel]
        for srcs in ([0], [1, 3], [0, 1, 2, 3]):
            ref = definition_bc(k, s, d, srcs)
            assert close(obc(k, s, d, srcs, oracle_lib), [float(x) for x in ref]), (mask, srcs)


def test_exhaustive_three_vertex_digraphs_match_definition(oracle_lib):
    k = 3
    offd = [(i, j) for i in range(k) for j in range(k) if i != j]
    for mask in range(1 << len(offd)):
        sel = [offd[b] for b in range(len(offd)) if (mask >> b) & 1]
        s = [p[0] for p in sel]
        d = [p[1] for p in sel]
        for srcs in ([0], [2, 1]):
            ref = definition_bc(k, s, d, srcs, directed=True)
            got = obc(k, s, d, srcs, oracle_lib, directed=True)
            assert close(got, [float(x) for x in ref]), (mask, srcs)


def test_random_small_graphs_match_definition(oracle_lib):
    rng = np.random.default_rng(61)
    for trial in range(80):
        n = int(rng.integers(2, 8))
        m = int(rng.integers(0, 2 * n + 2))
        s = rng.integers(0, n, m)
        d = rng.integers(0, n, m)
        directed = bool(trial % 2)
        srcs = [int(x) for x in rng.integers(0, n, int(rng.integers(1, 5)))]
        ref = definition_bc(n, s, d, srcs, directed=directed)
        got = obc(n, s, d, srcs, oracle_lib, directed=directed)
        assert close(got, [float(x) for x in ref]), (trial, n, srcs, directed)


def test_closed_forms(oracle_lib):
    L = oracle_lib
    for n in (2, 3, 7, 20):
        n_, s, d, _ = sg.path(n)
        got = obc(n, s, d, [0], L)
        assert got.tolist() == [0.0] + [float(n - 1 - i) for i in range(1, n - 1)] + ([0.0] if n > 1 else [])
    # star: centre 0, leaves 1..n-1
    for n in (3, 9):
        n_, s, d, _ = sg.star(n)
        assert obc(n, s, d, [1], L).tolist() == [float(n - 2)] + [0.0] * (n - 1)
        assert obc(n, s, d, [0], L).tolist() == [0.0] * n
    # complete graph: every pair adjacent
    n_, s, d, _ = sg.complete(7)
    assert obc(7, s, d, [0, 3], L).tolist() == [0.0] * 7
    # odd cycle 2m+1: the two vertices at distance i carry m - i
    m = 5
    n_, s, d, _ = sg.cycle(2 * m + 1)
    got = obc(2 * m + 1, s, d, [0], L)
    for v in range(1, 2 * m + 1):
        i = min(v, 2 * m + 1 - v)
        assert got[v] == float(m - i)
    # even cycle 2m: the antipode has two shortest paths, one on each side
    n_, s, d, _ = sg.cycle(2 * m)
    got = obc(2 * m, s, d, [0], L)
    for v in range(1, 2 * m):
        i = min(v, 2 * m - v)
        want = 0.0 if i == m else (m - 1 - i) + 0.5
        assert abs(got[v] - want) < 1e-12, (v, got[v], want)
    # K_{a,b} from a vertex of the a-side: the other a-1 vertices of that side
    # are two hops away through any of the b vertices
    a, b = 4, 3
    n_, s, d, _ = sg.bipartite(a, b)
    got = obc(a + b, s, d, [0], L)
    assert np.allclose(got[:a], 0.0) and np.allclose(got[a:], (a - 1) / b)


def dependency_identity_ok(L, n, s, d, sources, directed=False) -> bool:
    """One source's raw scores add up to sum over reached t of (dist - 1)."""
    A = oracle.Adjacency(n, np.asarray(s, np.int32), np.asarray(d, np.int32), _lib=L,
                         directed=directed)
    for src in sources:
        dep = A.bc([int(src)], normalise=False)
        depth = A.bfs(int(src))[0]
        want = float(np.sum(depth[depth > 0] - 1))
        if abs(dep.sum() - want) > 1e-9 * max(1.0, want):
            return False
        if dep[src] != 0.0 or np.any(dep[depth < 0] != 0.0) or np.any(dep < 0):
            return False
    return True


def test_dependency_sum_identity_rmat(oracle_lib):
    from paper_1508_03619_amd import inputs
    el = inputs.rmat(12, 16, seed=62)
    assert dependency_identity_ok(oracle_lib, el.n, el.src, el.dst, inputs.pick_sources(el, 4, seed=63))
    assert dependency_identity_ok(oracle_lib, el.n, el.src, el.dst,
                                  inputs.pick_sources(el, 4, seed=64, directed=True), directed=True)
    g = inputs.grid(40, 30, seed=65)
    assert dependency_identity_ok(oracle_lib, g.n, g.src, g.dst, inputs.pick_sources(g, 2, seed=66))


def test_additivity_repeats_and_normalisation(oracle_lib):
    from paper_1508_03619_amd import inputs
    el = inputs.rmat(10, 8, seed=67)
    A = oracle.Adjacency(el.n, el.src, el.dst, _lib=oracle_lib)
    a, b = [int(x) for x in inputs.pick_sources(el, 2, seed=68)]
    ra, rb, rab = A.bc([a], False), A.bc([b], False), A.bc([a, b], False)
    assert close(rab, ra + rb)
    assert close(A.bc([a, a], False), 2 * ra)
    nab = A.bc([a, b])
    assert nab.max() == 1.0 and close(nab, rab / rab.max())
    # isolated source: no paths, every score zero (normalisation leaves zeros)
    n_, s, d, _ = sg.disjoint_union(sg.path(3), sg.path(1))
    z = obc(4, s, d, [3], oracle_lib, normalise=True)
    assert z.tolist() == [0.0] * 4


# ---- pin function for the mutation tests ----------------------------------

def bc_pins_ok(L) -> bool:
    try:
        for k, srcs in ((4, [0]), (4, [1, 3])):
            pairs = list(itertools.combinations(range(k), 2))
            for mask in range(1 << len(pairs)):
                sel = [pairs[b] for b in range(len(pairs)) if (mask >> b) & 1]
                s = [p[0] for p in sel]
                d = [p[1] for p in sel]
                ref = definition_bc(k, s, d, srcs)
                if not close(obc(k, s, d, srcs, L), [float(x) for x in ref]):
                    return False
        n_, s, d, _ = sg.cycle(10)
        if not close(obc(10, s, d, [0], L), [0, 3.5, 2.5, 1.5, 0.5, 0, 0.5, 1.5, 2.5, 3.5]):
            return False
        n_, s, d, _ = sg.path(6)
        got = obc(6, s, d, [0, 2], L, normalise=True)
        if not close(got, np.array([0, 5, 3, 4, 2, 0]) / 5.0):
            return False
        from paper_1508_03619_amd import inputs
        el = inputs.rmat(9, 8, seed=69)
        return dependency_identity_ok(L, el.n, el.src, el.dst, inputs.pick_sources(el, 2, seed=70))
    except Exception:
        return False


def test_bc_pin_function_passes(oracle_lib):
    assert bc_pins_ok(oracle_lib)
