"""Directed graphs on the device against the directed oracle.

Section 2.1 allows directed edges (the paper's Twitter, Web and Road inputs
are directed): a search follows edges from tail to head, parent[v] = u needs
the edge u -> v, and the bottom-up step of Section 3 reads in-neighbours.
The handle keeps out-lists and in-lists; both are compared with the
oracle's lists, and every schedule (top-down only, bottom-up forced,
direction-optimizing; persistent, level-by-level and captured) is checked
on exhaustive tiny graphs, closed forms, random graphs with repeats and
self-loops, and R-MAT taken as directed."""
import numpy as np
import pytest

import oracle
from tests import smallgraphs as sg
from tests.gpuutil import assert_valid, device_bfs, say

pytestmark = pytest.mark.gpu

SCHEDULES = [dict(mode=m, direction=d) for m in (0, 1, 2) for d in (0, 1, 2)] + \
    [dict(mode=0, direction=d, small_frontier=sf) for d in (0, 1) for sf in (0, 1 << 30)] + \
    [dict(mode=0, direction=d, lds_bitmap=0) for d in (0, 2)] + \
    [dict(mode=0, alpha=1, beta=1), dict(mode=0, hub_degree=1, chunk_edges=64)]


def dpair(gb, n, src, dst):
    src = np.asarray(src, np.int32)
    dst = np.asarray(dst, np.int32)
    return (gb.build_csr(n, src, dst, directed=True),
            oracle.Adjacency(n, src, dst, directed=True))


def test_directed_csr_matches_oracle(gpu):
    from paper_1508_03619_amd import inputs
    for el in (inputs.rmat(12, 16, seed=41), inputs.urand(3000, 20000, seed=42),
               inputs.grid(30, 20, seed=43)):
        say(f"directed csr {el.name}")
        g = gpu.build_csr(el.n, el.src, el.dst, directed=True)
        assert g.directed
        out_ref = oracle.Adjacency(el.n, el.src, el.dst, directed=True)
        in_ref = oracle.Adjacency(el.n, el.dst, el.src, directed=True)
        rp, col = g.export()
        assert np.array_equal(rp, out_ref.offsets) and np.array_equal(col, out_ref.adj)
        rp, col = g.export_in()
        assert np.array_equal(rp, in_ref.offsets) and np.array_equal(col, in_ref.adj)
        assert g.nnz == len(out_ref.adj)
        g.free()
    # an undirected handle reports the same lists both ways
    el = inputs.rmat(10, 8, seed=44)
    g = gpu.build_csr(el.n, el.src, el.dst)
    assert not g.directed
    a, b = g.export(), g.export_in()
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
    g.free()


def test_exhaustive_three_vertex_digraphs(gpu):
    """All 64 directed graphs on 3 vertices, every source, every schedule."""
    k = 3
    offd = [(i, j) for i in range(k) for j in range(k) if i != j]
    say("exhaustive k=3 digraphs")
    for mask in range(1 << len(offd)):
        sel = [offd[b] for b in range(len(offd)) if (mask >> b) & 1]
        s = [p[0] for p in sel]
        d = [p[1] for p in sel]
        g, A = dpair(gpu, k, s, d)
        for src in range(k):
            ref = A.bfs(src)[0]
            for sch in SCHEDULES:
                parent, depth = device_bfs(gpu, g, src, params=sch)
                assert_valid(A, src, parent, depth, ref, what=f"mask {mask} {sch}")
        g.free()


def test_directed_closed_forms(gpu):
    for k in (9, 65, 130):
        say(f"directed closed forms k={k}")
        cases = {
            "path": (range(k - 1), range(1, k)),
            "cycle": (range(k), [(v + 1) % k for v in range(k)]),
            "out-star": ([0] * (k - 1), range(1, k)),
            "in-star": (range(1, k), [0] * (k - 1)),
        }
        for name, (s, d) in cases.items():
            g, A = dpair(gpu, k, list(s), list(d))
            for src in sorted({0, 1, k // 2, k - 1}):
                ref = A.bfs(src)[0]
                if name == "path":
                    assert ref.tolist() == [v - src if v >= src else -1 for v in range(k)]
                for sch in SCHEDULES:
                    parent, depth = device_bfs(gpu, g, src, params=sch)
                    assert_valid(A, src, parent, depth, ref, what=f"{name} k={k} {sch}")
            g.free()


def test_random_digraphs_with_repeats_and_self_loops(gpu):
    for seed in range(30):
        rng = np.random.default_rng(5000 + seed)
        n = int(rng.integers(1, 400))
        m = int(rng.integers(0, 5 * n + 1))
        s = rng.integers(0, n, m).astype(np.int32)
        d = rng.integers(0, n, m).astype(np.int32)
        if m:
            s = np.concatenate([s, s[: m // 5 + 1], d[: m // 7 + 1]]).astype(np.int32)
            d = np.concatenate([d, d[: m // 5 + 1], d[: m // 7 + 1]]).astype(np.int32)
        g, A = dpair(gpu, n, s, d)
        say(f"random digraph seed={seed} n={n} m={len(s)}")
        for src in sorted({0, n - 1, int(rng.integers(0, n))}):
            ref = A.bfs(src)[0]
            for sch in SCHEDULES:
                parent, depth = device_bfs(gpu, g, src, params=sch)
                assert_valid(A, src, parent, depth, ref, what=f"seed {seed} {sch}")
        g.free()


def test_symmetric_digraph_equals_undirected(gpu):
    """Both directions of every pair as directed edges give the undirected
    graph: the same lists and the same depths."""
    from paper_1508_03619_amd import inputs
    el = inputs.rmat(13, 16, seed=45)
    s2 = np.concatenate([el.src, el.dst])
    d2 = np.concatenate([el.dst, el.src])
    gd = gpu.build_csr(el.n, s2, d2, directed=True)
    gu = gpu.build_csr(el.n, el.src, el.dst)
    assert np.array_equal(gd.export()[1], gu.export()[1])
    A = oracle.Adjacency(el.n, el.src, el.dst)
    for src in inputs.pick_sources(el, 4, seed=46):
        ref = A.bfs(int(src))[0]
        for sch in (dict(mode=0), dict(mode=0, direction=2), dict(mode=2)):
            pd, dd = device_bfs(gpu, gd, int(src), params=sch)
            assert np.array_equal(dd, ref)
            assert_valid(A, int(src), pd, dd, ref, what=f"symmetric digraph {sch}")
    gd.free()
    gu.free()


@pytest.mark.parametrize("name", ["rmat16d"])
def test_rmat_directed_sources(gpu, name):
    """R-MAT scale 16 taken as directed (skewed in- and out-degrees): 32
    sources with out-edges, default schedule, plus a few forced schedules."""
    from paper_1508_03619_amd import inputs
    el = inputs.workload(name)
    srcs = [int(x) for x in inputs.pick_sources(el, 32, seed=inputs.SOURCE_SEEDS[name], directed=True)]
    g, A = dpair(gpu, el.n, el.src, el.dst)
    for i, src in enumerate(srcs):
        if i % 8 == 0:
            say(f"{name} source {i}")
        ref = A.bfs(src)[0]
        parent, depth = device_bfs(gpu, g, src)
        assert_valid(A, src, parent, depth, ref, what=name)
        if i < 4:
            for sch in SCHEDULES:
                parent, depth = device_bfs(gpu, g, src, params=sch)
                assert_valid(A, src, parent, depth, ref, what=f"{name} {sch}")
    g.free()


def test_batch_rejects_directed(gpu):
    import torch
    g, _ = dpair(gpu, 4, [0, 1], [1, 2])
    p = torch.empty(4, dtype=torch.int32, device="cuda")
    with pytest.raises(gpu.GapError, match="directed"):
        gpu.bfs_batch([g], [0], [0], [p], [None])
    g.free()
