"""Shortest paths on the device against the oracle (Section 2.1: distances
are unique, so they must match exactly; Section 2.2: weights 1..255).

Covers the weighted device CSR (a repeated pair keeps its smallest weight),
every 4-vertex graph and 3-vertex digraph under random small weights and
several bucket widths, closed forms over thousands of buckets, random
graphs with repeats and self-loops both ways, unit weights against the BFS
depths, R-MAT 16 both ways, a high-diameter grid, edge cases, argument
errors and two streams at once."""
import itertools

import numpy as np
import pytest

import oracle
from tests import smallgraphs as sg
from tests.gpuutil import say

pytestmark = pytest.mark.gpu

INF = 0xFFFFFFFF


def pair(gb, n, s, d, w, directed=False):
    s = np.asarray(s, np.int32)
    d = np.asarray(d, np.int32)
    w = np.asarray(w, np.int32)
    return (gb.build_csr(n, s, d, directed=directed, weights=w),
            oracle.WeightedAdjacency(n, s, d, w, directed=directed))


def gpu_sssp(gb, g, src, delta=0):
    import torch
    out = torch.empty(g.n, dtype=torch.int32, device="cuda")
    gb.sssp(g, int(src), out, delta=delta)
    torch.cuda.synchronize()
    return out.cpu().numpy().view(np.uint32).astype(np.int64)


def ref_of(A, src):
    d = A.sssp(int(src))
    return np.where(d < 0, INF, d)


def check(gb, g, A, src, delta=0, what=""):
    got = gpu_sssp(gb, g, src, delta)
    ref = ref_of(A, src)
    bad = np.nonzero(got != ref)[0]
    assert bad.size == 0, f"{what} src={src} delta={delta}: {bad.size} differ, v={bad[0]} gpu={got[bad[0]]} ref={ref[bad[0]]}"


def test_weighted_csr_matches_oracle(gpu):
    from paper_1508_03619_amd import inputs
    for directed in (False, True):
        el = inputs.rmat(12, 16, seed=101)
        w = inputs.weights(el, seed=102, directed=directed)
        # repeated pairs with other weights: the smallest must win
        s = np.concatenate([el.src, el.src[:500]])
        d = np.concatenate([el.dst, el.dst[:500]])
        w = np.concatenate([w, np.maximum(1, w[:500] - 7)]).astype(np.int32)
        say(f"weighted csr directed={directed}")
        g, A = pair(gpu, el.n, s, d, w, directed)
        rp, col = g.export()
        assert np.array_equal(rp, A.offsets) and np.array_equal(col, A.adj)
        assert np.array_equal(g.export_weights(), A.wadj)
        g.free()


@pytest.mark.parametrize("delta", [1, 2, 1000])
def test_all_four_vertex_graphs(gpu, delta):
    k = 4
    pairs = list(itertools.combinations(range(k), 2))
    rng = np.random.default_rng(103)
    say(f"sssp: all 4-vertex graphs delta={delta}")
    for mask in range(1 << len(pairs)):
        sel = [pairs[b] for b in range(len(pairs)) if (mask >> b) & 1]
        w = rng.integers(1, 4, len(sel))
        g, A = pair(gpu, k, [p[0] for p in sel], [p[1] for p in sel], w)
        for src in range(k):
            check(gpu, g, A, src, delta, f"mask {mask}")
        g.free()


def test_all_three_vertex_digraphs(gpu):
    k = 3
    offd = [(i, j) for i in range(k) for j in range(k) if i != j]
    rng = np.random.default_rng(104)
    say("sssp: all 3-vertex digraphs")
    for mask in range(1 << len(offd)):
        sel = [offd[b] for b in range(len(offd)) if (mask >> b) & 1]
        w = rng.integers(1, 5, len(sel))
        g, A = pair(gpu, k, [p[0] for p in sel], [p[1] for p in sel], w, directed=True)
        for src in range(k):
            for delta in (1, 3):
                check(gpu, g, A, src, delta, f"mask {mask}")
        g.free()


def test_closed_forms_many_buckets(gpu):
    rng = np.random.default_rng(105)
    for name, (n, s, d, _) in [("path3000", sg.path(3000)), ("cycle1001", sg.cycle(1001)),
                               ("star300", sg.star(300)), ("grid60x40", sg.full_grid(60, 40)),
                               ("K40", sg.complete(40))]:
        w = rng.integers(1, 256, len(s)).astype(np.int32)
        say(f"sssp: {name}")
        g, A = pair(gpu, n, s, d, w)
        for src in sorted({0, n // 2, n - 1}):
            for delta in (0, 1, 50, 1 << 20):
                check(gpu, g, A, src, delta, name)
        if name == "path3000":
            got = gpu_sssp(gpu, g, 0, 16)
            assert got.tolist() == np.concatenate([[0], np.cumsum(w)]).tolist()
        g.free()


def test_random_graphs_with_repeats_and_self_loops(gpu):
    for seed in range(30):
        rng = np.random.default_rng(106 + seed)
        n = int(rng.integers(1, 400))
        m = int(rng.integers(0, 5 * n + 1))
        s = rng.integers(0, n, m).astype(np.int32)
        d = rng.integers(0, n, m).astype(np.int32)
        w = rng.integers(1, 256, m).astype(np.int32)
        if m:
            s = np.concatenate([s, s[: m // 4 + 1], d[:3]]).astype(np.int32)
            d = np.concatenate([d, d[: m // 4 + 1], d[:3]]).astype(np.int32)
            w = np.concatenate([w, rng.integers(1, 256, m // 4 + 1 + min(3, m))]).astype(np.int32)
        directed = bool(seed % 2)
        g, A = pair(gpu, n, s, d, w, directed)
        say(f"sssp: random seed={seed} n={n} directed={directed}")
        for src in sorted({0, n - 1, int(rng.integers(0, n))}):
            for delta in (0, 1, 7, 300):
                check(gpu, g, A, src, delta, f"seed {seed}")
        g.free()


def test_unweighted_graph_gives_bfs_depths(gpu):
    from paper_1508_03619_amd import inputs
    el = inputs.rmat(14, 16, seed=107)
    g = gpu.build_csr(el.n, el.src, el.dst)
    B = oracle.Adjacency(el.n, el.src, el.dst)
    for src in inputs.pick_sources(el, 4, seed=108):
        ref = B.bfs(int(src))[0].astype(np.int64)
        ref = np.where(ref < 0, INF, ref)
        for delta in (0, 1, 4):
            assert np.array_equal(gpu_sssp(gpu, g, src, delta), ref)
    g.free()


@pytest.mark.parametrize("directed", [False, True])
def test_rmat16_sources(gpu, directed):
    from paper_1508_03619_amd import inputs
    name = "rmat16d" if directed else "rmat16"
    el = inputs.workload(name)
    w = inputs.weights(el, seed=inputs.WEIGHT_SEEDS[name], directed=directed)
    g, A = pair(gpu, el.n, el.src, el.dst, w, directed)
    srcs = inputs.pick_sources(el, 16, seed=inputs.SOURCE_SEEDS[name] + 11, directed=directed)
    say(f"sssp: {name} 16 sources")
    for i, src in enumerate(srcs):
        for delta in ((0, 16, 256) if i < 3 else (0,)):
            check(gpu, g, A, int(src), delta, name)
    g.free()


def test_grid_high_diameter(gpu):
    from paper_1508_03619_amd import inputs
    el = inputs.grid(300, 300, seed=109)
    w = inputs.weights(el, seed=110)
    g, A = pair(gpu, el.n, el.src, el.dst, w)
    say("sssp: grid 300x300")
    for src in inputs.pick_sources(el, 2, seed=111):
        for delta in (0, 32, 1024):
            check(gpu, g, A, int(src), delta, "grid300")
    g.free()


def test_edge_cases_and_errors(gpu):
    import torch
    say("sssp: edge cases")
    g, A = pair(gpu, 1, [], [], [])
    assert gpu_sssp(gpu, g, 0).tolist() == [0]
    n, s, d, _ = sg.disjoint_union(sg.path(5), sg.path(1), sg.cycle(6))
    w = np.arange(1, len(s) + 1, dtype=np.int32)
    g, A = pair(gpu, n, s, d, w)
    assert gpu_sssp(gpu, g, 5).tolist() == [INF] * 5 + [0] + [INF] * 6
    check(gpu, g, A, 0, 0, "union")
    out = torch.empty(n, dtype=torch.int32, device="cuda")
    with pytest.raises(gpu.GapError):
        gpu.sssp(g, n, out)
    with pytest.raises(gpu.GapError):
        gpu.build_csr(3, np.array([0], np.int32), np.array([1], np.int32), weights=np.array([0], np.int32))
    # (n - 1) * max weight must stay below 2^32 - 1
    big = gpu.build_csr(5, np.array([0, 1], np.int32), np.array([1, 2], np.int32),
                        weights=np.array([1 << 30, 1], np.int32))
    with pytest.raises(gpu.GapError, match="2\\^32"):
        gpu.sssp(big, 0, torch.empty(5, dtype=torch.int32, device="cuda"))


def test_two_streams_concurrently(gpu):
    import torch
    from paper_1508_03619_amd import inputs
    el = inputs.rmat(14, 16, seed=112)
    w = inputs.weights(el, seed=113)
    g, A = pair(gpu, el.n, el.src, el.dst, w)
    srcs = [int(x) for x in inputs.pick_sources(el, 2, seed=114)]
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    outs = [torch.empty(g.n, dtype=torch.int32, device="cuda") for _ in range(2)]
    say("sssp: two streams")
    for st, o, s in zip(streams, outs, srcs):
        gpu.sssp(g, s, o, stream=st)
    torch.cuda.synchronize()
    for o, s in zip(outs, srcs):
        assert np.array_equal(o.cpu().numpy().view(np.uint32).astype(np.int64), ref_of(A, s))
    g.free()
