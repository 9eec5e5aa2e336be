"""Multi-source (batched) parity: every lane equals the single-source
definition for its (graph, source) -- depths bit-exact against the CPU
oracle, parents valid (Section 2.1)."""
import numpy as np
import pytest

import oracle
from tests import smallgraphs as sg
from tests.gpuutil import assert_valid, say

pytestmark = pytest.mark.gpu


def run_batch(gb, graphs, gos, srcs, with_depth=True):
    import torch
    parents = [torch.full((graphs[g].n,), -7, dtype=torch.int32, device="cuda") for g in gos]
    depths = ([torch.full((graphs[g].n,), -7, dtype=torch.int32, device="cuda") for g in gos]
              if with_depth else None)
    gb.bfs_batch(graphs, list(gos), list(srcs), parents, depths)
    torch.cuda.synchronize()
    return ([p.cpu().numpy() for p in parents],
            [d.cpu().numpy() for d in depths] if with_depth else None)


def check_lanes(adjs, gos, srcs, parents, depths, what=""):
    refs = {}
    for i, (g, s) in enumerate(zip(gos, srcs)):
        key = (g, int(s))
        if key not in refs:
            refs[key] = adjs[g].bfs(int(s))[0]
        assert_valid(adjs[g], int(s), parents[i], depths[i] if depths is not None else None,
                     refs[key], what=f"{what} lane {i} graph {g}")


def test_batch_small_graphs_all_sources(gpu):
    for name, n, s, d in [("petersen",) + tuple(sg.read_golden()[0][1:4])] + \
            [("grid9x7",) + sg.full_grid(9, 7)[:3], ("union",) + sg.disjoint_union(
                sg.path(5), sg.cycle(9), sg.path(1), sg.star(6))[:3]]:
        say(f"batch small {name}")
        g = gpu.build_csr(n, s, d)
        A = oracle.Adjacency(n, s, d)
        srcs = list(range(n))
        P, D = run_batch(gpu, [g], [0] * n, srcs)
        check_lanes([A], [0] * n, srcs, P, D, name)


@pytest.mark.parametrize("nlanes", [1, 37, 64, 100, 256, 300])
def test_batch_lane_counts(gpu, nlanes):
    from paper_1508_03619_amd import inputs
    el = inputs.rmat(13, 16, seed=61)
    g = gpu.build_csr(el.n, el.src, el.dst)
    A = oracle.Adjacency(el.n, el.src, el.dst)
    rng = np.random.default_rng(nlanes)
    srcs = rng.integers(0, el.n, nlanes)  # includes isolated vertices and repeats
    say(f"batch lanes={nlanes}")
    P, D = run_batch(gpu, [g], [0] * nlanes, srcs)
    check_lanes([A], [0] * nlanes, srcs, P, D, f"lanes={nlanes}")


def test_batch_duplicate_sources(gpu):
    from paper_1508_03619_amd import inputs
    el = inputs.rmat(12, 16, seed=71)
    g = gpu.build_csr(el.n, el.src, el.dst)
    A = oracle.Adjacency(el.n, el.src, el.dst)
    s0 = int(inputs.pick_sources(el, 1, seed=72)[0])
    srcs = [s0] * 10 + [s0 ^ 1] * 5
    P, D = run_batch(gpu, [g], [0] * len(srcs), srcs)
    check_lanes([A], [0] * len(srcs), srcs, P, D, "dups")
    for i in range(1, 10):
        assert np.array_equal(D[i], D[0])


def test_batch_mixed_graphs_one_launch(gpu):
    from paper_1508_03619_amd import inputs
    els = [inputs.rmat(10, 16, seed=81), inputs.rmat(12, 8, seed=82), inputs.grid(50, 40, seed=83),
           inputs.urand(3000, 24000, seed=84), inputs.rmat(11, 16, seed=85)]
    n0, s0, d0, _ = sg.path(70)
    graphs = [gpu.build_csr(e.n, e.src, e.dst) for e in els] + [gpu.build_csr(n0, s0, d0)]
    adjs = [oracle.Adjacency(e.n, e.src, e.dst) for e in els] + [oracle.Adjacency(n0, s0, d0)]
    gos, srcs = [], []
    rng = np.random.default_rng(5)
    for gi, A in enumerate(adjs):
        k = [9, 64, 3, 20, 1, 5][gi]
        for s in rng.integers(0, A.n, k):
            gos.append(gi)
            srcs.append(int(s))
    perm = rng.permutation(len(gos))  # lanes of one graph need not be adjacent
    gos = [gos[i] for i in perm]
    srcs = [srcs[i] for i in perm]
    say(f"mixed batch: {len(gos)} lanes over {len(graphs)} graphs")
    P, D = run_batch(gpu, graphs, gos, srcs)
    check_lanes(adjs, gos, srcs, P, D, "mixed")


def test_batch_without_depths(gpu):
    from paper_1508_03619_amd import inputs
    el = inputs.rmat(11, 16, seed=91)
    g = gpu.build_csr(el.n, el.src, el.dst)
    A = oracle.Adjacency(el.n, el.src, el.dst)
    srcs = [int(x) for x in inputs.pick_sources(el, 8, seed=92)]
    P, _ = run_batch(gpu, [g], [0] * 8, srcs, with_depth=False)
    for s, p in zip(srcs, P):
        ref = A.bfs(s)[0]
        assert A.check(s, ref, p)[0] == 0


def test_batch_rmat16_64_sources_matches_single(gpu):
    """R-MAT 16 with the 64 trial sources in one launch; each lane equals the
    single-source search of the same source on depth."""
    import torch
    from paper_1508_03619_amd import inputs
    el = inputs.workload("rmat16")
    srcs = [int(x) for x in inputs.pick_sources(el, 64, seed=inputs.SOURCE_SEEDS["rmat16"])]
    g = gpu.build_csr(el.n, el.src, el.dst)
    A = oracle.Adjacency(el.n, el.src, el.dst)
    say("rmat16 batch of 64")
    P, D = run_batch(gpu, [g], [0] * 64, srcs)
    check_lanes([A], [0] * 64, srcs, P, D, "rmat16")
    p1 = torch.empty(g.n, dtype=torch.int32, device="cuda")
    d1 = torch.empty(g.n, dtype=torch.int32, device="cuda")
    for i in (0, 31, 63):
        gpu.bfs(g, srcs[i], p1, d1)
        torch.cuda.synchronize()
        assert np.array_equal(d1.cpu().numpy(), D[i])


def test_batch_grid_high_diameter(gpu):
    from paper_1508_03619_amd import inputs
    el = inputs.grid(120, 90, seed=93)
    g = gpu.build_csr(el.n, el.src, el.dst)
    A = oracle.Adjacency(el.n, el.src, el.dst)
    srcs = [int(x) for x in inputs.pick_sources(el, 70, seed=94)]
    say("grid batch of 70")
    P, D = run_batch(gpu, [g], [0] * 70, srcs)
    check_lanes([A], [0] * 70, srcs, P, D, "grid")


def test_batch_level_records(gpu):
    """gap_bfs_batch_ex: results as without records; one record per level
    the batch ran; level 0's frontier is the set of distinct sources and each
    level's claimed count is the next level's frontier; the records agree
    with the lanes' oracle depths (frontier of level d = vertices some lane
    reaches at depth d)."""
    import torch
    from paper_1508_03619_amd import gapbfs as gb, inputs
    el = inputs.rmat(13, 16, seed=7301)
    g = gb.build_csr(el.n, el.src, el.dst)
    A = oracle.Adjacency(el.n, el.src, el.dst)
    srcs = [int(x) for x in inputs.pick_sources(el, 40, seed=7302)]
    srcs += srcs[:3]  # repeated sources are separate lanes
    P = [torch.empty(g.n, dtype=torch.int32, device="cuda") for _ in srcs]
    D = [torch.empty(g.n, dtype=torch.int32, device="cuda") for _ in srcs]
    recs = gb.bfs_batch([g], [0] * len(srcs), srcs, P, D, stats=True)
    torch.cuda.synchronize()
    depths = np.stack([A.bfs(s)[0] for s in srcs])
    for i, s in enumerate(srcs):
        assert_valid(A, s, P[i].cpu().numpy(), D[i].cpu().numpy(), depths[i], what=f"lane {i}")
    maxd = int(depths.max())
    assert len(recs) == maxd + 1  # levels 0..maxd expand a non-empty frontier
    deg = np.diff(A.offsets)
    for r in recs:
        d = r["level"]
        front = np.any(depths == d, axis=0)
        assert r["frontier"] == int(front.sum()), r
        assert r["frontier_edges"] == int(deg[front].sum()), r
        assert r["direction"] in (1, 2)
        if r["direction"] == 2:  # every vertex found was searched for, and read an entry
            assert r["claimed"] <= r["unvisited"] <= r["scanned"], r
    assert recs[0]["frontier"] == len(set(srcs))
    for a, b in zip(recs, recs[1:]):
        assert a["claimed"] == b["frontier"]
    g.free()
