"""Betweenness centrality on the device against the oracle (Section 2.1).

Tolerance: both sides sum positive terms in fp64 in different orders; with
at most D levels and lists of at most Delta entries the relative error of a
score is below about (2 D + log2 Delta) * 2^-53 per source, far under 1e-9
for every graph here.  A score passes when |gpu - oracle| <= 1e-9 |oracle| +
1e-12 max|oracle|.  Raw sums and normalised scores are both checked, on
exhaustive tiny graphs, closed forms, random graphs with repeats and
self-loops (directed and not), depths beyond the LDS-binned range, R-MAT
with long lists (several chunk items per vertex), and the identity that one
source's raw scores sum to the total of (distance - 1) over the vertices it
reaches."""
import itertools

import numpy as np
import pytest

import oracle
from tests import smallgraphs as sg
from tests.gpuutil import say

pytestmark = pytest.mark.gpu


def gpu_bc(gb, g, sources, normalise=True):
    import torch
    out = torch.empty(g.n, dtype=torch.float64, device="cuda")
    gb.bc(g, [int(s) for s in sources], out, normalise=normalise)
    torch.cuda.synchronize()
    return out.cpu().numpy()


def assert_close(got, ref, what=""):
    ref = np.asarray(ref, np.float64)
    tol = 1e-9 * np.abs(ref) + 1e-12 * max(float(np.abs(ref).max(initial=0.0)), 1e-300)
    bad = np.nonzero(~(np.abs(got - ref) <= tol))[0]
    assert bad.size == 0, (f"{what}: {bad.size} scores differ, first v={bad[0]} "
                           f"gpu={got[bad[0]]!r} oracle={ref[bad[0]]!r}")


def pair(gb, n, s, d, directed=False):
    s = np.asarray(s, np.int32)
    d = np.asarray(d, np.int32)
    return gb.build_csr(n, s, d, directed=directed), oracle.Adjacency(n, s, d, directed=directed)


def test_all_four_vertex_graphs(gpu):
    k = 4
    pairs = list(itertools.combinations(range(k), 2))
    say("bc: all 4-vertex graphs")
    for mask in range(1 << len(pairs)):
        sel = [pairs[b] for b in range(len(pairs)) if (mask >> b) & 1]
        g, A = pair(gpu, k, [p[0] for p in sel], [p[1] for p in sel])
        for srcs in ([0], [1, 3], [0, 1, 2, 3], [2, 2]):
            assert_close(gpu_bc(gpu, g, srcs, False), A.bc(srcs, False), f"mask {mask} {srcs}")
            assert_close(gpu_bc(gpu, g, srcs), A.bc(srcs), f"mask {mask} {srcs} normalised")
        g.free()


def test_all_three_vertex_digraphs(gpu):
    k = 3
    offd = [(i, j) for i in range(k) for j in range(k) if i != j]
    say("bc: all 3-vertex digraphs")
    for mask in range(1 << len(offd)):
        sel = [offd[b] for b in range(len(offd)) if (mask >> b) & 1]
        g, A = pair(gpu, k, [p[0] for p in sel], [p[1] for p in sel], directed=True)
        for srcs in ([0], [2, 1]):
            assert_close(gpu_bc(gpu, g, srcs, False), A.bc(srcs, False), f"mask {mask} {srcs}")
        g.free()


def test_closed_forms_and_deep_levels(gpu):
    # path of 3000 vertices: depths beyond the LDS bins; raw scores n-1-i
    for name, (n, s, d, _) in [("path3000", sg.path(3000)), ("cycle1001", sg.cycle(1001)),
                               ("cycle1000", sg.cycle(1000)), ("star200", sg.star(200)),
                               ("K30", sg.complete(30)), ("K5,70", sg.bipartite(5, 70)),
                               ("grid60x40", sg.full_grid(60, 40))]:
        say(f"bc: {name}")
        g, A = pair(gpu, n, s, d)
        for srcs in ([0], [n - 1, n // 2, 1]):
            assert_close(gpu_bc(gpu, g, srcs, False), A.bc(srcs, False), f"{name} {srcs}")
        if name == "path3000":
            got = gpu_bc(gpu, g, [0], False)
            assert np.array_equal(got, np.array([0.0] + [float(n - 1 - i) for i in range(1, n - 1)] + [0.0]))
        g.free()


def test_random_graphs_with_repeats_and_self_loops(gpu):
    for seed in range(30):
        rng = np.random.default_rng(7000 + seed)
        n = int(rng.integers(1, 300))
        m = int(rng.integers(0, 4 * n + 1))
        s = rng.integers(0, n, m).astype(np.int32)
        d = rng.integers(0, n, m).astype(np.int32)
        if m:
            s = np.concatenate([s, s[: m // 5 + 1], d[: 3]]).astype(np.int32)
            d = np.concatenate([d, d[: m // 5 + 1], d[: 3]]).astype(np.int32)
        directed = bool(seed % 2)
        g, A = pair(gpu, n, s, d, directed)
        srcs = [int(x) for x in rng.integers(0, n, 4)]
        say(f"bc: random seed={seed} n={n} directed={directed}")
        assert_close(gpu_bc(gpu, g, srcs, False), A.bc(srcs, False), f"seed {seed}")
        assert_close(gpu_bc(gpu, g, srcs), A.bc(srcs), f"seed {seed} normalised")
        g.free()


def test_edge_cases(gpu):
    say("bc: edge cases")
    g, A = pair(gpu, 1, [], [])
    assert gpu_bc(gpu, g, [0]).tolist() == [0.0]
    # isolated source among edges: every score zero, also after normalising
    n, s, d, _ = sg.disjoint_union(sg.path(5), sg.path(1), sg.cycle(6))
    g, A = pair(gpu, n, s, d)
    assert gpu_bc(gpu, g, [5]).tolist() == [0.0] * n
    assert_close(gpu_bc(gpu, g, [5, 0, 8], False), A.bc([5, 0, 8], False), "union")
    with pytest.raises(gpu.GapError):
        gpu_bc(gpu, g, [])
    with pytest.raises(gpu.GapError):
        gpu_bc(gpu, g, [n])


@pytest.mark.parametrize("directed", [False, True])
def test_rmat16_four_sources(gpu, directed):
    """R-MAT scale 16 (hubs with hundreds to thousands of entries: several
    chunk items each), four sources as the benchmark uses."""
    from paper_1508_03619_amd import inputs
    name = "rmat16d" if directed else "rmat16"
    el = inputs.workload(name)
    g, A = pair(gpu, el.n, el.src, el.dst, directed)
    srcs = [int(x) for x in inputs.pick_sources(el, 4, seed=inputs.SOURCE_SEEDS[name] + 7,
                                                directed=directed)]
    say(f"bc: {name} sources {srcs}")
    assert_close(gpu_bc(gpu, g, srcs), A.bc(srcs), name)
    for src in srcs[:2]:
        raw = gpu_bc(gpu, g, [src], False)
        assert_close(raw, A.bc([src], False), f"{name} raw {src}")
        depth = A.bfs(src)[0]
        want = float(np.sum(depth[depth > 0] - 1))
        assert abs(raw.sum() - want) <= 1e-9 * want, (raw.sum(), want)
    g.free()


def test_two_calls_on_two_streams(gpu):
    import torch
    from paper_1508_03619_amd import inputs
    el = inputs.rmat(14, 16, seed=71)
    g, A = pair(gpu, el.n, el.src, el.dst)
    srcs = [[int(x) for x in inputs.pick_sources(el, 4, seed=72 + i)] for i in range(2)]
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    outs = [torch.empty(g.n, dtype=torch.float64, device="cuda") for _ in range(2)]
    say("bc: two streams")
    for st, o, ss in zip(streams, outs, srcs):
        gpu.bc(g, ss, o, stream=st)
    torch.cuda.synchronize()
    for o, ss in zip(outs, srcs):
        assert_close(o.cpu().numpy(), A.bc(ss), "two streams")
    g.free()
