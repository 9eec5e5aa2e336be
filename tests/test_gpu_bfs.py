"""Single-source parity on the device: depths bit-exact against the CPU
oracle, parents valid by the definition (Section 2.1), through the C ABI."""
import itertools

import numpy as np
import pytest

import oracle
from tests import smallgraphs as sg
from tests.gpuutil import assert_valid, device_bfs, graph_pair, say

pytestmark = pytest.mark.gpu

SCHEDULES = [dict(mode=m, direction=d) for m in (0, 1, 2) for d in (0, 1, 2)] + \
    [dict(mode=0, direction=d, small_frontier=sf) for d in (0, 1) for sf in (0, 1 << 30)] + \
    [dict(mode=0, direction=d, lds_bitmap=0) for d in (0, 2)] + \
    [dict(mode=0, direction=d, bu_mapping=1) for d in (0, 2)] + \
    [dict(mode=0, direction=d, td_plain=1 << 30, small_frontier=0) for d in (0, 1)] + \
    [dict(mode=0, direction=0, td_plain=0), dict(mode=0, direction=0, coop_launch=1)]


def small_cases():
    cases = [(name, n, s, d) for name, n, s, d, _ in sg.read_golden()]
    for name, mk in [("path33", lambda: sg.path(33)), ("cycle70", lambda: sg.cycle(70)),
                     ("star130", lambda: sg.star(130)), ("K12", lambda: sg.complete(12)),
                     ("K5,70", lambda: sg.bipartite(5, 70)), ("Q7", lambda: sg.hypercube(7)),
                     ("grid13x11", lambda: sg.full_grid(13, 11)),
                     ("union", lambda: sg.disjoint_union(sg.path(5), sg.cycle(65), sg.path(1), sg.star(3)))]:
        n, s, d, _ = mk()
        cases.append((name, n, s, d))
    return cases


def test_golden_depths_on_device(gpu):
    for name, n, s, d, cases in sg.read_golden():
        say(f"golden {name}")
        g = gpu.build_csr(n, s, d)
        for src, want in cases:
            for sch in SCHEDULES:
                parent, depth = device_bfs(gpu, g, src, params=sch)
                assert np.array_equal(depth, want), (name, src, sch)
        g.free()


def test_small_graphs_all_sources_all_schedules(gpu):
    for name, n, s, d in small_cases():
        say(f"small {name} n={n}")
        g, A = graph_pair(gpu, n, s, d)
        for src in range(n):
            ref = A.bfs(src)[0]
            for sch in SCHEDULES:
                parent, depth = device_bfs(gpu, g, src, params=sch)
                assert_valid(A, src, parent, depth, ref, what=f"{name} {sch}")
        g.free()


def test_random_graphs_with_repeats_and_self_loops(gpu):
    for seed in range(40):
        rng = np.random.default_rng(1000 + seed)
        n = int(rng.integers(1, 300))
        m = int(rng.integers(0, 4 * n + 1))
        s = rng.integers(0, n, m).astype(np.int32)
        d = rng.integers(0, n, m).astype(np.int32)
        if m:
            s = np.concatenate([s, s[: m // 5 + 1], d[: m // 7 + 1]]).astype(np.int32)
            d = np.concatenate([d, d[: m // 5 + 1], d[: m // 7 + 1]]).astype(np.int32)
        say(f"random seed={seed} n={n} m={len(s)}")
        g, A = graph_pair(gpu, n, s, d)
        for src in rng.integers(0, n, 6):
            ref = A.bfs(int(src))[0]
            for sch in SCHEDULES:
                parent, depth = device_bfs(gpu, g, int(src), params=sch)
                assert_valid(A, int(src), parent, depth, ref, what=f"seed {seed} {sch}")
        g.free()


def test_csr_matches_oracle_adjacency(gpu):
    from paper_1508_03619_amd import inputs
    for el in (inputs.rmat(14, 16, seed=3), inputs.grid(40, 30, seed=5),
               inputs.urand(3000, 40000, seed=9)):
        say(f"csr {el.name}")
        g = gpu.build_csr(el.n, el.src, el.dst)
        A = oracle.Adjacency(el.n, el.src, el.dst)
        row_ptr, col = g.export()
        assert np.array_equal(row_ptr, A.offsets)
        assert np.array_equal(col, A.adj)
        g.free()


def test_edge_cases(gpu):
    say("edge cases")
    # one vertex, no edges
    g, A = graph_pair(gpu, 1, np.zeros(0, np.int32), np.zeros(0, np.int32))
    for sch in SCHEDULES:
        parent, depth = device_bfs(gpu, g, 0, params=sch)
        assert parent.tolist() == [0] and depth.tolist() == [0]
    # only self-loops
    g, A = graph_pair(gpu, 70, np.arange(70, dtype=np.int32), np.arange(70, dtype=np.int32))
    assert g.nnz == 0
    for sch in SCHEDULES:
        parent, depth = device_bfs(gpu, g, 69, params=sch)
        assert_valid(A, 69, parent, depth)
    # isolated source in a graph with edges, ragged n, source n-1
    for n in (63, 64, 65, 127, 129):
        s = np.arange(0, n - 3, dtype=np.int32)
        d = (s + 1).astype(np.int32)
        g, A = graph_pair(gpu, n, s, d)
        for src in (0, n - 3, n - 2, n - 1):
            for sch in SCHEDULES:
                parent, depth = device_bfs(gpu, g, src, params=sch)
                assert_valid(A, src, parent, depth, what=f"n={n} {sch}")
    # depth output omitted
    g, A = graph_pair(gpu, 100, np.arange(99, dtype=np.int32), np.arange(1, 100, dtype=np.int32))
    parent, _ = device_bfs(gpu, g, 50, with_depth=False)
    dref = A.bfs(50)[0]
    assert A.check(50, dref, parent)[0] == 0


def test_hub_splitting_and_tuning_invariance(gpu):
    """Every parameter setting gives the same depths (they are unique)."""
    from paper_1508_03619_amd import inputs
    el = inputs.rmat(14, 16, seed=21)
    g, A = graph_pair(gpu, el.n, el.src, el.dst)
    deg = np.diff(A.offsets)
    srcs = [int(np.argmax(deg))] + [int(x) for x in inputs.pick_sources(el, 3, seed=22)]
    settings = [dict(hub_degree=1, chunk_edges=64), dict(hub_degree=64, chunk_edges=64),
                dict(hub_degree=4096, chunk_edges=1024), dict(alpha=1, beta=1),
                dict(alpha=1000, beta=1000), dict(alpha=2, beta=200),
                dict(block=512), dict(block=1024), dict(block=256, blocks_per_cu=1),
                dict(block=1024, blocks_per_cu=1),
                # hub claims (listed per workgroup, and beyond the list's
                # capacity) in levels that switch direction often, so the
                # frontier bitmap is turned back into a queue with hubs in it
                dict(hub_degree=1, chunk_edges=64, alpha=2, beta=200),
                dict(hub_degree=8, chunk_edges=64, alpha=1, beta=1),
                # top-down claims by plain stores at every level (F_{d+1}
                # read back from the depths, queued again when top-down
                # follows), with hub chunk items in the input queues
                dict(td_plain=1 << 30, small_frontier=0),
                dict(td_plain=1 << 30, small_frontier=0, hub_degree=1, chunk_edges=64),
                dict(td_plain=1 << 30, small_frontier=0, alpha=2, beta=200), dict(td_plain=0)]
    for src in srcs:
        ref = A.bfs(src)[0]
        for st in settings:
            for mode in (0, 1, 2):
                say(f"tuning src={src} {st} mode={mode}")
                parent, depth = device_bfs(gpu, g, src, params=dict(st, mode=mode))
                assert_valid(A, src, parent, depth, ref, what=str(st))


def test_rmat16_64_sources(gpu):
    """R-MAT scale 16, edge factor 16, 64 seeded non-zero-degree sources."""
    from paper_1508_03619_amd import inputs
    el = inputs.workload("rmat16")
    srcs = inputs.pick_sources(el, 64, seed=inputs.SOURCE_SEEDS["rmat16"])
    assert len(srcs) == 64
    g, A = graph_pair(gpu, el.n, el.src, el.dst)
    for i, src in enumerate(srcs):
        if i % 16 == 0:
            say(f"rmat16 source {i}")
        parent, depth = device_bfs(gpu, g, int(src))
        assert_valid(A, int(src), parent, depth, what="rmat16")


def test_repeat_same_result(gpu):
    from paper_1508_03619_amd import inputs
    el = inputs.rmat(15, 16, seed=31)
    g, A = graph_pair(gpu, el.n, el.src, el.dst)
    src = int(inputs.pick_sources(el, 1, seed=32)[0])
    ref = A.bfs(src)[0]
    say("repeat x30")
    for _ in range(30):
        parent, depth = device_bfs(gpu, g, src)
        assert_valid(A, src, parent, depth, ref)


def test_two_streams_concurrently(gpu):
    import torch
    from paper_1508_03619_amd import inputs
    el = inputs.rmat(15, 16, seed=41)
    g, A = graph_pair(gpu, el.n, el.src, el.dst)
    srcs = [int(x) for x in inputs.pick_sources(el, 8, seed=42)]
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    outs = []
    say("two streams")
    for i, src in enumerate(srcs):
        st = streams[i % 2]
        p = torch.empty(g.n, dtype=torch.int32, device="cuda")
        d = torch.empty(g.n, dtype=torch.int32, device="cuda")
        with torch.cuda.stream(st):
            gpu.bfs(g, src, p, d, stream=st)
        outs.append((src, p, d))
    torch.cuda.synchronize()
    for src, p, d in outs:
        assert_valid(A, src, p.cpu().numpy(), d.cpu().numpy())


@pytest.mark.parametrize("split,coop", [(1, 0), (2, 0), (3, 0), (4, 0), (2, 1)])
def test_grid_split_streams_overlap(gpu, split, coop):
    """With grid_split = k, k persistent launches (single and batched) run at
    once on k streams (ordinary launches ordered by the device's launch
    ring; with coop_launch = 1 cooperative launches, which do not overlap);
    every result stays exact."""
    import torch
    from paper_1508_03619_amd import inputs
    el = inputs.rmat(14, 16, seed=43)
    g, A = graph_pair(gpu, el.n, el.src, el.dst)
    srcs = [int(x) for x in inputs.pick_sources(el, 24, seed=44)]
    saved = gpu.get_params()
    gpu.set_params(grid_split=split, coop_launch=coop)
    streams = [torch.cuda.Stream() for _ in range(split + 1)]
    outs = []
    say(f"grid_split={split} coop_launch={coop}")
    try:
        for i, src in enumerate(srcs):
            st = streams[i % len(streams)]
            with torch.cuda.stream(st):
                if i % 4 == 3:
                    lanes = srcs[i - 3:i + 1]
                    ps = [torch.empty(g.n, dtype=torch.int32, device="cuda") for _ in lanes]
                    ds = [torch.empty(g.n, dtype=torch.int32, device="cuda") for _ in lanes]
                    gpu.bfs_batch([g], [0] * len(lanes), lanes, ps, ds, stream=st)
                    outs += list(zip(lanes, ps, ds))
                else:
                    p = torch.empty(g.n, dtype=torch.int32, device="cuda")
                    d = torch.empty(g.n, dtype=torch.int32, device="cuda")
                    gpu.bfs(g, src, p, d, stream=st)
                    outs.append((src, p, d))
        torch.cuda.synchronize()
    finally:
        gpu.set_params(**saved)
    for src, p, d in outs:
        assert_valid(A, src, p.cpu().numpy(), d.cpu().numpy(), what=f"split={split}")


@pytest.mark.parametrize("block", [256, 512, 1024])
def test_small_group_levels(gpu, block):
    """Levels handed to the small group and back: thresholds that keep every
    top-down level small, none, and ones that switch several times."""
    from paper_1508_03619_amd import inputs
    for el, what in [(inputs.rmat(14, 16, seed=45), "rmat14"), (inputs.grid(300, 200, seed=46), "grid"),
                     (inputs.urand(20000, 60000, seed=47), "urand")]:
        g, A = graph_pair(gpu, el.n, el.src, el.dst)
        for src in inputs.pick_sources(el, 2, seed=48):
            ref = A.bfs(int(src))[0]
            for sf in (0, 16, 64, 700, 5000, 1 << 30):
                for direction in (0, 1):
                    say(f"small group {what} block={block} small={sf} dir={direction}")
                    parent, depth = device_bfs(gpu, g, int(src), params=dict(
                        block=block, small_frontier=sf, direction=direction))
                    assert_valid(A, int(src), parent, depth, ref, what=f"{what} small={sf}")
        g.free()


def test_lds_frontier_bitmap(gpu):
    """Bottom-up steps with the frontier bitmap wholly in LDS (R-MAT 16),
    its low words in LDS and the rest in L2 (a 10^6-vertex grid and a
    2^21-vertex graph: probes on both sides of the split), and in L2 only
    (the option off), with refilled
    lanes over per-workgroup ranges (ranges of 4, 128 and 61 words: shorter
    than a chunk, several chunks, a ragged last chunk) and with fixed words
    per wave."""
    from paper_1508_03619_amd import inputs
    for el, what in [(inputs.rmat(16, 16, seed=55), "rmat16"), (inputs.grid(1000, 1000, seed=56), "grid1000"),
                     (inputs.urand(1 << 21, 1 << 24, seed=57), "urand2M")]:
        g, A = graph_pair(gpu, el.n, el.src, el.dst)
        for src in inputs.pick_sources(el, 2, seed=58):
            ref = A.bfs(int(src))[0]
            for lds in (0, 1):
                for direction in (0, 2):
                    for bu in (0, 1):
                        say(f"lds bitmap {what} lds={lds} dir={direction} bu_mapping={bu}")
                        parent, depth = device_bfs(gpu, g, int(src), params=dict(
                            lds_bitmap=lds, direction=direction, bu_mapping=bu))
                        assert_valid(A, int(src), parent, depth, ref,
                                     what=f"{what} lds={lds} bu_mapping={bu}")
        g.free()


def test_bottom_up_mappings_repeated(gpu):
    """Both bottom-up mappings, with and without the LDS bitmap copy and
    plain-store claims, five times each on R-MAT 16: the sources include
    one (34524) whose search has many vertices whose first frontier
    neighbour is the seventh list entry (the second round of four), where
    one build of the kernel once lost finds now and then."""
    from paper_1508_03619_amd import inputs
    el = inputs.rmat(16, 16, seed=55)
    g, A = graph_pair(gpu, el.n, el.src, el.dst)
    srcs = [int(x) for x in inputs.pick_sources(el, 2, seed=58)] + [34524]
    for src in srcs:
        ref = A.bfs(src)[0]
        for lds, bu, tp in itertools.product((0, 1), (0, 1), (0, 8)):
            say(f"repeated src={src} lds={lds} bu_mapping={bu} td_plain={tp}")
            for rep in range(5):
                parent, depth = device_bfs(gpu, g, src, params=dict(lds_bitmap=lds, bu_mapping=bu, td_plain=tp))
                assert_valid(A, src, parent, depth, ref, what=f"lds={lds} bu={bu} td_plain={tp} rep {rep}")
    g.free()


def test_grid_road_like(gpu):
    from paper_1508_03619_amd import inputs
    el = inputs.grid(300, 200, seed=7)
    g, A = graph_pair(gpu, el.n, el.src, el.dst)
    for src in inputs.pick_sources(el, 3, seed=8):
        for mode in (0, 1, 2):
            say(f"grid300x200 src={src} mode={mode}")
            parent, depth = device_bfs(gpu, g, int(src), params=dict(mode=mode))
            assert_valid(A, int(src), parent, depth, what="grid")


def test_stats_records(gpu):
    from paper_1508_03619_amd import inputs
    el = inputs.rmat(14, 16, seed=51)
    g, A = graph_pair(gpu, el.n, el.src, el.dst)
    src = int(inputs.pick_sources(el, 1, seed=52)[0])
    import torch
    dref = A.bfs(src)[0]
    deg = np.diff(A.offsets)
    for mode in (0, 1, 2):
        parent = torch.empty(g.n, dtype=torch.int32, device="cuda")
        depth = torch.empty(g.n, dtype=torch.int32, device="cuda")
        recs = gpu.bfs(g, src, parent, depth, params=dict(mode=mode), stats=True)
        assert len(recs) == dref.max() + 1  # levels 0..max depth; the last claims nothing
        for r in recs:
            dd = r["level"]
            assert r["frontier"] == int((dref == dd).sum())
            assert r["frontier_edges"] == int(deg[dref == dd].sum())
            assert r["claimed"] == int((dref == dd + 1).sum())
