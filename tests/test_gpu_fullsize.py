"""Parity at the measured sizes, in the launch configuration the benchmark
times: R-MAT scale 22 and uniform-random 2^22 (single-source and the
64-lane batch), the 4096^2 road-like grid (persistent kernel and captured
level graphs), R-MAT scale 24 in batches of 64 and 256 lanes, the mixed
batch of 16 R-MAT graphs of scales 14-20, R-MAT scale 22 taken as a
directed graph, betweenness centrality on R-MAT scale 22, shortest paths
on R-MAT and uniform scale 22 with weights 1..255, and connected components
at scale 22.

Checked in full against the oracle (depths bit-exact, parents valid,
Section 2.1): all 64 benchmark sources of R-MAT 22 and uniform 2^22 as
single searches and every lane of their 64-lane batches; every lane of the
R-MAT 24 64-lane batch and 16 lanes of the 256-lane batch; 4 grid sources
in both schedules; every lane of the mixed batches.  Every lane of every
batch is also checked on the device against properties that hold at any
size: parent[s] = s, depth[s] = 0, and the reached set is exactly the
source's connected component from the oracle's union-find."""
import numpy as np
import pytest

import oracle
from tests.gpuutil import assert_valid, check_all, say

pytestmark = pytest.mark.gpu

_cache = {}


def workload(name):
    """(edge list, oracle adjacency or None, component labels, device graph)."""
    if name not in _cache:
        from paper_1508_03619_amd import inputs, gapbfs as gb
        if name.startswith("mixed"):
            raise KeyError(name)
        say(f"{name}: generating")
        el = inputs.workload(name)
        say(f"{name}: building the device CSR")
        g = gb.build_csr(el.n, el.src, el.dst)
        _cache[name] = {"el": el, "g": g, "A": None, "cc": None}
    return _cache[name]


def adjacency(name):
    w = workload(name)
    if w["A"] is None:
        say(f"{name}: oracle adjacency")
        w["A"] = oracle.Adjacency(w["el"].n, w["el"].src, w["el"].dst)
    return w["A"]


def comp_labels(name):
    w = workload(name)
    if w["cc"] is None:
        say(f"{name}: oracle components")
        w["cc"] = oracle.components(w["el"].n, w["el"].src, w["el"].dst)
    return w["cc"]


def drop(name):
    w = _cache.pop(name, None)
    if w is not None:
        w["g"].free()


def bench_sources(name, k=64):
    from paper_1508_03619_amd import inputs
    return [int(x) for x in inputs.pick_sources(workload(name)["el"], k, seed=inputs.SOURCE_SEEDS[name])]


def run_single(g, s, params=None, p=None, d=None):
    import torch
    from paper_1508_03619_amd import gapbfs as gb
    p = torch.empty(g.n, dtype=torch.int32, device="cuda") if p is None else p
    d = torch.empty(g.n, dtype=torch.int32, device="cuda") if d is None else d
    gb.bfs(g, s, p, d, params=params)
    torch.cuda.synchronize()
    gb.stream_status()
    return p.cpu().numpy(), d.cpu().numpy()


def check_batch_properties(what, labels, lanes, P, D):
    """Every lane, on the device: source entries, and the reached set equals
    the source's component (oracle union-find labels, uploaded once)."""
    import torch
    lab_t = torch.from_numpy(np.ascontiguousarray(labels)).to("cuda")
    for i, s in enumerate(lanes):
        assert int(P[i][s]) == s and int(D[i][s]) == 0, f"{what} lane {i}: source entries"
        reached = D[i] >= 0
        comp = lab_t == int(labels[s])
        assert torch.equal(reached, comp), \
            f"{what} lane {i}: reached {int(reached.sum())} vertices, component has {int(comp.sum())}"
        assert torch.equal(P[i] >= 0, reached), f"{what} lane {i}: parent/depth reach differ"
        assert int(P[i].min()) >= -1 and int(D[i].min()) >= -1
    del lab_t


@pytest.mark.timeout(900)
@pytest.mark.parametrize("name", ["rmat22", "urand22"])
def test_fullsize_single_and_batch(gpu, name):
    """All 64 benchmark sources: the single search and the batch lane of
    each, in full against one oracle search per source."""
    import torch
    from paper_1508_03619_amd import gapbfs as gb
    srcs = bench_sources(name)
    g = workload(name)["g"]
    A = adjacency(name)
    say(f"{name}: 64-lane batch")
    P = [torch.empty(g.n, dtype=torch.int32, device="cuda") for _ in srcs]
    D = [torch.empty(g.n, dtype=torch.int32, device="cuda") for _ in srcs]
    gb.bfs_batch([g], [0] * 64, srcs, P, D)
    torch.cuda.synchronize()
    gb.stream_status()
    check_batch_properties(name, comp_labels(name), srcs, P, D)
    p1 = torch.empty(g.n, dtype=torch.int32, device="cuda")
    d1 = torch.empty(g.n, dtype=torch.int32, device="cuda")

    def items():
        for i, s in enumerate(srcs):
            p, d = run_single(g, s, p=p1, d=d1)
            yield A, s, [(f"single {i}", p, d), (f"lane {i}", P[i].cpu().numpy(), D[i].cpu().numpy())]

    say(f"{name}: 64 single searches and 64 lanes vs the oracle")
    assert check_all(items(), what=name) == 128
    del P, D
    drop(name)


@pytest.mark.timeout(900)
def test_fullsize_grid4096_persistent_and_graph(gpu):
    """Four benchmark sources of the road-like grid, each in the persistent
    kernel and in captured level graphs."""
    name = "grid4096"
    srcs = bench_sources(name, 4)
    g = workload(name)["g"]
    A = adjacency(name)

    def items():
        for s in srcs:
            res = []
            for mode in (0, 2):
                say(f"grid4096: source {s} mode {mode}")
                p, d = run_single(g, s, params={"mode": mode})
                res.append((f"mode {mode}", p, d))
            yield A, s, res

    assert check_all(items(), what="grid4096") == 8
    drop(name)


@pytest.mark.timeout(1200)
@pytest.mark.parametrize("lanes", [64, 256])
def test_fullsize_rmat24_batch(gpu, lanes):
    """Every lane against the source's component on the device; all 64
    lanes of the 64-lane batch and 16 spread lanes of the 256-lane batch in
    full against the oracle."""
    import torch
    from paper_1508_03619_amd import gapbfs as gb
    name = "rmat24"
    srcs = bench_sources(name, lanes)
    g = workload(name)["g"]
    say(f"rmat24: batch of {lanes}")
    P = [torch.empty(g.n, dtype=torch.int32, device="cuda") for _ in srcs]
    D = [torch.empty(g.n, dtype=torch.int32, device="cuda") for _ in srcs]
    gb.bfs_batch([g], [0] * lanes, srcs, P, D)
    torch.cuda.synchronize()
    gb.stream_status()
    say(f"rmat24: properties of {lanes} lanes")
    check_batch_properties(name, comp_labels(name), srcs, P, D)
    A = adjacency(name)
    full = list(range(lanes)) if lanes == 64 else list(range(0, lanes, lanes // 16))
    say(f"rmat24: {len(full)} lanes vs the oracle")
    items = ((A, srcs[i], [(f"lane {i}", P[i].cpu().numpy(), D[i].cpu().numpy())]) for i in full)
    assert check_all(items, what=f"rmat24 batch {lanes}") == len(full)
    del P, D
    torch.cuda.empty_cache()
    if lanes == 256:
        drop(name)


MIXED_SCALES = [14, 14, 15, 15, 16, 16, 17, 17, 18, 18, 19, 19, 20, 20, 20, 20]


@pytest.mark.timeout(900)
@pytest.mark.parametrize("per_graph", [4, 16])
def test_fullsize_mixed_batch(gpu, per_graph):
    """16 R-MAT graphs of scales 14-20 in one launch: every lane in full
    against the oracle of its own graph, and its reached set against that
    graph's components."""
    import torch
    from paper_1508_03619_amd import inputs, gapbfs as gb
    els = [inputs.rmat(s, 16, seed=30000 + i) for i, s in enumerate(MIXED_SCALES)]
    graphs = [gb.build_csr(e.n, e.src, e.dst) for e in els]
    gos, srcs = [], []
    for gi, e in enumerate(els):
        for s in inputs.pick_sources(e, per_graph, seed=1030000 + gi):
            gos.append(gi)
            srcs.append(int(s))
    say(f"mixed: {len(srcs)} lanes over 16 graphs")
    P = [torch.empty(graphs[gi].n, dtype=torch.int32, device="cuda") for gi in gos]
    D = [torch.empty(graphs[gi].n, dtype=torch.int32, device="cuda") for gi in gos]
    gb.bfs_batch(graphs, gos, srcs, P, D)
    torch.cuda.synchronize()
    gb.stream_status()
    As = [oracle.Adjacency(e.n, e.src, e.dst) for e in els]
    for gi, e in enumerate(els):
        idx = [k for k in range(len(gos)) if gos[k] == gi]
        check_batch_properties(f"mixed graph {gi}", oracle.components(e.n, e.src, e.dst),
                               [srcs[k] for k in idx], [P[k] for k in idx], [D[k] for k in idx])
    items = ((As[gi], s, [(f"graph {gi} lane {i}", P[i].cpu().numpy(), D[i].cpu().numpy())])
             for i, (gi, s) in enumerate(zip(gos, srcs)))
    assert check_all(items, what="mixed") == len(srcs)
    for g in graphs:
        g.free()


@pytest.mark.timeout(900)
def test_fullsize_rmat22_directed(gpu):
    """R-MAT scale 22 with the pairs as directed edges: all 64 benchmark
    sources in full against the directed oracle, in the configuration the
    benchmark times, and the forced bottom-up and captured-level schedules
    on one of them."""
    import torch
    from paper_1508_03619_amd import inputs, gapbfs as gb
    name = "rmat22d"
    say(f"{name}: generating")
    el = inputs.workload(name)
    srcs = [int(x) for x in inputs.pick_sources(el, 64, seed=inputs.SOURCE_SEEDS[name], directed=True)]
    say(f"{name}: building the directed device CSR")
    g = gb.build_csr(el.n, el.src, el.dst, directed=True)
    say(f"{name}: oracle adjacency")
    A = oracle.Adjacency(el.n, el.src, el.dst, directed=True)
    p1 = torch.empty(g.n, dtype=torch.int32, device="cuda")
    d1 = torch.empty(g.n, dtype=torch.int32, device="cuda")

    def items():
        for i, s in enumerate(srcs):
            res = [("default", *run_single(g, s, p=p1, d=d1))]
            if i == 0:
                for sch in (dict(direction=2), dict(mode=2)):
                    res.append((str(sch), *run_single(g, s, params=sch, p=p1, d=d1)))
            yield A, s, res

    say(f"{name}: 64 sources vs the directed oracle")
    assert check_all(items(), what=name) == 66
    g.free()


@pytest.mark.timeout(900)
def test_fullsize_bc_rmat22(gpu):
    """Betweenness centrality on R-MAT 22 from 4 sources (the benchmark's
    trial), every score against the oracle (|gpu - oracle| <= 1e-9 |oracle|
    + 1e-12 max), and one source's raw scores against the identity
    sum = total of (distance - 1) over the reached vertices."""
    import torch
    from paper_1508_03619_amd import inputs, gapbfs as gb
    name = "rmat22"
    srcs = [int(x) for x in inputs.pick_sources(workload(name)["el"], 32,
                                                seed=inputs.SOURCE_SEEDS[name] + 5)][:4]
    g = workload(name)["g"]
    A = adjacency(name)
    out = torch.empty(g.n, dtype=torch.float64, device="cuda")
    say(f"{name}: betweenness from {srcs}")
    gb.bc(g, srcs, out)
    torch.cuda.synchronize()
    got = out.cpu().numpy()
    say(f"{name}: oracle betweenness")
    ref = A.bc(srcs)
    tol = 1e-9 * np.abs(ref) + 1e-12 * float(ref.max())
    bad = np.nonzero(~(np.abs(got - ref) <= tol))[0]
    assert bad.size == 0, (bad.size, int(bad[0]), got[bad[0]], ref[bad[0]])
    gb.bc(g, srcs[:1], out, normalise=False)
    torch.cuda.synchronize()
    raw = out.cpu().numpy()
    depth = A.bfs(srcs[0])[0]
    want = float(np.sum(depth[depth > 0] - 1))
    assert abs(raw.sum() - want) <= 1e-9 * want
    drop(name)


@pytest.mark.timeout(900)
@pytest.mark.parametrize("name", ["rmat22", "urand22"])
def test_fullsize_sssp(gpu, name):
    """Shortest paths at scale 22 with the generator's weights 1..255:
    two sources against Dijkstra (exact distances), with the default bucket
    width the benchmark uses and one other."""
    import torch
    from paper_1508_03619_amd import inputs, gapbfs as gb
    el = inputs.workload(name)
    w = inputs.weights(el, seed=inputs.WEIGHT_SEEDS[name])
    say(f"{name}: weighted device CSR")
    g = gb.build_csr(el.n, el.src, el.dst, weights=w)
    say(f"{name}: oracle weighted adjacency")
    A = oracle.WeightedAdjacency(el.n, el.src, el.dst, w)
    srcs = [int(x) for x in inputs.pick_sources(el, 2, seed=inputs.SOURCE_SEEDS[name] + 21)]
    out = torch.empty(g.n, dtype=torch.int32, device="cuda")
    for s in srcs:
        say(f"{name}: Dijkstra from {s}")
        ref = A.sssp(s)
        ref = np.where(ref < 0, 0xFFFFFFFF, ref)
        for delta in (0, 256):
            say(f"{name}: gpu delta={delta}")
            gb.sssp(g, s, out, delta=delta)
            torch.cuda.synchronize()
            got = out.cpu().numpy().view(np.uint32).astype(np.int64)
            bad = np.nonzero(got != ref)[0]
            assert bad.size == 0, (name, s, delta, bad.size, int(bad[0]), got[bad[0]], ref[bad[0]])
    g.free()


@pytest.mark.timeout(900)
@pytest.mark.parametrize("name", ["rmat22", "urand22", "rmat22d"])
def test_fullsize_cc(gpu, name):
    """Connected components at scale 22 (weak components for the directed
    R-MAT): every label against the oracle's union-find."""
    import torch
    from paper_1508_03619_amd import inputs, gapbfs as gb
    el = inputs.workload(name)
    g = gb.build_csr(el.n, el.src, el.dst, directed=name.endswith("d"))
    out = torch.empty(g.n, dtype=torch.int32, device="cuda")
    say(f"{name}: components")
    gb.cc(g, out)
    torch.cuda.synchronize()
    got = out.cpu().numpy()
    ref = oracle.components(el.n, el.src, el.dst)
    bad = np.nonzero(got != ref)[0]
    assert bad.size == 0, (name, bad.size, int(bad[0]), got[bad[0]], ref[bad[0]])
    g.free()
