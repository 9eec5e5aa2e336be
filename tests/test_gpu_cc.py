"""Connected components on the device against the oracle (Section 2.1).

Both sides label a vertex with the smallest vertex of its component, so
labels must match exactly; the paper's verifier (one traversal per label,
Section 3) also runs on the device result.  Covers every graph on 5
vertices, random graphs with repeats and self-loops both ways (weak
components when directed), long paths, hubs split into chunk items,
generated graphs, repeated runs, edge cases, two streams and replays of a
captured call."""
import itertools

import numpy as np
import pytest

import oracle
from tests import smallgraphs as sg
from tests.gpuutil import say

pytestmark = pytest.mark.gpu


def gpu_cc(gb, g):
    import torch
    out = torch.empty(g.n, dtype=torch.int32, device="cuda")
    gb.cc(g, out)
    torch.cuda.synchronize()
    return out.cpu().numpy()


def check(gb, n, s, d, directed=False, what=""):
    s = np.asarray(s, np.int32)
    d = np.asarray(d, np.int32)
    g = gb.build_csr(n, s, d, directed=directed)
    got = gpu_cc(gb, g)
    ref = oracle.components(n, s, d)
    bad = np.nonzero(got != ref)[0]
    assert bad.size == 0, f"{what}: {bad.size} labels differ, v={bad[0]} gpu={got[bad[0]]} ref={ref[bad[0]]}"
    A = oracle.Adjacency(n, s, d)  # undirected view for the verifier
    assert A.cc_check(got)[0] == 0, what
    g.free()
    return got


def test_all_five_vertex_graphs(gpu):
    k = 5
    pairs = list(itertools.combinations(range(k), 2))
    say("cc: all 5-vertex graphs")
    for mask in range(1 << len(pairs)):
        sel = [pairs[b] for b in range(len(pairs)) if (mask >> b) & 1]
        check(gpu, k, [p[0] for p in sel], [p[1] for p in sel], what=f"mask {mask}")


def test_random_graphs_both_ways(gpu):
    for seed in range(40):
        rng = np.random.default_rng(130 + seed)
        n = int(rng.integers(1, 3000))
        m = int(rng.integers(0, 2 * n))
        s = rng.integers(0, n, m).astype(np.int32)
        d = rng.integers(0, n, m).astype(np.int32)
        if m:
            s = np.concatenate([s, s[: m // 4 + 1], d[:3]])
            d = np.concatenate([d, d[: m // 4 + 1], d[:3]])
        say(f"cc: random seed={seed} n={n}")
        check(gpu, n, s, d, directed=bool(seed % 2), what=f"seed {seed}")


def test_closed_forms_and_hubs(gpu):
    for name, (n, s, d, _) in [("path5000", sg.path(5000)), ("cycle4001", sg.cycle(4001)),
                               ("star20000", sg.star(20000)), ("K60", sg.complete(60)),
                               ("grid80x70", sg.full_grid(80, 70)),
                               ("union", sg.disjoint_union(sg.path(7), sg.star(300), sg.path(1), sg.cycle(9)))]:
        say(f"cc: {name}")
        check(gpu, n, s, d, what=name)
        # reversed vertex numbering: the smallest vertex sits at the far end
        rs, rd = n - 1 - np.asarray(s), n - 1 - np.asarray(d)
        check(gpu, n, rs, rd, what=name + " reversed")


@pytest.mark.parametrize("name", ["rmat16", "rmat16d"])
def test_generated_graphs(gpu, name):
    from paper_1508_03619_amd import inputs
    el = inputs.workload(name)
    say(f"cc: {name}")
    first = check(gpu, el.n, el.src, el.dst, directed=name.endswith("d"), what=name)
    for el2 in (inputs.urand(1 << 16, 1 << 15, seed=131), inputs.grid(200, 150, seed=132),
                inputs.rmat(16, 2, seed=133)):
        check(gpu, el2.n, el2.src, el2.dst, what=el2.name)
    # scheduling changes nothing: the labels are unique
    g = gpu.build_csr(el.n, el.src, el.dst, directed=name.endswith("d"))
    for _ in range(5):
        assert np.array_equal(gpu_cc(gpu, g), first)
    g.free()


def test_edge_cases(gpu):
    say("cc: edge cases")
    check(gpu, 1, [], [], what="one vertex")
    check(gpu, 70, [], [], what="no edges")
    check(gpu, 70, np.arange(70), np.arange(70), what="self-loops only")
    with pytest.raises(ValueError):
        gpu.cc(gpu.build_csr(3, np.array([0], np.int32), np.array([1], np.int32)),
               __import__("torch").empty(2, dtype=__import__("torch").int32, device="cuda"))


def test_two_streams(gpu):
    import torch
    from paper_1508_03619_amd import inputs
    els = [inputs.rmat(14, 4, seed=134), inputs.urand(1 << 14, 1 << 13, seed=135)]
    gs = [gpu.build_csr(e.n, e.src, e.dst) for e in els]
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    outs = [torch.empty(g.n, dtype=torch.int32, device="cuda") for g in gs]
    say("cc: two streams")
    for g, st, o in zip(gs, streams, outs):
        gpu.cc(g, o, stream=st)
    torch.cuda.synchronize()
    for e, o in zip(els, outs):
        assert np.array_equal(o.cpu().numpy(), oracle.components(e.n, e.src, e.dst))
    for g in gs:
        g.free()


@pytest.mark.parametrize("directed", [False, True])
def test_captured_graph_replays(gpu, directed):
    """The call only queues work (no host wait, no memset), so it can be
    captured once its stream's scratch exists; every replay, with eager
    calls in between, gives the oracle's labels."""
    import torch
    from paper_1508_03619_amd import inputs
    el = inputs.rmat(14, 8, seed=136)
    g = gpu.build_csr(el.n, el.src, el.dst, directed=directed)
    ref = oracle.components(el.n, el.src, el.dst)
    st = torch.cuda.Stream()
    labels = torch.empty(g.n, dtype=torch.int32, device="cuda")
    eager = torch.empty(g.n, dtype=torch.int32, device="cuda")
    gpu.cc(g, labels, stream=st)  # sizes the stream's scratch
    st.synchronize()
    say(f"cc: graph capture directed={directed}")
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph, stream=st):
        gpu.cc(g, labels, stream=st)
    for _ in range(3):
        labels.fill_(-7)
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        assert np.array_equal(labels.cpu().numpy(), ref)
        gpu.cc(g, eager, stream=st)
        st.synchronize()
        assert np.array_equal(eager.cpu().numpy(), ref)
    del graph
    g.free()
