"""gap_bfs_noalloc (the search whose scratch is the library's per-device
array, for callers that cannot allocate) against gap_bfs on the same
inputs, through the C ABI: depths bit-exact, parents valid against the
oracle (Section 2.1), on two calls in a row, the second on a smaller graph,
then a NULL depth, and a graph too large for the array (GAP_EINVAL, nothing
queued)."""
import numpy as np
import pytest

import oracle
from tests import smallgraphs as sg
from tests.gpuutil import assert_valid, say

pytestmark = pytest.mark.gpu


def _search_pair(gb, g, A, s, with_depth=True):
    import torch
    p0 = torch.empty(g.n, dtype=torch.int32, device="cuda")
    d0 = torch.empty(g.n, dtype=torch.int32, device="cuda")
    gb.bfs(g, s, p0, d0)
    p1 = torch.full((g.n,), 7, dtype=torch.int32, device="cuda")
    d1 = torch.full((g.n,), 7, dtype=torch.int32, device="cuda") if with_depth else None
    gb.bfs_noalloc(g, s, p1, d1)
    torch.cuda.synchronize()
    gb.stream_status()
    ref = assert_valid(A, s, p0.cpu().numpy(), d0.cpu().numpy(), what="gap_bfs")
    if with_depth:
        dn = d1.cpu().numpy()
        assert np.array_equal(dn, d0.cpu().numpy()), "noalloc depths differ from gap_bfs"
        assert_valid(A, s, p1.cpu().numpy(), dn, ref=ref, what="gap_bfs_noalloc")
    else:
        assert_valid(A, s, p1.cpu().numpy(), None, ref=ref, what="gap_bfs_noalloc (no depth)")


def test_noalloc_matches_bfs_two_calls_then_smaller(gpu):
    from paper_1508_03619_amd import gapbfs as gb, inputs
    big = inputs.rmat(16, 16, seed=5516)
    small = inputs.rmat(11, 16, seed=5511)
    gs = []
    for tag, el in (("rmat16", big), ("rmat11", small)):
        say(f"noalloc: {tag}")
        g = gb.build_csr(el.n, el.src, el.dst)
        A = oracle.Adjacency(el.n, el.src, el.dst)
        for s in inputs.pick_sources(el, 2, seed=5500 + el.n % 97):
            _search_pair(gb, g, A, int(s))
        gs.append((g, A, el))
    say("noalloc: NULL depth, then back to the larger graph")
    g, A, el = gs[1]
    _search_pair(gb, g, A, int(inputs.pick_sources(el, 1, seed=5590)[0]), with_depth=False)
    g, A, el = gs[0]
    _search_pair(gb, g, A, int(inputs.pick_sources(el, 1, seed=5591)[0]))
    for g, _, _ in gs:
        g.free()


def test_noalloc_closed_forms_and_degenerate(gpu):
    """A long path (thousands of small levels), an isolated source, and a
    disconnected graph: depths from the closed forms."""
    import torch
    from paper_1508_03619_amd import gapbfs as gb
    cases = [("path 3000", sg.path(3000), 0), ("path 3000 mid", sg.path(3000), 1500),
             ("cycle 513", sg.cycle(513), 7)]
    for what, (n, src, dst, dist), s in cases:
        say(f"noalloc: {what}")
        g = gb.build_csr(n, src, dst)
        A = oracle.Adjacency(n, src, dst)
        p = torch.empty(n, dtype=torch.int32, device="cuda")
        d = torch.empty(n, dtype=torch.int32, device="cuda")
        gb.bfs_noalloc(g, s, p, d)
        torch.cuda.synchronize()
        gb.stream_status()
        dd = d.cpu().numpy()
        assert np.array_equal(dd, dist(s)), what
        assert_valid(A, s, p.cpu().numpy(), dd, what=what)
        g.free()
    # an isolated source: vertex 4 has no edges
    n, src, dst = 5, np.array([0, 1], np.int32), np.array([1, 2], np.int32)
    g = gb.build_csr(n, src, dst)
    p = torch.empty(n, dtype=torch.int32, device="cuda")
    d = torch.empty(n, dtype=torch.int32, device="cuda")
    gb.bfs_noalloc(g, 4, p, d)
    torch.cuda.synchronize()
    gb.stream_status()
    assert p.cpu().tolist() == [-1, -1, -1, -1, 4]
    assert d.cpu().tolist() == [-1, -1, -1, -1, 0]
    g.free()


def test_noalloc_rejects_a_graph_beyond_the_array(gpu):
    import torch
    from paper_1508_03619_amd import gapbfs as gb
    n = 600_000  # 132 bytes per vertex: beyond 64 MiB
    n_, src, dst, _ = sg.path(n)
    g = gb.build_csr(n, src, dst)
    p = torch.full((n,), 5, dtype=torch.int32, device="cuda")
    with pytest.raises(gb.GapError) as ei:
        gb.bfs_noalloc(g, 0, p, None)
    assert ei.value.status == gb.GAP_EINVAL
    torch.cuda.synchronize()
    assert int((p != 5).sum()) == 0, "nothing may run for a rejected call"
    g.free()
