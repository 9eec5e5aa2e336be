"""Continuous batching (gap_serve_*): queries join a running multi-source
search at level boundaries and complete on their own.  Every query is
checked against the oracle (depths bit-exact, parents valid, Section 2.1),
and a query alone and in the mix give the same depths.

Injection mid-flight is observed directly: on a graph made of a long path
and a small star, a star query submitted while a path query runs completes
first, which only a query that joined the running launch can do (a later
launch on the same stream would start after the path query ends)."""
import time

import numpy as np
import pytest

import oracle
from tests import smallgraphs as sg
from tests.gpuutil import assert_valid, say

pytestmark = pytest.mark.gpu


def _drain(srv, want, timeout=60.0):
    """Polls until `want` queries completed (bounded)."""
    got = []
    t0 = time.time()
    while len(got) < want:
        got += srv.poll()
        if time.time() - t0 > timeout:
            raise AssertionError(f"only {len(got)} of {want} queries completed in {timeout}s")
        time.sleep(0.0002)
    return got


def _host(t):
    """Device tensor -> numpy, read on a side stream (the server's stream is
    busy while its launch runs)."""
    import torch
    side = torch.cuda.Stream()
    with torch.cuda.stream(side):
        out = t.cpu().numpy()
    side.synchronize()
    return out


@pytest.fixture
def window():
    from paper_1508_03619_amd import gapbfs as gb
    saved = gb.get_params()
    yield lambda us: gb.set_params(serve_window_us=us)
    gb.set_params(**saved)


def _outputs(n, k):
    import torch
    P = [torch.full((n,), 7, dtype=torch.int32, device="cuda") for _ in range(k)]
    D = [torch.full((n,), 7, dtype=torch.int32, device="cuda") for _ in range(k)]
    torch.cuda.synchronize()
    return P, D


def test_serve_matches_oracle_many_queries(gpu, window):
    """150 queries on R-MAT 14 (more than 64 lanes: the rest wait in the
    ring and join as lanes free up), with the default window."""
    import torch
    from paper_1508_03619_amd import gapbfs as gb, inputs
    el = inputs.rmat(14, 16, seed=6101)
    g = gb.build_csr(el.n, el.src, el.dst)
    A = oracle.Adjacency(el.n, el.src, el.dst)
    srcs = [int(x) for x in inputs.pick_sources(el, 150, seed=6102)]
    st = torch.cuda.Stream()
    srv = gb.Server(g.n, g.nnz, stream=st)
    P, D = _outputs(g.n, len(srcs))
    for q, s in enumerate(srcs):
        assert srv.submit(g, q, s, P[q], D[q])
    done = _drain(srv, len(srcs))
    assert sorted(done) == list(range(len(srcs)))
    st.synchronize()
    gb.stream_status(st)
    for q, s in enumerate(srcs):
        assert_valid(A, s, _host(P[q]), _host(D[q]), what=f"served query {q}")
    srv.close()
    g.free()


def test_serve_injects_into_a_running_launch(gpu, window):
    """A 6000-level path query runs; star queries submitted meanwhile finish
    before it (they joined its launch), with exact depths."""
    import torch
    from paper_1508_03619_amd import gapbfs as gb
    window(2_000_000)  # long enough that the launch takes every query below
    n, s, d, _ = sg.disjoint_union(sg.path(6000), sg.star(40))
    g = gb.build_csr(n, s, d)
    A = oracle.Adjacency(n, s, d)
    st = torch.cuda.Stream()
    srv = gb.Server(g.n, g.nnz, stream=st)
    P, D = _outputs(g.n, 4)
    assert srv.submit(g, 0, 0, P[0], D[0])  # path end: ~6000 levels
    time.sleep(0.002)
    order = []
    for q in (1, 2, 3):  # the star's centre and two leaves
        assert srv.submit(g, q, 6000 + (0 if q == 1 else q), P[q], D[q])
        order += srv.poll()
    order += _drain(srv, 4 - len(order))
    say(f"completion order {order}")
    assert order[-1] == 0, f"the path query should finish last: {order}"
    st.synchronize()
    gb.stream_status(st)
    for q, src in enumerate((0, 6000, 6002, 6003)):
        assert_valid(A, src, _host(P[q]), _host(D[q]), what=f"query {q} from {src}")
    srv.close()
    g.free()


def test_serve_alone_and_in_the_mix_agree(gpu, window):
    """The same queries alone (one at a time) and in a mix of 64 staggered
    submissions: identical depths, both parent arrays valid."""
    import torch
    from paper_1508_03619_amd import gapbfs as gb, inputs
    el = inputs.grid(120, 90, seed=6201)
    g = gb.build_csr(el.n, el.src, el.dst)
    A = oracle.Adjacency(el.n, el.src, el.dst)
    srcs = [int(x) for x in inputs.pick_sources(el, 64, seed=6202)]
    st = torch.cuda.Stream()
    srv = gb.Server(g.n, g.nnz, stream=st)
    alone_d = []
    P1, D1 = _outputs(g.n, 1)
    for q in range(6):
        assert srv.submit(g, q, srcs[q], P1[0], D1[0])
        _drain(srv, 1)
        st.synchronize()
        alone_d.append(_host(D1[0]))
        assert_valid(A, srcs[q], _host(P1[0]), alone_d[-1], what=f"alone {q}")
    P, D = _outputs(g.n, len(srcs))
    pending = 0
    for q, s in enumerate(srcs):
        assert srv.submit(g, 100 + q, s, P[q], D[q])
        pending += 1
        if q % 8 == 7:  # let some levels pass between groups of arrivals
            time.sleep(0.0003)
    _drain(srv, pending)
    st.synchronize()
    gb.stream_status(st)
    for q, s in enumerate(srcs):
        dq = _host(D[q])
        assert_valid(A, s, _host(P[q]), dq, what=f"mix {q}")
        if q < 6:
            assert np.array_equal(dq, alone_d[q]), f"query {q}: alone and in the mix differ"
    srv.close()
    g.free()


def test_serve_window_zero_graphs_in_turn_and_limits(gpu, window):
    """Window 0 (requests taken at a launch's first boundary only), two
    graphs served in turn by one server, the ring limit, argument errors."""
    import torch
    from paper_1508_03619_amd import gapbfs as gb, inputs
    window(0)
    e1 = inputs.rmat(10, 8, seed=6301)
    e2 = inputs.urand(700, 2800, seed=6302)
    g1 = gb.build_csr(e1.n, e1.src, e1.dst)
    g2 = gb.build_csr(e2.n, e2.src, e2.dst)
    A1 = oracle.Adjacency(e1.n, e1.src, e1.dst)
    A2 = oracle.Adjacency(e2.n, e2.src, e2.dst)
    st = torch.cuda.Stream()
    srv = gb.Server(max(g1.n, g2.n), max(g1.nnz, g2.nnz), stream=st)
    for g, A, el, seed in ((g1, A1, e1, 6303), (g2, A2, e2, 6304), (g1, A1, e1, 6305)):
        srcs = [int(x) for x in inputs.pick_sources(el, 20, seed=seed)]
        P, D = _outputs(g.n, len(srcs))
        for q, s in enumerate(srcs):
            assert srv.submit(g, q, s, P[q], D[q])
        _drain(srv, len(srcs))
        st.synchronize()
        for q, s in enumerate(srcs):
            assert_valid(A, s, _host(P[q]), _host(D[q]), what=f"window 0 query {q}")
    # a server holding queries on one graph refuses another graph
    P, D = _outputs(g1.n, 1)
    assert srv.submit(g1, 0, 1, P[0], D[0])
    P2, D2 = _outputs(g2.n, 1)
    assert srv.submit(g2, 1, 1, P2[0], D2[0]) is False
    _drain(srv, 1)
    # argument errors
    with pytest.raises(gb.GapError) as ei:
        srv.submit(g1, 2, g1.n, P[0], D[0])
    assert ei.value.status == gb.GAP_EINVAL
    big = inputs.rmat(12, 16, seed=6306)
    gbig = gb.build_csr(big.n, big.src, big.dst)
    Pb, Db = _outputs(gbig.n, 1)
    with pytest.raises(gb.GapError) as ei:
        srv.submit(gbig, 3, 0, Pb[0], Db[0])
    assert ei.value.status == gb.GAP_EINVAL
    st.synchronize()
    gb.stream_status(st)
    srv.close()
    for g in (g1, g2, gbig):
        g.free()


def test_serve_ring_limit(gpu, window):
    """256 queries in flight at most: the 257th submission is refused until
    completions are polled."""
    import torch
    from paper_1508_03619_amd import gapbfs as gb
    n, s, d, dist = sg.cycle(300)
    g = gb.build_csr(n, s, d)
    st = torch.cuda.Stream()
    srv = gb.Server(g.n, g.nnz, stream=st)
    P, D = _outputs(g.n, 1)  # every query writes the same arrays: only the count matters here
    for q in range(gb.SERVE_RING):
        assert srv.submit(g, q, q % n, P[0], D[0])
    assert srv.submit(g, 999, 0, P[0], D[0]) is False
    done = _drain(srv, gb.SERVE_RING)
    assert sorted(done) == list(range(gb.SERVE_RING))
    assert srv.submit(g, 999, 5, P[0], D[0])
    _drain(srv, 1)
    st.synchronize()
    gb.stream_status(st)
    assert np.array_equal(_host(D[0]), dist(5))
    srv.close()
    g.free()
