"""Device-side failures are reported, never lost, and every kernel exits.

A search's bounded waits (grid barriers, parked workgroups) give up after
``wait_limit_us`` without progress.  Setting that bound to one microsecond
from the host makes the first barrier wait of a search give up on the
device: every workgroup then leaves the kernel normally, the search records
GAP_ETIMEOUT, and the stream's sticky status word carries it past the
control-block reset of the next search until gap_stream_status reads it.

The parked-workgroup watchdog is bounded by time without progress: a path
graph runs tens of thousands of small levels in a row, far longer in total
than a 50 ms bound, and must still finish with exact depths."""
import numpy as np
import pytest

import oracle
from tests.gpuutil import assert_valid, say
from tests import smallgraphs as sg

pytestmark = pytest.mark.gpu


def _rmat(scale):
    from paper_1508_03619_amd import inputs
    return inputs.rmat(scale, 16, seed=4400 + scale)


def test_single_search_timeout_is_sticky(gpu):
    import torch
    from paper_1508_03619_amd import gapbfs as gb, inputs
    el = _rmat(14)
    g = gb.build_csr(el.n, el.src, el.dst)
    A = oracle.Adjacency(el.n, el.src, el.dst)
    s = int(inputs.pick_sources(el, 1, seed=4401)[0])
    p = torch.empty(g.n, dtype=torch.int32, device="cuda")
    d = torch.empty(g.n, dtype=torch.int32, device="cuda")
    gb.stream_status()  # nothing pending from earlier tests on this stream
    say("single search with a 1 us wait bound")
    gb.bfs(g, s, p, d, params={"wait_limit_us": 1})  # queues and returns GAP_OK
    # a good search queued behind it clears the failed search's control
    # block; the failure must survive that
    gb.bfs(g, s, p, d)
    with pytest.raises(gb.GapError) as ei:
        gb.stream_status()
    assert ei.value.status == gb.GAP_ETIMEOUT
    gb.stream_status()  # read once, then cleared
    p_, d_ = p.cpu().numpy(), d.cpu().numpy()
    assert_valid(A, s, p_, d_, what="search after a failed one")
    say("with statistics the failure comes back from the call itself")
    with pytest.raises(gb.GapError) as ei:
        gb.bfs(g, s, p, d, params={"wait_limit_us": 1}, stats=True)
    assert ei.value.status == gb.GAP_ETIMEOUT
    with pytest.raises(gb.GapError) as ei:  # the sticky word holds it too
        gb.stream_status()
    assert ei.value.status == gb.GAP_ETIMEOUT
    gb.stream_status()  # and reading it cleared it
    gb.bfs(g, s, p, d)
    torch.cuda.synchronize()
    gb.stream_status()
    assert_valid(A, s, p.cpu().numpy(), d.cpu().numpy(), what="recovered search")
    g.free()


def test_batch_timeout_poisons_outputs(gpu):
    import torch
    from paper_1508_03619_amd import gapbfs as gb, inputs
    el = _rmat(13)
    g = gb.build_csr(el.n, el.src, el.dst)
    A = oracle.Adjacency(el.n, el.src, el.dst)
    srcs = [int(x) for x in inputs.pick_sources(el, 8, seed=4402)]
    P = [torch.zeros(g.n, dtype=torch.int32, device="cuda") for _ in srcs]
    D = [torch.zeros(g.n, dtype=torch.int32, device="cuda") for _ in srcs]
    saved = gb.get_params()
    gb.stream_status()
    try:
        gb.set_params(wait_limit_us=1)
        say("batch of 8 with a 1 us wait bound")
        gb.bfs_batch([g], [0] * len(srcs), srcs, P, D)
    finally:
        gb.set_params(**saved)
    with pytest.raises(gb.GapError) as ei:
        gb.stream_status()
    assert ei.value.status == gb.GAP_ETIMEOUT
    imin = np.iinfo(np.int32).min
    for p, d in zip(P, D):
        assert (p.cpu().numpy() == imin).all() and (d.cpu().numpy() == imin).all()
    say("the same batch with the built-in bounds")
    gb.bfs_batch([g], [0] * len(srcs), srcs, P, D)
    gb.stream_status()
    for s, p, d in zip(srcs, P, D):
        assert_valid(A, s, p.cpu().numpy(), d.cpu().numpy(), what="batch after a failed one")
    g.free()


def test_parked_wait_is_bounded_by_progress(gpu):
    """40,000-vertex path from one end: ~40,000 small top-down levels (far
    more than 50 ms in all), each well inside the bound."""
    import time
    import torch
    from paper_1508_03619_amd import gapbfs as gb
    n, src, dst, closed_form = sg.path(40000)
    g = gb.build_csr(n, src, dst)
    A = oracle.Adjacency(n, src, dst)
    p = torch.empty(n, dtype=torch.int32, device="cuda")
    d = torch.empty(n, dtype=torch.int32, device="cuda")
    gb.stream_status()
    t0 = time.perf_counter()
    gb.bfs(g, 0, p, d, params={"wait_limit_us": 50000})
    gb.stream_status()
    took = time.perf_counter() - t0
    say(f"path of {n}: {took * 1e3:.0f} ms")
    assert took > 0.05, "the search should outlast the bound several times over"
    dd = p.cpu().numpy(), d.cpu().numpy()
    assert_valid(A, 0, dd[0], dd[1], what="long path")
    assert (dd[1] == closed_form(0)).all()
    g.free()


def test_shutdown_then_search(gpu):
    import torch
    from paper_1508_03619_amd import gapbfs as gb, inputs
    el = _rmat(12)
    g = gb.build_csr(el.n, el.src, el.dst)
    A = oracle.Adjacency(el.n, el.src, el.dst)
    s = int(inputs.pick_sources(el, 1, seed=4403)[0])
    p = torch.empty(g.n, dtype=torch.int32, device="cuda")
    d = torch.empty(g.n, dtype=torch.int32, device="cuda")
    gb.bfs(g, s, p, d)
    gb.shutdown()  # waits, then releases every pool
    gb.bfs(g, s, p, d)  # allocates again
    torch.cuda.synchronize()
    gb.stream_status()
    assert_valid(A, s, p.cpu().numpy(), d.cpu().numpy(), what="after shutdown")
    g.free()
