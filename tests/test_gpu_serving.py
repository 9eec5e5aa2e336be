"""Serving parity: every query served in the mix (batched with others of its
graph, several launches in flight) has the depth array it has alone, and
both parent arrays are valid (Section 2.1); depths also equal the oracle's."""
import numpy as np
import pytest

import oracle
from tests.gpuutil import say

pytestmark = pytest.mark.gpu


def test_serving_mix_equals_alone(gpu):
    import torch
    from paper_1508_03619_amd import serving as sv
    pool = sv.Pool(sv.pool_spec(small=True), keep_edges=True)
    adjs = [oracle.Adjacency(el.n, el.src, el.dst) for el in pool.edges]
    # a backlog (large batches) followed by Poisson arrivals (small batches
    # and single-source launches while earlier launches run)
    qs = sv.poisson_queries(0.0, 150, pool.sources, seed=777)
    tail = sv.poisson_queries(4000.0, 150, pool.sources, seed=778, first_id=150)
    qs += tail
    results = {}

    def on_done(batch, outs):
        for q, p, d in zip(batch, *outs):
            results[q.qid] = (p.cpu().numpy(), d.cpu().numpy())

    say(f"serving {len(qs)} queries over {len(pool.graphs)} graphs, 4 slots")
    sched = sv.Scheduler(pool.sizes, budget_bytes=1 << 28, max_lanes=64)
    ex = sv.GpuExecutor(pool.graphs, slots=4, sources=pool.sources)
    try:
        done = sv.serve(ex, sched, qs, on_done)
    finally:
        ex.close()
    assert sorted(q.qid for q in done) == list(range(300))
    assert ex.launch_kinds["batch"] > 0 and ex.launch_kinds["single"] > 0, \
        f"both launch kinds must be exercised: {dict(ex.launch_kinds)}"
    say("serving: checking each query alone")
    refs = {}
    p1 = {}
    for q in done:
        A = adjs[q.graph]
        key = (q.graph, q.source)
        if key not in refs:
            refs[key] = A.bfs(q.source)[0]
        pm, dm = results[q.qid]
        assert A.check(q.source, refs[key], pm, dm)[0] == 0, f"query {q.qid} in the mix"
        g = pool.graphs[q.graph]
        if g.n not in p1:
            p1[g.n] = (torch.empty(g.n, dtype=torch.int32, device="cuda"),
                       torch.empty(g.n, dtype=torch.int32, device="cuda"))
        pa, da = p1[g.n]
        from paper_1508_03619_amd import gapbfs as gb
        gb.bfs(g, q.source, pa, da)
        torch.cuda.synchronize()
        pa_h, da_h = pa.cpu().numpy(), da.cpu().numpy()
        assert np.array_equal(da_h, dm), f"query {q.qid}: depth alone != depth in the mix"
        assert A.check(q.source, refs[key], pa_h, da_h)[0] == 0, f"query {q.qid} alone"
    pool.free()


def test_continuous_serving_mix_equals_alone(gpu):
    """Continuous batching (servers that take queries into running searches):
    every query's depths equal its depths alone and the oracle's, and both
    parent arrays are valid; a budget of 8 outputs of the largest graph makes
    admission wait."""
    import torch
    from paper_1508_03619_amd import gapbfs as gb, serving as sv
    pool = sv.Pool(sv.pool_spec(small=True), keep_edges=True)
    adjs = [oracle.Adjacency(el.n, el.src, el.dst) for el in pool.edges]
    qs = sv.poisson_queries(0.0, 120, pool.sources, seed=787)
    qs += sv.poisson_queries(3000.0, 180, pool.sources, seed=788, first_id=120)
    results = {}
    side = torch.cuda.Stream()

    def on_done(batch, outs):
        p, d = outs
        with torch.cuda.stream(side):
            results[batch[0].qid] = (p.cpu().numpy(), d.cpu().numpy())

    budget = 8 * 8 * max(pool.sizes)
    sched = sv.Scheduler(pool.sizes, budget_bytes=budget, max_lanes=64)
    ex = sv.ContinuousExecutor(pool.graphs, slots=4, lanes=64, sources=pool.sources)
    say(f"continuous: {len(qs)} queries, single-search graphs {sorted(ex.single_graphs)}")
    try:
        done = sv.serve_continuous(ex, sched, qs, on_done)
    finally:
        ex.close()
    assert sorted(q.qid for q in done) == list(range(len(qs)))
    assert ex.launch_kinds["joined"] > 0, dict(ex.launch_kinds)
    assert sched.peak_used <= budget and sched.admission_waits > 0
    pa = {}
    for q in done:
        A, g = adjs[q.graph], pool.graphs[q.graph]
        ref = A.bfs(q.source)[0]
        pm, dm = results[q.qid]
        assert A.check(q.source, ref, pm, dm)[0] == 0, f"query {q.qid} in the mix"
        if g.n not in pa:
            pa[g.n] = (torch.empty(g.n, dtype=torch.int32, device="cuda"),
                       torch.empty(g.n, dtype=torch.int32, device="cuda"))
        p1, d1 = pa[g.n]
        gb.bfs(g, q.source, p1, d1)
        torch.cuda.synchronize()
        assert np.array_equal(d1.cpu().numpy(), dm), f"query {q.qid}: alone != in the mix"
    pool.free()
