"""Serving loop host logic on a simulated clock: admission against the
memory budget, FIFO order, same-graph batching, slot limits, latency
accounting.  No device is used."""
import math

import numpy as np
import pytest

from paper_1508_03619_amd import serving as sv


def linear_service(n, lanes):
    return 1e-4 + 1e-9 * n * (1 + 0.05 * lanes)


SIZES = [1 << 10, 1 << 12, 1 << 14, 5000]


def make_queries(rate, count, seed=777):
    cands = [np.arange(n, dtype=np.int32) for n in SIZES]
    return sv.poisson_queries(rate, count, cands, seed)


class Recorder(sv.SimExecutor):
    """SimExecutor that checks the budget at every launch."""

    def __init__(self, sched, *a, **k):
        super().__init__(*a, **k)
        self.sched = sched
        self.max_used = 0

    def launch(self, slot, batch):
        assert self.sched.used <= self.sched.budget
        self.max_used = max(self.max_used, self.sched.used)
        super().launch(slot, batch)


@pytest.mark.parametrize("rate", [50.0, 2000.0, 0.0])
def test_every_query_completes_once(rate):
    qs = make_queries(rate, 500)
    sched = sv.Scheduler(SIZES, budget_bytes=64 * 8 * max(SIZES), max_lanes=16)
    ex = Recorder(sched, 3, linear_service, SIZES)
    done = sv.serve(ex, sched, qs)
    assert sorted(q.qid for q in done) == list(range(500))
    assert sched.used == 0 and sched.pending == 0
    for q in done:
        assert q.arrival <= q.start <= q.done
        assert 1 <= q.batch_size <= 16
    assert ex.max_inflight <= 3


def test_batches_hold_one_graph_in_arrival_order():
    qs = make_queries(0.0, 300, seed=5)
    sched = sv.Scheduler(SIZES, budget_bytes=1 << 30, max_lanes=8)
    ex = sv.SimExecutor(2, linear_service, SIZES)
    sv.serve(ex, sched, qs)
    byid = {q.qid: q for q in qs}
    seen = set()
    for _, _, ids in ex.launches:
        assert len({byid[i].graph for i in ids}) == 1
        assert ids == sorted(ids)        # arrival order inside a batch
        assert len(ids) <= 8
        seen.update(ids)
    assert seen == set(range(300))
    # the head of line is always in the next batch: launches start with the
    # oldest query not yet launched
    launched = set()
    for _, _, ids in ex.launches:
        oldest = min(set(range(300)) - launched)
        assert oldest in ids
        launched.update(ids)


def test_budget_is_never_exceeded_and_blocks_admission():
    # budget for only 3 outputs of the largest graph
    budget = 3 * sv.query_output_bytes(max(SIZES))
    qs = make_queries(0.0, 200, seed=9)
    sched = sv.Scheduler(SIZES, budget_bytes=budget, max_lanes=64)
    ex = Recorder(sched, 4, linear_service, SIZES)
    done = sv.serve(ex, sched, qs)
    assert len(done) == 200
    assert sched.peak_used <= budget
    assert ex.max_used <= budget
    # a budget that admits 3 large outputs cannot put 4 of them in flight
    big = [q for q in done if SIZES[q.graph] == max(SIZES)]
    assert big
    for q in big:
        overlapping = [r for r in big if r.start < q.done and q.start < r.done]
        assert len(overlapping) <= 3


def test_query_larger_than_budget_is_rejected():
    sched = sv.Scheduler(SIZES, budget_bytes=sv.query_output_bytes(SIZES[0]))
    with pytest.raises(sv.AdmissionError):
        sched.submit(sv.Query(0, 2, 0, 0.0))
    with pytest.raises(sv.AdmissionError):
        sched.submit(sv.Query(1, 7, 0, 0.0))
    with pytest.raises(sv.AdmissionError):
        sched.submit(sv.Query(2, 0, SIZES[0], 0.0))


def test_new_arrivals_do_not_wait_for_running_batches():
    # one long launch in flight; a query arriving later starts on a free slot
    sizes = [1000, 1000]
    service = lambda n, lanes: 1.0 if lanes > 1 else 0.01
    qs = [sv.Query(i, 0, i, 0.0) for i in range(4)] + [sv.Query(4, 1, 0, 0.5)]
    sched = sv.Scheduler(sizes, budget_bytes=1 << 30, max_lanes=64)
    ex = sv.SimExecutor(2, service, sizes)
    done = {q.qid: q for q in sv.serve(ex, sched, qs)}
    assert done[4].start == pytest.approx(0.5)
    assert done[4].done == pytest.approx(0.51)
    assert done[0].done == pytest.approx(1.0)


def test_latency_summary_and_poisson_rate():
    qs = make_queries(1000.0, 4000, seed=11)
    gaps = np.diff([q.arrival for q in qs])
    assert abs(gaps.mean() - 1e-3) < 1e-4            # mean inter-arrival 1/rate
    assert abs(np.std(gaps) / gaps.mean() - 1) < 0.1  # exponential: cv = 1
    counts = np.bincount([q.graph for q in qs], minlength=len(SIZES))
    assert counts.min() > 0.2 * len(qs) / len(SIZES) * 3.5
    for q in qs:
        q.start, q.done, q.batch_size = q.arrival, q.arrival + 0.002, 1
    s = sv.latency_summary(qs, skip=100)
    assert s["queries"] == 3900
    assert s["p50_ms"] == pytest.approx(2.0) and s["p99_ms"] == pytest.approx(2.0)


def test_workspace_bound_matches_layout():
    # one 64-lane segment of n vertices: 24n (bitsets) + 512n (lane staging) + 128n (queues)
    n = 1 << 16
    assert sv.batch_workspace_bytes(n, 64) == 664 * n
    assert sv.batch_workspace_bytes(n, 65) == (48 + 1024 + 128) * n
    assert sv.batch_workspace_bytes(n, 300) == 2 * (96 + 2048 + 128) * n


def test_prefer_batch_cost_model():
    # level-bound graph: a batch costs about one search -> batch from 2 lanes
    assert sv.prefer_batch(2, 10.0, {8: 12.0, 64: 20.0})
    # cheap singles, costly batches -> singles until the batch amortises
    tb = {8: 2.5, 64: 8.0}
    assert not sv.prefer_batch(4, 0.33, tb)
    assert not sv.prefer_batch(7, 0.33, tb)
    assert sv.prefer_batch(40, 0.33, tb)
    assert not sv.prefer_batch(1, 100.0, tb)       # one query: always a single search
    # interpolation between the calibrated points, extrapolation above
    assert sv.prefer_batch(36, 5.25 / 36 + 1e-3, tb)
    assert not sv.prefer_batch(36, 5.25 / 36 - 1e-3, tb)
    assert sv.prefer_batch(128, 16.0 / 128 + 1e-3, tb)
    assert not sv.prefer_batch(128, 16.0 / 128 - 1e-3, tb)


def test_closed_loop_keeps_client_count_in_flight():
    sizes = [1000, 2000]
    cands = [np.arange(n, dtype=np.int32) for n in sizes]
    pool = sv.poisson_queries(0.0, 300, cands, seed=3)
    sched = sv.Scheduler(sizes, budget_bytes=1 << 30, max_lanes=8)
    ex = sv.SimExecutor(2, linear_service, sizes)
    src = sv.ClosedArrivals(16, 300, lambda k: pool[k])
    done = sv.serve(ex, sched, src)
    assert sorted(q.qid for q in done) == list(range(300))
    # at every arrival after the first 16, exactly one query had just completed
    events = sorted([(q.arrival, 1) for q in done] + [(q.done, -1) for q in done])
    level, peak = 0, 0
    for _, dlt in events:
        level += dlt
        peak = max(peak, level)
    assert peak <= 16
    arrivals = sorted(q.arrival for q in done)
    assert arrivals[:16] == [0.0] * 16 and arrivals[16] > 0.0


# ---- continuous batching (serve_continuous) on the simulated device ----------

def sim_service(n):
    return 2e-4 + 2e-9 * n


@pytest.mark.parametrize("rate", [100.0, 5000.0, 0.0])
def test_continuous_every_query_once_within_budget(rate):
    qs = make_queries(rate, 600, seed=11)
    sched = sv.Scheduler(SIZES, budget_bytes=40 * 8 * max(SIZES), max_lanes=16)
    ex = sv.SimContinuous(3, 16, sim_service, SIZES)
    done = sv.serve_continuous(ex, sched, qs)
    assert sorted(q.qid for q in done) == list(range(600))
    assert sched.used == 0 and sched.pending == 0
    assert sched.peak_used <= sched.budget
    for q in done:
        assert q.arrival <= q.start <= q.done
    assert ex.max_lanes_used <= 16


def test_continuous_queries_join_running_searches():
    """Under a backlog most queries join a server that is already running a
    search of their graph, rather than waiting for it to finish."""
    qs = make_queries(0.0, 400, seed=12)
    sched = sv.Scheduler(SIZES, budget_bytes=1 << 30, max_lanes=64)
    ex = sv.SimContinuous(2, 64, sim_service, SIZES)
    sv.serve_continuous(ex, sched, qs)
    assert ex.joined_running > 200


def test_continuous_budget_binds_and_fifo_on_memory():
    """A budget of 3 queries of the largest graph: admission stops at the
    first query that does not fit (nothing overtakes it on memory)."""
    qs = make_queries(0.0, 200, seed=13)
    budget = 3 * 8 * max(SIZES)
    sched = sv.Scheduler(SIZES, budget_bytes=budget, max_lanes=64)
    ex = sv.SimContinuous(4, 64, sim_service, SIZES)
    done = sv.serve_continuous(ex, sched, qs)
    assert len(done) == 200 and sched.admission_waits > 0
    assert sched.peak_used <= budget


def test_continuous_closed_loop():
    cands = [np.arange(n, dtype=np.int32) for n in SIZES]
    qs = sv.poisson_queries(0.0, 300, cands, 14)
    src = sv.ClosedArrivals(10, 300, lambda k: qs[k])
    sched = sv.Scheduler(SIZES, budget_bytes=1 << 30, max_lanes=64)
    ex = sv.SimContinuous(2, 64, sim_service, SIZES)
    done = sv.serve_continuous(ex, sched, src)
    assert len(done) == 300
