"""Query serving over a pool of device-resident graphs.

A query is one breadth-first search (graph, source) with the output of
Section 2.1 (parent and depth arrays).  The server keeps every graph of the
pool resident in HBM (built once, untimed, as Section 2.3 prescribes for the
graph), admits queries against a device-memory budget, groups queries of the
same graph into multi-source launches (``gap_bfs_batch``) and keeps several
launches in flight on separate HIP streams (``grid_split``: each persistent
launch takes a 1/k share of the compute units, k launches run at once).
While launches run, newly arrived queries are grouped into the next launch
of a free stream, so no query waits for a batch it did not join.

The host logic (``Scheduler``, ``serve``) is independent of the device: the
``GpuExecutor`` runs batches through the library, a ``SimExecutor`` runs the
same loop on a simulated clock for host-only tests.
"""
from __future__ import annotations

import collections
import math
import time
from dataclasses import dataclass, field
from typing import Callable, Dict, List, Optional, Sequence

import numpy as np

# ---------------------------------------------------------------------------
# memory accounting

# Device memory one multi-source launch uses per segment of 64*W lanes of a
# graph with n vertices: visit/frontier/next bitsets (3 * 8W bytes per
# vertex, rounded to 64-vertex words), per-lane parent/depth staging
# (8 bytes per lane slot), two vertex queues of 16 segments each.
# Mirrors the workspace layout of the multi-source kernel.
def batch_workspace_bytes(n: int, lanes: int) -> int:
    W = 1 if lanes <= 64 else (2 if lanes <= 128 else 4)
    segs = -(-lanes // (64 * W))
    nv = -(-n // 64) * 64
    per_seg = 3 * 8 * W * nv + 8 * 64 * W * nv + 2 * 4 * 16 * nv
    return segs * per_seg


def query_output_bytes(n: int) -> int:
    """Parent and depth arrays of one query (int32 each)."""
    return 8 * n


@dataclass
class Query:
    qid: int
    graph: int
    source: int
    arrival: float          # seconds, on the server clock
    start: float = math.nan  # launch time
    done: float = math.nan   # completion observed by the host
    batch_size: int = 0

    @property
    def latency(self) -> float:
        return self.done - self.arrival


class AdmissionError(ValueError):
    pass


class Scheduler:
    """FIFO admission against a memory budget, same-graph batching.

    ``submit`` queues a query.  ``take_batch`` forms the next launch: the
    graph of the oldest waiting query, and up to ``max_lanes`` of that
    graph's waiting queries in arrival order, as many as the budget admits.
    The oldest query is never overtaken: when its outputs do not fit, no
    batch is formed until earlier launches release memory.
    """

    def __init__(self, graph_sizes: Sequence[int], budget_bytes: int, max_lanes: int = 64):
        if max_lanes < 1:
            raise ValueError("max_lanes must be >= 1")
        self.sizes = [int(n) for n in graph_sizes]
        self.budget = int(budget_bytes)
        self.max_lanes = int(max_lanes)
        self.used = 0
        self.peak_used = 0
        self.admission_waits = 0  # walks stopped by a query that did not fit
        self._order: collections.deque = collections.deque()   # qids in arrival order
        self._by_graph: Dict[int, collections.deque] = collections.defaultdict(collections.deque)
        self._live: Dict[int, Query] = {}                       # waiting queries

    def cost(self, q: Query) -> int:
        return query_output_bytes(self.sizes[q.graph])

    @property
    def pending(self) -> int:
        return len(self._live)

    def submit(self, q: Query) -> None:
        if not (0 <= q.graph < len(self.sizes)):
            raise AdmissionError(f"query {q.qid}: graph {q.graph} not in the pool")
        if not (0 <= q.source < self.sizes[q.graph]):
            raise AdmissionError(f"query {q.qid}: source {q.source} out of range")
        if self.cost(q) > self.budget:
            raise AdmissionError(f"query {q.qid}: needs {self.cost(q)} bytes, budget {self.budget}")
        self._order.append(q.qid)
        self._by_graph[q.graph].append(q)
        self._live[q.qid] = q

    def take_batch(self) -> List[Query]:
        while self._order and self._order[0] not in self._live:
            self._order.popleft()
        if not self._order:
            return []
        head = self._live[self._order[0]]
        dq = self._by_graph[head.graph]
        batch: List[Query] = []
        while dq and len(batch) < self.max_lanes:
            q = dq[0]
            c = self.cost(q)
            if self.used + c > self.budget:
                break
            dq.popleft()
            self.used += c
            del self._live[q.qid]
            batch.append(q)
        self.peak_used = max(self.peak_used, self.used)
        return batch

    def start_each(self, start: Callable[[Query], bool]) -> int:
        """Continuous batching: walks the waiting queries in arrival order and
        calls ``start(q)`` for each one whose outputs fit the budget; a query
        that ``start`` takes is charged and leaves the queue.  A query that
        does not fit stops the walk (nothing overtakes it on memory); one that
        ``start`` refuses (no room for its graph now) is passed over.
        Returns the number of queries started."""
        started = 0
        for qid in list(self._order):
            q = self._live.get(qid)
            if q is None:
                continue
            c = self.cost(q)
            if self.used + c > self.budget:
                self.admission_waits += 1
                break
            if start(q):
                self.used += c
                self.peak_used = max(self.peak_used, self.used)
                del self._live[qid]
                self._by_graph[q.graph].remove(q)
                started += 1
        while self._order and self._order[0] not in self._live:
            self._order.popleft()
        return started

    def release(self, batch: Sequence[Query]) -> None:
        for q in batch:
            self.used -= self.cost(q)
        if self.used < 0:
            raise RuntimeError("scheduler released more memory than it admitted")


# ---------------------------------------------------------------------------
# serving loop

class OpenArrivals:
    """Queries that arrive at preset times (open loop)."""

    def __init__(self, queries: Sequence[Query]):
        self.q = sorted(queries, key=lambda q: (q.arrival, q.qid))
        self.i = 0

    def due(self, now: float) -> List[Query]:
        out = []
        while self.i < len(self.q) and self.q[self.i].arrival <= now:
            out.append(self.q[self.i])
            self.i += 1
        return out

    def completed(self, q: Query, now: float) -> None:
        pass

    def next_time(self) -> Optional[float]:
        return self.q[self.i].arrival if self.i < len(self.q) else None

    @property
    def exhausted(self) -> bool:
        return self.i >= len(self.q)


class ClosedArrivals:
    """``clients`` clients, each sending its next query the moment its
    previous one completes, ``total`` queries in all (closed loop).
    ``make(k)`` builds query k; its arrival time is set on release."""

    def __init__(self, clients: int, total: int, make: Callable[[int], Query]):
        self.make = make
        self.total = total
        self.sent = 0
        self.ready: List[float] = [0.0] * min(clients, total)

    def due(self, now: float) -> List[Query]:
        out = []
        while self.ready and self.sent < self.total:
            self.ready.pop()
            q = self.make(self.sent)
            q.arrival = now
            self.sent += 1
            out.append(q)
        return out

    def completed(self, q: Query, now: float) -> None:
        if self.sent < self.total:
            self.ready.append(now)

    def next_time(self) -> Optional[float]:
        return None

    @property
    def exhausted(self) -> bool:
        return self.sent >= self.total


def serve(ex, sched: Scheduler, queries, on_done: Optional[Callable] = None) -> List[Query]:
    """Run every query to completion.  ``queries`` is a list of queries with
    arrival times on the executor's clock (seconds from the start of the
    call), or an arrival source (OpenArrivals / ClosedArrivals)."""
    src = queries if hasattr(queries, "due") else OpenArrivals(queries)
    inflight: Dict[int, List[Query]] = {}
    free = list(range(ex.slots))[::-1]
    finished: List[Query] = []
    ex.start()
    while not src.exhausted or sched.pending or inflight:
        progressed = False
        now = ex.now()
        for q in src.due(now):
            sched.submit(q)
            progressed = True
        for slot in list(inflight):
            if ex.poll(slot):
                t = ex.now()
                batch = inflight.pop(slot)
                for q in batch:
                    q.done = t
                if on_done is not None:
                    on_done(batch, ex.outputs(slot))
                ex.retire(slot)
                sched.release(batch)
                free.append(slot)
                finished.extend(batch)
                for q in batch:
                    src.completed(q, t)
                progressed = True
        while free:
            batch = sched.take_batch()
            if not batch:
                break
            slot = free.pop()
            t = ex.now()
            for q in batch:
                q.start = t
                q.batch_size = len(batch)
            ex.launch(slot, batch)
            inflight[slot] = batch
            progressed = True
        if not progressed:
            ex.idle(src.next_time())
    return finished


def serve_continuous(ex, sched: Scheduler, queries, on_done: Optional[Callable] = None) -> List[Query]:
    """Continuous batching: every admitted query starts as soon as the
    executor can take it (``ex.try_start``: it joins a running search of its
    graph at the next level boundary, or starts on an idle slot) and
    completes on its own (``ex.poll_done``).  Same arrival sources and
    budget accounting as ``serve``."""
    src = queries if hasattr(queries, "due") else OpenArrivals(queries)
    finished: List[Query] = []
    inflight = 0
    ex.start()
    while not src.exhausted or sched.pending or inflight:
        progressed = False
        now = ex.now()
        for q in src.due(now):
            sched.submit(q)
            progressed = True
        for q, outs in ex.poll_done():
            q.done = ex.now()
            sched.release([q])
            inflight -= 1
            finished.append(q)
            src.completed(q, q.done)
            if on_done is not None:
                on_done([q], outs)
            progressed = True
        started = sched.start_each(lambda q: ex.try_start(q, ex.now()))
        if started:
            inflight += started
            progressed = True
        if not progressed:
            ex.idle(src.next_time())
    return finished


def latency_summary(done: Sequence[Query], skip: int = 0) -> dict:
    """p50/p99/mean latency (ms) and throughput over queries after ``skip``
    warm-up queries (in arrival order)."""
    qs = sorted(done, key=lambda q: (q.arrival, q.qid))[skip:]
    if not qs:
        return {"queries": 0}
    lat = np.array([q.latency for q in qs]) * 1e3
    span = max(q.done for q in qs) - min(q.arrival for q in qs)
    return {"queries": len(qs),
            "p50_ms": float(np.percentile(lat, 50)),
            "p99_ms": float(np.percentile(lat, 99)),
            "mean_ms": float(lat.mean()),
            "max_ms": float(lat.max()),
            "throughput_qps": len(qs) / span if span > 0 else float("inf"),
            "mean_batch": float(np.mean([q.batch_size for q in qs]))}


# ---------------------------------------------------------------------------
# workload: arrivals

def poisson_queries(rate: float, count: int, graph_sources: Sequence[np.ndarray], seed: int,
                    first_id: int = 0) -> List[Query]:
    """``count`` queries with exponential inter-arrival times of mean 1/rate
    (rate <= 0 or inf: every query arrives at time 0, the closed backlog used
    to measure saturation throughput).  Graph uniform over the pool, source
    uniform over that graph's candidate vertices (``graph_sources[g]``)."""
    rng = np.random.default_rng(seed)
    if rate > 0 and math.isfinite(rate):
        t = np.cumsum(rng.exponential(1.0 / rate, count))
    else:
        t = np.zeros(count)
    gs = rng.integers(0, len(graph_sources), count)
    out = []
    for k in range(count):
        cand = graph_sources[int(gs[k])]
        s = int(cand[int(rng.integers(0, len(cand)))])
        out.append(Query(first_id + k, int(gs[k]), s, float(t[k])))
    return out


def nonzero_degree_vertices(n: int, src: np.ndarray, dst: np.ndarray) -> np.ndarray:
    """Vertices with at least one edge to another vertex (query sources)."""
    keep = src != dst
    deg = np.bincount(src[keep], minlength=n) + np.bincount(dst[keep], minlength=n)
    return np.nonzero(deg)[0].astype(np.int32)


# ---------------------------------------------------------------------------
# executors

class SimExecutor:
    """Simulated device for host-only tests: a launch of L lanes on a graph
    of n vertices takes ``service(n, L)`` seconds of simulated time, and
    ``slots`` launches may run at once."""

    def __init__(self, slots: int, service: Callable[[int, int], float], sizes: Sequence[int]):
        self.slots = slots
        self.service = service
        self.sizes = list(sizes)
        self.t = 0.0
        self.finish: Dict[int, float] = {}
        self.batches: Dict[int, List[Query]] = {}
        self.max_inflight = 0
        self.launches: List[tuple] = []

    def start(self):
        self.t = 0.0

    def now(self) -> float:
        return self.t

    def launch(self, slot: int, batch: List[Query]):
        assert slot not in self.finish, "launch on a busy slot"
        n = self.sizes[batch[0].graph]
        self.finish[slot] = self.t + self.service(n, len(batch))
        self.batches[slot] = batch
        self.max_inflight = max(self.max_inflight, len(self.finish))
        self.launches.append((self.t, slot, [q.qid for q in batch]))

    def poll(self, slot: int) -> bool:
        return self.finish[slot] <= self.t

    def outputs(self, slot: int):
        return None

    def retire(self, slot: int):
        del self.finish[slot]
        del self.batches[slot]

    def idle(self, next_arrival: Optional[float]):
        cands = list(self.finish.values())
        if next_arrival is not None:
            cands.append(next_arrival)
        if not cands:
            raise RuntimeError("serving loop idle with nothing pending")
        self.t = max(self.t, min(cands))


CALIBRATION_LANES = (8, 64)


def prefer_batch(lanes: int, t_single: float, t_batch: Dict[int, float]) -> bool:
    """True when one multi-source launch of ``lanes`` queries is expected to
    finish sooner than ``lanes`` single-source searches in a row.  The batch
    time is interpolated linearly in the lane count between the calibrated
    points (and held flat below the first)."""
    if lanes <= 1:
        return False
    pts = sorted(t_batch.items())
    if lanes <= pts[0][0]:
        tb = pts[0][1]
    elif lanes >= pts[-1][0]:
        tb = pts[-1][1] * lanes / pts[-1][0]
    else:
        tb = pts[-1][1]
        for (l0, t0), (l1, t1) in zip(pts, pts[1:]):
            if l0 <= lanes <= l1:
                tb = t0 + (t1 - t0) * (lanes - l0) / (l1 - l0)
                break
    return tb < lanes * t_single


class GpuExecutor:
    """Runs batches through the library on ``slots`` HIP streams.

    Each launch slot has its own stream; with grid_split = slots every
    persistent launch takes 1/slots of the compute units, so launches on
    different slots overlap.  A batch of queries on one graph runs either as
    one multi-source launch or as single-source searches in a row on the
    slot's stream, whichever the graph's calibration (``calibrate``) says is
    faster.  Outputs are allocated on the slot's stream when the batch is
    launched and released when the host retires it.
    """

    def __init__(self, graphs: Sequence, slots: int = 8, sources: Optional[Sequence] = None):
        import torch
        from . import gapbfs as gb
        self.torch = torch
        self.gb = gb
        self.graphs = list(graphs)
        self.slots = int(slots)
        self._saved_params = gb.get_params()
        gb.set_params(grid_split=self.slots)
        self.streams = [torch.cuda.Stream() for _ in range(self.slots)]
        self.events = [torch.cuda.Event() for _ in range(self.slots)]
        self.out: Dict[int, tuple] = {}
        self.t0 = 0.0
        self.launch_kinds = collections.Counter()
        # per graph: single-search time and batch times (ms); unknown -> batch
        self.t_single: List[float] = [math.inf] * len(self.graphs)
        self.t_batch: List[Dict[int, float]] = [{1: 0.0} for _ in self.graphs]
        if sources is not None:
            self.calibrate(sources)

    def calibrate(self, sources: Sequence[np.ndarray], reps: int = 2):
        """Time one single-source search and batches of CALIBRATION_LANES
        lanes on every graph, on one slot (the share of the device a launch
        gets while serving)."""
        torch, gb = self.torch, self.gb
        st = self.streams[0]
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)

        def timed(fn):
            with torch.cuda.stream(st):
                fn()
                best = math.inf
                for _ in range(reps):
                    e0.record(st)
                    fn()
                    e1.record(st)
                    e1.synchronize()
                    best = min(best, e0.elapsed_time(e1))
            return best

        for gi, g in enumerate(self.graphs):
            cand = sources[gi]
            L = max(CALIBRATION_LANES)
            srcs = [int(cand[(k * 7919) % len(cand)]) for k in range(L)]
            with torch.cuda.stream(st):
                ps = [torch.empty(g.n, dtype=torch.int32, device="cuda") for _ in range(L)]
                ds = [torch.empty(g.n, dtype=torch.int32, device="cuda") for _ in range(L)]
            self.t_single[gi] = timed(lambda: gb.bfs(g, srcs[0], ps[0], ds[0], stream=st))
            self.t_batch[gi] = {l: timed(lambda l=l: gb.bfs_batch([g], [0] * l, srcs[:l], ps[:l], ds[:l],
                                                                  stream=st))
                                for l in CALIBRATION_LANES}
            del ps, ds
        torch.cuda.synchronize()

    def start(self):
        self.torch.cuda.synchronize()
        self.t0 = time.perf_counter()

    def now(self) -> float:
        return time.perf_counter() - self.t0

    def launch(self, slot: int, batch: List[Query]):
        torch, gb = self.torch, self.gb
        st = self.streams[slot]
        g = self.graphs[batch[0].graph]
        with torch.cuda.stream(st):
            ps = [torch.empty(g.n, dtype=torch.int32, device="cuda") for _ in batch]
            ds = [torch.empty(g.n, dtype=torch.int32, device="cuda") for _ in batch]
            gi = batch[0].graph
            if prefer_batch(len(batch), self.t_single[gi], self.t_batch[gi]):
                gb.bfs_batch([g], [0] * len(batch), [q.source for q in batch], ps, ds, stream=st)
                self.launch_kinds["batch"] += 1
            else:
                self.launch_kinds["single"] += len(batch)
                for q, p, d in zip(batch, ps, ds):
                    gb.bfs(g, q.source, p, d, stream=st)
            self.events[slot].record(st)
        self.out[slot] = (ps, ds)

    def poll(self, slot: int) -> bool:
        return self.events[slot].query()

    def outputs(self, slot: int):
        return self.out[slot]

    def retire(self, slot: int):
        del self.out[slot]

    def close(self):
        """Wait for the streams and restore the process-wide parameters."""
        self.torch.cuda.synchronize()
        self.out.clear()
        self.gb.set_params(**self._saved_params)

    def idle(self, next_arrival: Optional[float]):
        # spin briefly: launches complete within tens of microseconds to
        # milliseconds, and the host clock decides the latency measured
        if next_arrival is not None:
            wait = next_arrival - self.now()
            if wait > 2e-4:
                time.sleep(min(wait, 1e-3) * 0.5)


class SimContinuous:
    """Simulated device for host tests of ``serve_continuous``: ``slots``
    servers of ``lanes`` lanes; a query joining a server runs for
    ``service(n)`` seconds from its start (lanes are independent), and a
    server is bound to one graph while it holds queries."""

    def __init__(self, slots: int, lanes: int, service: Callable[[int], float], sizes: Sequence[int]):
        self.slots, self.lanes, self.service, self.sizes = slots, lanes, service, list(sizes)
        self.t = 0.0
        self.bound: List[Optional[int]] = [None] * slots
        self.held: List[Dict[int, tuple]] = [dict() for _ in range(slots)]
        self.max_lanes_used = 0
        self.joined_running = 0

    def start(self):
        self.t = 0.0

    def now(self) -> float:
        return self.t

    def try_start(self, q: Query, t: float) -> bool:
        order = [s for s in range(self.slots) if self.bound[s] == q.graph] + \
                [s for s in range(self.slots) if not self.held[s]]
        for s in order:
            if len(self.held[s]) >= self.lanes:
                continue
            if self.held[s]:
                self.joined_running += 1
            self.bound[s] = q.graph
            q.start = t
            q.batch_size = len(self.held[s]) + 1
            self.held[s][q.qid] = (q, t + self.service(self.sizes[q.graph]))
            self.max_lanes_used = max(self.max_lanes_used, len(self.held[s]))
            return True
        return False

    def poll_done(self):
        out = []
        for s in range(self.slots):
            for qid, (q, end) in list(self.held[s].items()):
                if end <= self.t:
                    del self.held[s][qid]
                    out.append((q, None))
            if not self.held[s]:
                self.bound[s] = None
        return out

    def idle(self, next_arrival: Optional[float]):
        cands = [end for h in self.held for (_, end) in h.values()]
        if next_arrival is not None:
            cands.append(next_arrival)
        if not cands:
            raise RuntimeError("serving loop idle with nothing pending")
        self.t = max(self.t, min(cands))


class ContinuousExecutor:
    """Continuous batching on the device: ``slots`` servers (gap_serve_*), one
    HIP stream each, every one bound to one graph while it holds queries; a
    query joins its graph's running search at the next level boundary (up to
    ``lanes`` at once), or binds an idle server.  Graphs whose one-query
    serving time is far above a single-source search (high diameter: a
    serving level costs a dense pass over the vertices) run as single-source
    searches on an idle slot instead (``calibrate``).  With grid_split =
    slots every launch takes 1/slots of the compute units, so all slots run
    at once."""

    def __init__(self, graphs: Sequence, slots: int = 8, lanes: int = 64,
                 sources: Optional[Sequence] = None):
        import torch
        from . import gapbfs as gb
        self.torch, self.gb = torch, gb
        self.graphs = list(graphs)
        self.slots, self.lanes = int(slots), int(lanes)
        self._saved_params = gb.get_params()
        gb.set_params(grid_split=self.slots)
        self.streams = [torch.cuda.Stream() for _ in range(self.slots)]
        maxn = max(g.n for g in self.graphs)
        maxe = max(g.nnz for g in self.graphs)
        self.servers = [gb.Server(maxn, maxe, stream=st) for st in self.streams]
        self.bound: List[Optional[int]] = [None] * self.slots
        self.held: List[Dict[int, tuple]] = [dict() for _ in range(self.slots)]
        self.single: Dict[int, tuple] = {}  # slot -> (query, parent, depth, event)
        self.single_graphs: set = set()
        self.t0 = 0.0
        self.launch_kinds = collections.Counter()
        self.t_single: Dict[int, float] = {}
        self.t_serve: Dict[int, float] = {}
        if sources is not None:
            self.calibrate(sources)

    def calibrate(self, sources: Sequence[np.ndarray], reps: int = 2):
        """Per graph: one single-source search and one query through a
        server (best of ``reps``, host clock); graphs whose served query takes
        more than twice the single search run as single searches."""
        torch, gb = self.torch, self.gb
        st, srv = self.streams[0], self.servers[0]
        for gi, g in enumerate(self.graphs):
            s = int(sources[gi][0])
            p = torch.empty(g.n, dtype=torch.int32, device="cuda")
            d = torch.empty(g.n, dtype=torch.int32, device="cuda")
            best_single = best_serve = math.inf
            for _ in range(reps + 1):
                t = time.perf_counter()
                gb.bfs(g, s, p, d, stream=st)
                st.synchronize()
                best_single = min(best_single, time.perf_counter() - t)
                t = time.perf_counter()
                if not srv.submit(g, -1, s, p, d):
                    raise RuntimeError("calibration: the server refused a query")
                deadline = time.perf_counter() + 30.0
                while not srv.poll():
                    if time.perf_counter() > deadline:
                        raise RuntimeError("calibration: a served query did not complete in 30 s")
                st.synchronize()
                best_serve = min(best_serve, time.perf_counter() - t)
            self.t_single[gi], self.t_serve[gi] = best_single, best_serve
            if best_serve > 2.0 * best_single:
                self.single_graphs.add(gi)
            del p, d
        gb.stream_status(st)

    def start(self):
        self.torch.cuda.synchronize()
        self.t0 = time.perf_counter()

    def now(self) -> float:
        return time.perf_counter() - self.t0

    def _idle_slot(self) -> Optional[int]:
        for s in range(self.slots):
            if not self.held[s] and s not in self.single:
                return s
        return None

    def try_start(self, q: Query, t: float) -> bool:
        torch, gb = self.torch, self.gb
        g = self.graphs[q.graph]
        if q.graph in self.single_graphs:
            s = self._idle_slot()
            if s is None:
                return False
            p = torch.empty(g.n, dtype=torch.int32, device="cuda")
            d = torch.empty(g.n, dtype=torch.int32, device="cuda")
            gb.bfs(g, q.source, p, d, stream=self.streams[s])
            ev = torch.cuda.Event()
            ev.record(self.streams[s])
            self.single[s] = (q, p, d, ev)
            q.start, q.batch_size = t, 1
            self.launch_kinds["single"] += 1
            return True
        cands = [s for s in range(self.slots) if self.bound[s] == q.graph and len(self.held[s]) < self.lanes]
        if not cands:
            s = self._idle_slot()
            if s is None:
                return False
            cands = [s]
        s = cands[0]
        p = torch.empty(g.n, dtype=torch.int32, device="cuda")
        d = torch.empty(g.n, dtype=torch.int32, device="cuda")
        if not self.servers[s].submit(g, q.qid, q.source, p, d):
            return False
        self.launch_kinds["joined" if self.held[s] else "fresh"] += 1
        self.bound[s] = q.graph
        self.held[s][q.qid] = (q, p, d)
        q.start, q.batch_size = t, len(self.held[s])
        return True

    def poll_done(self):
        out = []
        for s in range(self.slots):
            if self.held[s]:
                for qid in self.servers[s].poll():
                    q, p, d = self.held[s].pop(qid)
                    out.append((q, (p, d)))
                if not self.held[s]:
                    self.bound[s] = None
            if s in self.single and self.single[s][3].query():
                q, p, d, _ = self.single.pop(s)
                out.append((q, (p, d)))
        return out

    def idle(self, next_arrival: Optional[float]):
        if next_arrival is not None:
            wait = next_arrival - self.now()
            if wait > 2e-4:
                time.sleep(min(wait, 1e-3) * 0.5)

    def close(self):
        """Wait for every slot, check the streams' status, release the servers
        and restore the process-wide parameters."""
        self.torch.cuda.synchronize()
        for st in self.streams:
            self.gb.stream_status(st)
        for srv in self.servers:
            srv.close()
        self.gb.set_params(**self._saved_params)


# ---------------------------------------------------------------------------
# resident pool

def pool_spec(small: bool = False) -> List[tuple]:
    """The serving pool: R-MAT scales 14..20 with 3 seeds each and scales 21
    and 22 with 2 seeds each (25 graphs), and road-like grids of side 512,
    768, ..., 2048 (7 graphs).  ``small`` gives a 6-graph pool for tests."""
    if small:
        return [("rmat", 10, 50000), ("rmat", 11, 50001), ("rmat", 12, 50002),
                ("grid", 48, 50003), ("grid", 80, 50004), ("rmat", 9, 50005)]
    spec, j = [], 0
    for scale in range(14, 21):
        for _ in range(3):
            spec.append(("rmat", scale, 50000 + j))
            j += 1
    for scale in (21, 22):
        for _ in range(2):
            spec.append(("rmat", scale, 50000 + j))
            j += 1
    for side in (512, 768, 1024, 1280, 1536, 1792, 2048):
        spec.append(("grid", side, 50000 + j))
        j += 1
    return spec


def pool_edges(kind: str, size: int, seed: int):
    from . import inputs
    if kind == "rmat":
        return inputs.rmat(size, 16, seed=seed)
    if kind == "grid":
        return inputs.grid(size, size, seed=seed)
    if kind == "urand":
        return inputs.urand_scale(size, 16, seed=seed)
    raise KeyError(kind)


class Pool:
    """Graphs of ``spec`` built into device memory, with the candidate
    sources of each (vertices of non-zero degree)."""

    def __init__(self, spec: Sequence[tuple], keep_edges: bool = False):
        from . import gapbfs as gb
        self.spec = list(spec)
        self.graphs, self.sources, self.edges = [], [], []
        for kind, size, seed in self.spec:
            el = pool_edges(kind, size, seed)
            self.graphs.append(gb.build_csr(el.n, el.src, el.dst))
            self.sources.append(nonzero_degree_vertices(el.n, el.src, el.dst))
            self.edges.append(el if keep_edges else None)

    @property
    def sizes(self) -> List[int]:
        return [g.n for g in self.graphs]

    def workspace_bytes(self, slots: int, max_lanes: int) -> int:
        """Upper bound of the library workspaces the serving streams hold."""
        return slots * batch_workspace_bytes(max(self.sizes), max_lanes)

    def free(self):
        for g in self.graphs:
            g.free()
        self.graphs = []
