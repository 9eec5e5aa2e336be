"""Helpers for GPU parity tests: run the library, check against the oracle."""
from __future__ import annotations

import collections
import os
import sys
from concurrent.futures import ThreadPoolExecutor

import numpy as np

import oracle


def say(msg: str):
    print(f"[gpu-test] {msg}", flush=True)
    sys.stdout.flush()


def device_bfs(gb, g, source, params=None, stream=None, with_depth=True):
    import torch
    parent = torch.empty(g.n, dtype=torch.int32, device="cuda")
    depth = torch.empty(g.n, dtype=torch.int32, device="cuda") if with_depth else None
    gb.bfs(g, int(source), parent, depth, stream=stream, params=params)
    torch.cuda.synchronize()
    gb.stream_status(stream)
    return parent.cpu().numpy(), (depth.cpu().numpy() if with_depth else None)


def assert_valid(A: oracle.Adjacency, source: int, parent, depth, ref=None, what=""):
    """Depth bit-exact against the oracle, parents valid (Section 2.1)."""
    dref = ref if ref is not None else A.bfs(int(source))[0]
    code, bad = A.check(int(source), dref, parent, depth)
    if code != 0:
        detail = ""
        if bad >= 0:
            detail = (f" vertex {bad}: parent={parent[bad]}"
                      + (f" depth={depth[bad]}" if depth is not None else "")
                      + f" ref_depth={dref[bad]}")
        raise AssertionError(f"{what} source={source}: {oracle.CHECK_NAMES.get(code, code)}{detail}")
    return dref


def graph_pair(gb, n, src, dst):
    """(device graph, oracle adjacency) from the same raw edge list."""
    return gb.build_csr(n, src, dst), oracle.Adjacency(n, src, dst)


def oracle_threads() -> int:
    """Host threads for oracle checks: the cores this process may use, at
    most 16 (a GPU machine's CPU share)."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def check_all(items, what=""):
    """Checks GPU results against the oracle on several host threads (the
    oracle's C calls release the GIL).  ``items`` yields (A, source,
    results) with ``results`` a list of (label, parent, depth) host arrays
    from the same source; the oracle searches once per item.  Raises on the
    first invalid result; returns the number of results checked."""
    def job(A, s, results):
        dref = A.bfs(int(s))[0]
        out = []
        for label, p, d in results:
            code, bad = A.check(int(s), dref, p, d)
            if code != 0:
                out.append(f"{what} {label} source={s}: {oracle.CHECK_NAMES.get(code, code)}"
                           + (f" vertex {bad}: parent={p[bad]} depth={None if d is None else d[bad]}"
                              f" ref_depth={dref[bad]}" if bad >= 0 else ""))
        return len(results), out

    threads = oracle_threads()
    checked = 0
    with ThreadPoolExecutor(threads) as ex:
        pending = collections.deque()

        def finish(f):
            nonlocal checked
            k, errs = f.result()
            if errs:
                raise AssertionError("; ".join(errs[:3]))
            checked += k

        for A, s, results in items:
            pending.append(ex.submit(job, A, s, results))
            while len(pending) >= 2 * threads:
                finish(pending.popleft())
        while pending:
            finish(pending.popleft())
    return checked
