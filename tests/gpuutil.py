"""Helpers for GPU parity tests: run the library, check against the oracle."""
from __future__ import annotations

import sys

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
