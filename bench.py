"""Benchmark: direction-optimizing BFS GTEPS on one MI355X.

Workload (one "step"): 64 single-source direction-optimizing searches on an
R-MAT scale-22 graph (edge factor 16, a=.57 b=.19 c=.19) and 64 on a
uniform-random graph with 2^22 vertices and 16*2^22 raw pairs, each from
seeded random non-zero-degree sources (the paper's 64-trial protocol).
Graphs are generated and built before timing (graph building is untimed in
the paper's methodology) and stay resident in HBM.

GTEPS = sum over trials of m_s / elapsed, where m_s is the number of
undirected edges in the source's connected component.

Also reported, outside the timed steps: a 64-lane batched search over the
same sources (per-source throughput vs repeated single-source searches), the
same R-MAT pairs taken as a directed graph, betweenness centrality from 4
sources, shortest paths with weights 1..255, connected components, the
serving loop, the measured
stream-copy bandwidth, the roofline of the dominant kernel and the CPU
oracle timed on a bounded sample.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, published


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


PROFILE_COPY_BYTES = 1 << 30


def algorithmic_bytes(recs, n, directed=False) -> int:
    """Bytes the search must move (per launch), from per-level records.

    init: row_ptr read 8(n+1), parent+depth written 8n
    top-down level, frontier F, N_F edges, C claimed:
        4|F| queue + 16|F| row_ptr + 4 N_F col + 4 N_F parent probes + 12|C|
    bottom-up level, U unvisited, S_U scanned entries, H found:
        16|U| row_ptr + 4 S_U col + 3 n/8 bitmaps + 8|H|
    switch to bottom-up: 4|F| + n/8; switch back to top-down (the frontier
    bitmap becomes the queue): 20|F| + n/8; final pass: 8n
    directed graphs add, per bottom-up level, 16|H| for the out-degrees of
    the found vertices, and at the switch 16|U| for the in-degree test
    """
    total = 8 * (n + 1) + 8 * n + 8 * n
    prev_dir = 1
    for r in recs:
        if r["direction"] == 1:
            if prev_dir == 2:
                total += 20 * r["frontier"] + n // 8
            total += 20 * r["frontier"] + 8 * r["frontier_edges"] + 12 * r["claimed"]
        else:
            if prev_dir == 1:
                total += 4 * r["frontier"] + n // 8
                if directed:
                    total += 16 * r["unvisited"]
            total += 16 * r["unvisited"] + 4 * r["scanned"] + 3 * n // 8 + 8 * r["claimed"]
            if directed:
                total += 16 * r["claimed"]
        prev_dir = r["direction"]
    return int(total)


def batch_algorithmic_bytes(recs, n, lanes) -> int:
    """Bytes one multi-source launch must move, from its per-level records
    (W = ceil(lanes / 64) 64-bit words per vertex for each bitset, S = lanes):
    init 24 W n (visited and frontier cleared, next cleared by the first
    advance); outputs 8 S n, written once; every level's dense advance
    24 W n (visited |= frontier, frontier read, next cleared);
    top-down level, A frontier vertices with N_A edges:
        8 W |A| (their frontier words) + 16 |A| (row offsets)
        + N_A (4 + 8 W) (column entry and the neighbour's visited word);
    bottom-up level, U searched vertices, S_U scanned entries:
        16 |U| (row offsets) + 16 W |U| (visited and next words)
        + S_U (4 + 8 W) (column entry and the neighbour's frontier word)."""
    W = max(1, -(-int(lanes) // 64))
    total = 24 * W * n + 8 * int(lanes) * n
    for r in recs:
        total += 24 * W * n
        if r["direction"] == 1:
            total += 8 * W * r["frontier"] + 16 * r["frontier"] + r["frontier_edges"] * (4 + 8 * W)
        else:
            total += 16 * r["unvisited"] + 16 * W * r["unvisited"] + r["scanned"] * (4 + 8 * W)
    return int(total)


class GraphCase:
    def __init__(self, name, el, gb, torch, nsrc, src_seed):
        from paper_1508_03619_amd import inputs
        t0 = time.time()
        self.name = name
        self.el = el
        self.g = gb.build_csr(el.n, el.src, el.dst)
        self.sources = inputs.pick_sources(el, nsrc, seed=src_seed)
        rp, _ = self.g.export_row_ptr()
        self.deg = np.diff(rp)
        # m_s and reach from the raw pairs (scipy), not from any GPU output
        rdeg, self.lab, self.comp_size, comp_edges = raw_components(el)
        if not np.array_equal(rdeg, self.deg):
            raise SystemExit(f"{name}: device CSR degrees differ from the raw edge list's")
        self.ms = np.array([comp_edges[self.lab[s]] for s in self.sources], np.int64)
        self.parent = torch.empty(self.g.n, dtype=torch.int32, device="cuda")
        self.depth = torch.empty(self.g.n, dtype=torch.int32, device="cuda")
        log(f"{name}: n={self.g.n} nnz={self.g.nnz} max_deg={int(self.deg.max())} "
            f"built in {time.time() - t0:.1f}s")


def committed_traffic(kernel):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter
    summary, if it was taken from the current kernel sources; else None."""
    tpath = os.path.join(ROOT, "profiles", f"traffic_{kernel}_rmat22_urand22.txt")
    if not os.path.exists(tpath):
        return None
    from paper_1508_03619_amd.rocprof_summary import kernel_source_hash
    try:
        tj = json.load(open(tpath))
        if tj.get("source_hash") == kernel_source_hash(kernel):
            return int(tj.get("bytes_per_launch"))
    except (OSError, ValueError, TypeError):
        pass
    return None


def raw_components(el):
    """From the raw pairs alone (scipy, independent of the library): the
    degree of every vertex in the cleaned undirected graph (distinct
    neighbours other than itself), its connected-component label, and per
    component the vertex count and the undirected edge count."""
    import scipy.sparse as sp
    from scipy.sparse.csgraph import connected_components
    keep = el.src != el.dst
    a, b = el.src[keep], el.dst[keep]
    A = sp.coo_matrix((np.ones(2 * a.size, np.int8), (np.concatenate([a, b]), np.concatenate([b, a]))),
                      shape=(el.n, el.n)).tocsr()  # duplicates merge: one entry per neighbour
    deg = np.diff(A.indptr).astype(np.int64)
    ncomp, lab = connected_components(A, directed=False)
    size = np.bincount(lab, minlength=ncomp).astype(np.int64)
    edges = (np.bincount(lab, weights=deg, minlength=ncomp) // 2).astype(np.int64)
    return deg, lab, size, edges


def component_edges(g, el):
    """Per-vertex count of undirected edges in its connected component (m_s
    of a search from that vertex), from the raw pairs; fails if the device
    CSR's degrees differ from the raw graph's."""
    deg, lab, _, edges = raw_components(el)
    rp, _ = g.export_row_ptr()
    if not np.array_equal(np.diff(rp), deg):
        raise SystemExit("device CSR degrees differ from the raw edge list's")
    return edges[lab]


def time_launches(torch, stream, fn, reps=3):
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    fn()
    torch.cuda.synchronize()
    best = float("inf")
    for _ in range(reps):
        e0.record(stream)
        fn()
        e1.record(stream)
        e1.synchronize()
        best = min(best, e0.elapsed_time(e1))
    return best


def leg_grid(gb, torch, inputs, stream):
    """4096^2 road-like grid: 64 single-source searches, persistent kernel vs
    captured level graphs (level count and time per level)."""
    t0 = time.time()
    el = inputs.workload("grid4096")
    g = gb.build_csr(el.n, el.src, el.dst)
    srcs = [int(x) for x in inputs.pick_sources(el, 64, seed=inputs.SOURCE_SEEDS["grid4096"])]
    ce = component_edges(g, el)
    p = torch.empty(g.n, dtype=torch.int32, device="cuda")
    d = torch.empty(g.n, dtype=torch.int32, device="cuda")
    levels = []
    for s in srcs[:8]:
        levels.append(len(gb.bfs(g, s, p, d, stats=True, max_levels=1 << 16)))
    out = {"n": g.n, "nnz": g.nnz, "levels_mean_first8": float(np.mean(levels)),
           "build_s": round(time.time() - t0, 1)}
    ms = sum(int(ce[s]) for s in srcs)
    for mode, label in ((0, "persistent"), (2, "graph")):
        prm = {"mode": mode}
        gb.bfs(g, srcs[0], p, d, params=prm)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for s in srcs:
            gb.bfs(g, s, p, d, params=prm)
        e1.record(stream)
        e1.synchronize()
        t = e0.elapsed_time(e1)
        out[label] = {"ms_per_search": round(t / len(srcs), 3), "gteps": round(ms / (t * 1e-3) / 1e9, 3),
                      "us_per_level": round(t / len(srcs) / np.mean(levels) * 1e3, 2)}
        log(f"grid4096 {label}: {out[label]}")
    g.free()
    return out


def leg_rmat24(gb, torch, inputs, stream):
    """R-MAT scale 24: batches of 64 and 256 sources vs the same sources one
    by one (per-source throughput)."""
    el = inputs.workload("rmat24")
    g = gb.build_csr(el.n, el.src, el.dst)
    srcs = [int(x) for x in inputs.pick_sources(el, 256, seed=inputs.SOURCE_SEEDS["rmat24"])]
    ce = component_edges(g, el)
    del el
    out = {"n": g.n, "nnz": g.nnz}
    p1 = torch.empty(g.n, dtype=torch.int32, device="cuda")
    d1 = torch.empty(g.n, dtype=torch.int32, device="cuda")
    single = time_launches(torch, stream, lambda: [gb.bfs(g, s, p1, d1) for s in srcs[:64]], reps=2)
    for L in (64, 256):
        P = [torch.empty(g.n, dtype=torch.int32, device="cuda") for _ in range(L)]
        D = [torch.empty(g.n, dtype=torch.int32, device="cuda") for _ in range(L)]
        t = time_launches(torch, stream, lambda: gb.bfs_batch([g], [0] * L, srcs[:L], P, D), reps=2)
        ms = sum(int(ce[s]) for s in srcs[:L])
        out[f"batch{L}"] = {"ms": round(t, 3), "gteps": round(ms / (t * 1e-3) / 1e9, 2),
                            "output_floor_ms": round(8 * L * g.n / HBM_PEAK_GBS / 1e6, 3)}
        del P, D
        torch.cuda.empty_cache()
    ms64 = sum(int(ce[s]) for s in srcs[:64])
    out["single64"] = {"ms_sum": round(single, 3), "gteps": round(ms64 / (single * 1e-3) / 1e9, 2)}
    out["batch64_speedup_vs_single"] = round(single / out["batch64"]["ms"], 2)
    log(f"rmat24: {out}")
    g.free()
    return out


def leg_directed(gb, torch, inputs, stream):
    """R-MAT scale 22 with the pairs taken as directed edges (out-lists for
    top-down, in-lists for bottom-up): 64 single-source searches from
    sources with an out-edge.  m_s is the number of directed edges leaving
    the reached vertices (every one of them is examined)."""
    t0 = time.time()
    name = "rmat22d"
    el = inputs.workload(name)
    g = gb.build_csr(el.n, el.src, el.dst, directed=True)
    srcs = [int(x) for x in inputs.pick_sources(el, 64, seed=inputs.SOURCE_SEEDS[name], directed=True)]
    del el
    outdeg = np.diff(g.export_row_ptr()[0])
    p = torch.empty(g.n, dtype=torch.int32, device="cuda")
    d = torch.empty(g.n, dtype=torch.int32, device="cuda")
    ms, alg, levels = [], [], []
    for s in srcs:
        recs = gb.bfs(g, s, p, d, stats=True)
        dd = d.cpu().numpy()
        ms.append(int(outdeg[dd >= 0].sum()))
        alg.append(algorithmic_bytes(recs, g.n, directed=True))
        levels.append(len(recs))
    build_s = time.time() - t0
    pairs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in srcs]
    best = None
    for rep in range(3):  # warm-up, then the better of two timed passes
        for i, s in enumerate(srcs):
            pairs[i][0].record(stream)
            gb.bfs(g, s, p, d, stream=stream)
            pairs[i][1].record(stream)
        torch.cuda.synchronize()
        t = np.array([a.elapsed_time(b) for a, b in pairs])
        if rep > 0 and (best is None or t.sum() < best.sum()):
            best = t
    ms = np.array(ms, np.int64)
    out = {"n": int(g.n), "nnz_out": int(g.nnz), "build_and_stats_s": round(build_s, 1),
           "gteps_aggregate": round(float(ms.sum() / (best.sum() * 1e-3) / 1e9), 3),
           "gteps_median_trial": round(float(np.median(ms / (best * 1e-3) / 1e9)), 3),
           "trial_ms_median": round(float(np.median(best)), 4),
           "levels_mean": round(float(np.mean(levels)), 1),
           "mean_m_s": float(ms.mean()),
           "alg_gbs_median": round(float(np.median(np.array(alg) / (best * 1e-3) / 1e9)), 1)}
    log(f"{name}: {out}")
    g.free()
    return out


def bc_bytes(A_rp, A_col, rows, depth, directed_in=None):
    """Algorithmic bytes of the betweenness passes for one source (on top of
    the search): grouping, path counts over in-lists, dependencies over
    out-lists, accumulation.  Per reached vertex at depth >= 1 the forward
    pass reads its list offsets (16), its order slot (4), col and depth of
    every in-list entry (8 each) and sigma of every predecessor (8), and
    stores sigma (8); per reached vertex below the deepest level the
    backward pass reads offsets, order slot, col and depth of every out-list
    entry and the 16-byte (sigma, S) pair of every successor, and stores S.
    Grouping reads depth and list offsets twice and writes the order; the
    accumulation reads the order, the pair and updates the score."""
    n = len(depth)
    reached = depth >= 0
    R = int(reached.sum())
    D = int(depth.max())
    deg = np.diff(A_rp)
    du, dv = depth[rows], depth[A_col]
    succ = (du >= 0) & (dv == du + 1)           # out-list entries u -> v one level down
    n_succ = np.bincount(rows[succ], minlength=n)
    # every successor edge is a predecessor edge seen from the other end
    fwd_v = reached & (depth >= 1)
    bwd_v = reached & (depth < D)
    deg_in = np.diff(directed_in) if directed_in is not None else deg
    total = 20 * n + 2 * (4 * n + 16 * n) + 4 * R
    total += int(fwd_v.sum()) * 28 + 8 * int(deg_in[fwd_v].sum()) + 8 * int(succ.sum())
    total += int(bwd_v.sum()) * 28 + 8 * int(deg[bwd_v].sum()) + 16 * int(n_succ.sum())
    total += 36 * R
    return int(total)


def leg_bc(gb, torch, inputs, stream):
    """Betweenness centrality (Section 2.1: scores from 4 sources, normalised
    to one) on R-MAT 22 and uniform 2^22: 8 trials of 4 sources each."""
    out = {}
    for name in ("rmat22", "urand22"):
        el = inputs.workload(name)
        g = gb.build_csr(el.n, el.src, el.dst)
        del el
        rp, col = g.export()
        rows = np.repeat(np.arange(g.n, dtype=np.int32), np.diff(rp))
        srcs = [int(x) for x in inputs.pick_sources(inputs.workload(name), 32,
                                                    seed=inputs.SOURCE_SEEDS[name] + 5)]
        trials = [srcs[4 * i:4 * i + 4] for i in range(8)]
        score = torch.empty(g.n, dtype=torch.float64, device="cuda")
        p = torch.empty(g.n, dtype=torch.int32, device="cuda")
        dd = torch.empty(g.n, dtype=torch.int32, device="cuda")
        ms = []
        alg0 = 0
        for i, tr in enumerate(trials):  # m_s per trial; bytes of the first trial (untimed)
            m = 0
            for s in tr:
                recs = gb.bfs(g, s, p, dd, stats=True)
                d = dd.cpu().numpy()
                if i == 0:
                    alg0 += algorithmic_bytes(recs, g.n) + bc_bytes(rp, col, rows, d)
                m += int(np.diff(rp)[d >= 0].sum()) // 2
            ms.append(m)
        del col, rows
        gb.bc(g, trials[0], score)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        times = []
        for tr in trials:
            t0 = time.perf_counter()
            e0.record(stream)
            gb.bc(g, tr, score, stream=stream)
            e1.record(stream)
            e1.synchronize()
            times.append((e0.elapsed_time(e1), (time.perf_counter() - t0) * 1e3))
        t = np.array([x[0] for x in times])
        out[name] = {"trial_ms_median": round(float(np.median(t)), 3),
                     "trial_ms_min": round(float(t.min()), 3),
                     "wall_ms_median": round(float(np.median([x[1] for x in times])), 3),
                     "gteps_median": round(float(np.median(np.array(ms) / (t * 1e-3) / 1e9)), 2),
                     "alg_bytes_first_trial": int(alg0),
                     "alg_gbs_first_trial": round(float(alg0 / (t[0] * 1e-3) / 1e9), 1)}
        log(f"bc {name}: {out[name]}")
        del score, p, dd
        g.free()
        torch.cuda.empty_cache()
    return out


def leg_sssp(gb, torch, inputs, stream, sweep=True):
    """Shortest paths (Delta-stepping) on R-MAT 22 and uniform 2^22 with the
    generator's weights 1..255: 16 sources each at the default bucket width;
    m_s as for BFS (undirected edges in the source's component).  With
    ``sweep``, 4 sources at other widths."""
    out = {}
    for name in ("rmat22", "urand22"):
        el = inputs.workload(name)
        w = inputs.weights(el, seed=inputs.WEIGHT_SEEDS[name])
        g = gb.build_csr(el.n, el.src, el.dst, weights=w)
        srcs = [int(x) for x in inputs.pick_sources(el, 16, seed=inputs.SOURCE_SEEDS[name] + 21)]
        ce = component_edges(g, el)
        del el, w
        dist = torch.empty(g.n, dtype=torch.int32, device="cuda")
        phases = [gb.sssp(g, s, dist, stats=True) for s in srcs]
        pairs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in srcs]

        def timed(delta, ss):
            best = None
            for _ in range(2):
                for i, s in enumerate(ss):
                    pairs[i][0].record(stream)
                    gb.sssp(g, s, dist, delta=delta, stream=stream)
                    pairs[i][1].record(stream)
                torch.cuda.synchronize()
                t = np.array([pairs[i][0].elapsed_time(pairs[i][1]) for i in range(len(ss))])
                best = t if best is None or t.sum() < best.sum() else best
            return best

        t = timed(0, srcs)
        ms = np.array([int(ce[s]) for s in srcs], np.int64)
        out[name] = {"search_ms_median": round(float(np.median(t)), 3),
                     "gteps_aggregate": round(float(ms.sum() / (t.sum() * 1e-3) / 1e9), 2),
                     "phases_mean": round(float(np.mean(phases)), 1)}
        if sweep:
            out[name]["delta_sweep_ms_median"] = {
                str(dl): round(float(np.median(timed(dl, srcs[:4]))), 3)
                for dl in (8, 16, 32, 64, 128, 256, 512)}
        log(f"sssp {name}: {out[name]}")
        del dist
        g.free()
        torch.cuda.empty_cache()
    return out


def leg_cc(gb, torch, inputs, stream):
    """Connected components on R-MAT 22, uniform 2^22 and the directed
    R-MAT 22 (weak components): best of 5 runs; GTEPS = stored adjacency
    entries / 2 (undirected) or entries (directed) per second."""
    out = {}
    for name in ("rmat22", "urand22", "rmat22d"):
        el = inputs.workload(name)
        directed = name in inputs.DIRECTED
        g = gb.build_csr(el.n, el.src, el.dst, directed=directed)
        del el
        lab = torch.empty(g.n, dtype=torch.int32, device="cuda")
        t = time_launches(torch, stream, lambda: gb.cc(g, lab, stream=stream), reps=5)
        edges = g.nnz if directed else g.nnz // 2
        ncomp = int(torch.unique(lab).numel())
        out[name] = {"ms": round(t, 3), "gteps": round(edges / (t * 1e-3) / 1e9, 2),
                     "components": ncomp}
        log(f"cc {name}: {out[name]}")
        del lab
        g.free()
        torch.cuda.empty_cache()
    return out


MIXED_SCALES = [14, 14, 15, 15, 16, 16, 17, 17, 18, 18, 19, 19, 20, 20, 20, 20]


def leg_mixed(gb, torch, inputs, stream):
    """16 R-MAT graphs of scales 14-20 in one launch: 4 and 16 sources per
    graph (64 and 256 lanes)."""
    els = [inputs.rmat(s, 16, seed=30000 + i) for i, s in enumerate(MIXED_SCALES)]
    graphs = [gb.build_csr(e.n, e.src, e.dst) for e in els]
    ces = [component_edges(g, e) for g, e in zip(graphs, els)]
    out = {"sum_n": int(sum(g.n for g in graphs)), "sum_nnz": int(sum(g.nnz for g in graphs))}
    for per in (4, 16):
        gos, srcs = [], []
        for gi, e in enumerate(els):
            for s in inputs.pick_sources(e, per, seed=1030000 + gi):
                gos.append(gi)
                srcs.append(int(s))
        P = [torch.empty(graphs[gi].n, dtype=torch.int32, device="cuda") for gi in gos]
        D = [torch.empty(graphs[gi].n, dtype=torch.int32, device="cuda") for gi in gos]
        t = time_launches(torch, stream, lambda: gb.bfs_batch(graphs, gos, srcs, P, D))
        pa, da = P[0], D[0]
        single = time_launches(torch, stream, lambda: [gb.bfs(graphs[gi], s, P[i], D[i])
                                                       for i, (gi, s) in enumerate(zip(gos, srcs))],
                               reps=2)
        ms = sum(int(ces[gi][s]) for gi, s in zip(gos, srcs))
        out[f"lanes{len(srcs)}"] = {"batch_ms": round(t, 3), "batch_gteps": round(ms / (t * 1e-3) / 1e9, 2),
                                    "single_ms_sum": round(single, 3),
                                    "batch_speedup_vs_single": round(single / t, 2)}
        del P, D, pa, da
    log(f"mixed16: {out}")
    for g in graphs:
        g.free()
    return out


def leg_serving(gb, torch, nq):
    """Serving pool of 32 resident graphs, two loops over the same arrivals:
    launch-granular batching (a launch takes the queries waiting when it
    starts) and continuous batching (queries join running searches of their
    graph at level boundaries, gap_serve_*).  For each: saturation throughput
    R_sat from a closed loop (16 clients per slot), then Poisson arrivals at
    0.25, 0.6 and 0.9 of R_sat.  Admission: the outputs of queries in flight
    must fit a budget of 512 MiB (the working sets of the launches are
    resident beside it and reported)."""
    from paper_1508_03619_amd import serving as sv
    t0 = time.time()
    spec = sv.pool_spec()
    pool = sv.Pool(spec, keep_edges=True)
    ces = [component_edges(g, el) for g, el in zip(pool.graphs, pool.edges)]
    pool.edges = [None] * len(pool.edges)
    slots, lanes = 8, 64
    budget = 512 << 20
    out = {"graphs": len(pool.graphs), "sum_n": int(sum(pool.sizes)), "slots": slots,
           "max_lanes": lanes, "budget_bytes": budget,
           "build_s": round(time.time() - t0, 1)}

    def run(ex, continuous, rate, n, seed, clients=0):
        qs = sv.poisson_queries(rate, n, pool.sources, seed)
        src = sv.ClosedArrivals(clients, n, lambda k: qs[k]) if clients else qs
        sched = sv.Scheduler(pool.sizes, budget_bytes=budget, max_lanes=lanes)
        t = time.perf_counter()
        done = (sv.serve_continuous if continuous else sv.serve)(ex, sched, src)
        wall = time.perf_counter() - t
        summ = sv.latency_summary(done, skip=n // 10)
        kept = sorted(done, key=lambda q: (q.arrival, q.qid))[n // 10:]
        span = max(q.done for q in kept) - min(q.arrival for q in kept)
        summ["gteps"] = sum(int(ces[q.graph][q.source]) for q in kept) / span / 1e9
        summ["peak_admitted_bytes"] = sched.peak_used
        summ["admission_waits"] = sched.admission_waits
        summ["launches"] = dict(ex.launch_kinds)
        ex.launch_kinds.clear()
        return {k: (round(v, 3) if isinstance(v, float) else v) for k, v in summ.items()}, wall

    def rates(ex, continuous, tag):
        res = {}
        clients = 16 * slots
        run(ex, continuous, 0.0, 300, 1, clients)  # warm-up: workspaces, code objects
        s, wall = run(ex, continuous, 0.0, nq, 776, clients)
        rsat = s["throughput_qps"]
        res["r_sat_qps"] = round(rsat, 1)
        res["closed_loop_clients"] = clients
        res["closed"] = s
        log(f"serving {tag} closed loop ({clients} clients): R_sat={rsat:.1f} q/s {s}")
        for k, f in enumerate((0.25, 0.6, 0.9)):
            s, wall = run(ex, continuous, f * rsat, nq, 777 + k)
            s["offered_qps"] = round(f * rsat, 1)
            res[f"rate_{f}"] = s
            log(f"serving {tag} at {f} R_sat: {s}")
        return res

    try:
        ex = sv.GpuExecutor(pool.graphs, slots=slots, sources=pool.sources)
        try:
            out["launch_granular"] = rates(ex, False, "launch-granular")
        finally:
            ex.close()
        torch.cuda.synchronize()
        ex = sv.ContinuousExecutor(pool.graphs, slots=slots, lanes=lanes, sources=pool.sources)
        try:
            out["continuous_workspace_bytes"] = int(
                slots * (152 * max(pool.sizes) + 2 * max(g.nnz for g in pool.graphs)))
            out["continuous_single_search_graphs"] = sorted(int(x) for x in ex.single_graphs)
            out["continuous"] = rates(ex, True, "continuous")
        finally:
            ex.close()
    finally:
        pool.free()
    return out


def leg_strict(gb, torch, cases, stream):
    """T_strict (every allocation for the solution inside the timed region,
    as the paper's trial rules count it): per trial, hipMalloc of the two
    outputs, the search, gap_shutdown (which waits and releases the
    library's per-stream scratch, so every trial allocates it again inside
    gap_bfs) and hipFree of the outputs, timed on the host clock.  Beside
    it, the same sources with caller-held outputs and a resident scratch
    pool (T_trial, the headline's convention), on the same clock."""
    import ctypes
    hip = ctypes.CDLL(os.path.join(os.path.dirname(torch.__file__), "lib", "libamdhip64.so"))
    hip.hipMalloc.argtypes = [ctypes.POINTER(ctypes.c_void_p), ctypes.c_size_t]
    hip.hipFree.argtypes = [ctypes.c_void_p]
    L = gb.load()
    sh = ctypes.c_void_p(stream.cuda_stream)
    out = {}
    for c in cases:
        strict, trial = [], []
        p = ctypes.c_void_p()
        d = ctypes.c_void_p()
        for s in c.sources:
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            if hip.hipMalloc(ctypes.byref(p), 4 * c.g.n) or hip.hipMalloc(ctypes.byref(d), 4 * c.g.n):
                raise SystemExit("hipMalloc failed")
            st = L.gap_bfs(c.g.handle, int(s), p, d, sh)
            L.gap_shutdown()
            hip.hipFree(p)
            hip.hipFree(d)
            strict.append(time.perf_counter() - t0)
            if st != 0:
                raise SystemExit(f"gap_bfs: {L.gap_last_error().decode()}")
        for s in c.sources:
            t0 = time.perf_counter()
            gb.bfs(c.g, int(s), c.parent, c.depth, stream=stream)
            stream.synchronize()
            trial.append(time.perf_counter() - t0)
        gb.stream_status(stream)
        strict, trial = np.array(strict), np.array(trial)
        out[c.name] = {"t_strict_ms_median": round(float(np.median(strict)) * 1e3, 3),
                       "gteps_strict": round(float(c.ms.sum() / strict.sum() / 1e9), 2),
                       "t_trial_host_ms_median": round(float(np.median(trial)) * 1e3, 3),
                       "gteps_trial_host": round(float(c.ms.sum() / trial.sum() / 1e9), 2)}
    log(f"T_strict: {out}")
    return out


def host_cpu():
    """(threads this process may use, at most 16, and the CPU model name)."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    model = ""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return min(16, max(1, n)), n, model


def cpu_baseline_leg(gb, torch, cases, serial_seconds, stream):
    """The CPU oracle on the host cores, and validation of every headline
    search against it.

    (i) serial: the oracle on one core over the first sources of the first
    graph until ``serial_seconds`` have passed; (ii) source-parallel: one
    oracle search per source for every source of every graph, on as many
    threads as the host gives this process (at most 16), timed as a whole.
    Then each source's GPU search (the benchmark's configuration) is checked
    against the oracle's depths: depths bit-exact, parents valid."""
    import oracle
    from concurrent.futures import ThreadPoolExecutor
    threads, nproc, model = host_cpu()
    t0 = time.perf_counter()
    with ThreadPoolExecutor(threads) as ex:
        adjs = list(ex.map(lambda c: oracle.Adjacency(c.el.n, c.el.src, c.el.dst), cases))
    log(f"oracle adjacency for {len(cases)} graphs in {time.perf_counter() - t0:.1f}s")
    c, A = cases[0], adjs[0]
    done_edges, done_t, k = 0, 0.0, 0
    for s, m in zip(c.sources, c.ms):
        t1 = time.perf_counter()
        A.bfs(int(s))
        done_t += time.perf_counter() - t1
        done_edges += int(m)
        k += 1
        if done_t > serial_seconds:
            break
    serial = {"value": round(done_edges / done_t / 1e9, 5), "unit": "GTEPS", "cores": 1,
              "sample": f"{k} of the {len(c.sources)} {c.name} sources, {done_t:.1f}s"}
    jobs = [(ci, int(s)) for ci, cc in enumerate(cases) for s in cc.sources]
    t1 = time.perf_counter()
    with ThreadPoolExecutor(threads) as ex:
        refs = list(ex.map(lambda j: adjs[j[0]].bfs(j[1])[0], jobs))
    par_t = time.perf_counter() - t1
    par_edges = int(sum(int(cc.ms.sum()) for cc in cases))
    # validation: the GPU search of each source against the oracle's depths
    ok = {cc.name: 0 for cc in cases}

    def check(j, ref, p, d):
        code, bad = adjs[j[0]].check(j[1], ref, p, d)
        return j, code, bad

    for cc in cases:
        if cc.parent is None:
            cc.parent = torch.empty(cc.g.n, dtype=torch.int32, device="cuda")
            cc.depth = torch.empty(cc.g.n, dtype=torch.int32, device="cuda")
    with ThreadPoolExecutor(threads) as ex:
        futs = []
        for j, ref in zip(jobs, refs):
            cc = cases[j[0]]
            gb.bfs(cc.g, j[1], cc.parent, cc.depth, stream=stream)
            torch.cuda.synchronize()
            futs.append(ex.submit(check, j, ref, cc.parent.cpu().numpy(), cc.depth.cpu().numpy()))
        for f in futs:
            j, code, bad = f.result()
            if code != 0:
                raise SystemExit(f"{cases[j[0]].name} source {j[1]}: GPU result fails the oracle "
                                 f"check ({oracle.CHECK_NAMES.get(code, code)}, vertex {bad})")
            ok[cases[j[0]].name] += 1
    gb.stream_status(stream)
    validated = {cc.name: f"{ok[cc.name]}/{len(cc.sources)}" for cc in cases}
    log(f"validated against the oracle: {validated}")
    return {"value": round(par_edges / par_t / 1e9, 5), "unit": "GTEPS", "cores": threads,
            "kind": "oracle",
            "sample": (f"serial FIFO oracle run source-parallel on {threads} threads: all "
                       f"{len(jobs)} sources of {'+'.join(cc.name for cc in cases)} in "
                       f"{par_t:.1f}s wall (adjacency build untimed)"),
            "serial_1core": serial, "host_nproc": nproc, "host_cpu": model,
            "validated": validated}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--sources", type=int, default=64)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--graphs", default="rmat22,urand22")
    ap.add_argument("--legs", default="strict,grid4096,rmat24,mixed,serving,directed,bc,sssp,cc",
                    help="comma list of extra legs reported in detail: strict, serving, directed, "
                         "bc, sssp, cc, grid4096, rmat24, mixed, or all")
    ap.add_argument("--serve-queries", type=int, default=1000)
    ap.add_argument("--profile-levels", type=int, default=0, metavar="K",
                    help="for rocprofv3 counter runs: K sources per graph searched with the "
                         "per-level schedule (one launch per step), each after a statistics run "
                         "whose records are printed as JSON lines, so rocprof_summary levels can "
                         "attribute counters to levels")
    ap.add_argument("--profile-leg", action="store_true",
                    help="for rocprofv3 counter runs: a copy of known size, then one search per "
                         "source, no timing and no JSON")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(each search runs on a single MI355X).", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1508_03619_amd import gapbfs as gb
    from paper_1508_03619_amd import inputs

    gb.load()
    torch.cuda.set_device(0)
    dev = gb.device_query()
    log(f"device {dev['arch']} CUs={dev['compute_units']} params={gb.get_params()}")
    stream = torch.cuda.current_stream()

    cases = []
    for name in args.graphs.split(","):
        el = inputs.workload(name)
        cases.append(GraphCase(name, el, gb, torch, args.sources, inputs.SOURCE_SEEDS[name]))

    if args.profile_levels:
        a = torch.empty(PROFILE_COPY_BYTES // 4, dtype=torch.int32, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            gb.stream_copy(b, a, PROFILE_COPY_BYTES)
        torch.cuda.synchronize()
        del a, b
        for c in cases:
            for s in c.sources[:args.profile_levels]:
                recs = gb.bfs(c.g, int(s), c.parent, c.depth, params={"mode": 1}, stats=True)
                gb.bfs(c.g, int(s), c.parent, c.depth, params={"mode": 1})
                torch.cuda.synchronize()
                keep = ("direction", "frontier", "frontier_edges", "claimed", "scanned", "unvisited")
                print("LEVELS " + json.dumps({"graph": c.name, "n": c.g.n, "source": int(s),
                                              "levels": [[r[k] for k in keep] for r in recs]}), flush=True)
        log("profile levels done")
        return

    if args.profile_leg:
        a = torch.empty(PROFILE_COPY_BYTES // 4, dtype=torch.int32, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            gb.stream_copy(b, a, PROFILE_COPY_BYTES)
        torch.cuda.synchronize()
        for c in cases:
            for s in c.sources:
                gb.bfs(c.g, int(s), c.parent, c.depth)
        torch.cuda.synchronize()
        for c in cases:  # one 64-lane batch per graph (the batched kernel's counters)
            ns = len(c.sources)
            ps = [torch.empty(c.g.n, dtype=torch.int32, device="cuda") for _ in range(ns)]
            ds = [torch.empty(c.g.n, dtype=torch.int32, device="cuda") for _ in range(ns)]
            gb.bfs_batch([c.g], [0] * ns, [int(s) for s in c.sources], ps, ds)
            torch.cuda.synchronize()
            del ps, ds
        log("profile leg done")
        return

    # Per-level records (untimed); every search must reach exactly its
    # source's component (sizes from the raw pairs).
    for c in cases:
        c.alg_bytes = []
        c.levels = []
        for s in c.sources:
            recs = gb.bfs(c.g, int(s), c.parent, c.depth, stats=True)
            reached = int((c.depth >= 0).sum())
            want = int(c.comp_size[c.lab[s]])
            if reached != want:
                raise SystemExit(f"{c.name} source {s}: the search reached {reached} vertices, "
                                 f"its component has {want}")
            c.alg_bytes.append(algorithmic_bytes(recs, c.g.n))
            c.levels.append(len(recs))
        log(f"{c.name}: mean m_s={c.ms.mean():.3e} mean levels={np.mean(c.levels):.1f} "
            f"dirs(first source)={[r['direction'] for r in gb.last_stats()]}")

    ev_pairs = {c.name: [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
                         for _ in c.sources] for c in cases}

    def step(record=False):
        for c in cases:
            for i, s in enumerate(c.sources):
                e0, e1 = ev_pairs[c.name][i]
                if record:
                    e0.record(stream)
                gb.bfs(c.g, int(s), c.parent, c.depth, stream=stream)
                if record:
                    e1.record(stream)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()

    per_trial = {c.name: [] for c in cases}
    t0 = time.perf_counter()
    for k in range(args.steps):
        step(record=True)
        torch.cuda.synchronize()
        for c in cases:
            per_trial[c.name].append([ev_pairs[c.name][i][0].elapsed_time(ev_pairs[c.name][i][1])
                                      for i in range(len(c.sources))])
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    gb.stream_status(stream)  # no timed search failed on the device
    total_edges = sum(int(c.ms.sum()) for c in cases) * args.steps
    value = total_edges / wall / 1e9
    ms_per_step = wall / args.steps * 1e3

    detail = {}
    launches = 0
    launch_ms_sum = 0.0
    alg_sum = 0
    for c in cases:
        t = np.array(per_trial[c.name])  # steps x sources, ms
        gteps = c.ms[None, :] / (t * 1e-3) / 1e9
        detail[c.name] = {
            "n": int(c.g.n), "nnz": int(c.g.nnz),
            "gteps_aggregate": float(c.ms.sum() * args.steps / (t.sum() * 1e-3) / 1e9),
            "gteps_median_trial": float(np.median(gteps)),
            "trial_ms_median": float(np.median(t)), "trial_ms_min": float(t.min()),
            "trial_ms_max": float(t.max()),
            "levels_mean": float(np.mean(c.levels)),
            "alg_bytes_mean": float(np.mean(c.alg_bytes)),
            "alg_gbs_median": float(np.median(np.array(c.alg_bytes)[None, :] / (t * 1e-3) / 1e9)),
        }
        launches += t.size
        launch_ms_sum += float(t.sum())
        alg_sum += int(np.sum(c.alg_bytes)) * args.steps
    avg_launch_ms = launch_ms_sum / launches
    avg_alg_bytes = alg_sum / launches
    achieved = avg_alg_bytes / (avg_launch_ms * 1e-3) / 1e9

    traffic = committed_traffic("k_bfs_persistent")

    roofline = {"bound": "hbm", "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                "kernel": "k_bfs_persistent", "avg_launch_ms": round(avg_launch_ms, 4),
                "alg_bytes_per_launch": int(avg_alg_bytes)}

    # Measured copy bandwidth (read + write), reported beside the peak.
    nbytes = 1 << 32
    a = torch.empty(nbytes // 4, dtype=torch.int32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(2):
        gb.stream_copy(b, a, nbytes)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(5):
        gb.stream_copy(b, a, nbytes)
    e1.record(stream)
    torch.cuda.synchronize()
    copy_gbs = 2 * nbytes * 5 / (e0.elapsed_time(e1) * 1e-3) / 1e9
    del a, b
    detail["stream_copy_gbs"] = round(copy_gbs, 1)

    # Batched leg: one 64-lane launch per graph vs the same sources one by one.
    if not args.no_batch:
        for c in cases:
            ns = len(c.sources)
            parents = [torch.empty(c.g.n, dtype=torch.int32, device="cuda") for _ in range(ns)]
            depths = [torch.empty(c.g.n, dtype=torch.int32, device="cuda") for _ in range(ns)]
            brecs = gb.bfs_batch([c.g], [0] * ns, [int(s) for s in c.sources], parents, depths,
                                 stats=True)
            gb.stream_status()
            detail[c.name]["batch64_alg_bytes"] = batch_algorithmic_bytes(brecs, c.g.n, ns)
            detail[c.name]["batch64_levels"] = len(brecs)
            gb.bfs_batch([c.g], [0] * ns, [int(s) for s in c.sources], parents, depths)
            torch.cuda.synchronize()
            e0.record(stream)
            reps = 3
            for _ in range(reps):
                gb.bfs_batch([c.g], [0] * ns, [int(s) for s in c.sources], parents, depths)
            e1.record(stream)
            torch.cuda.synchronize()
            bt = e0.elapsed_time(e1) / reps
            single_ms = float(np.sum(np.mean(np.array(per_trial[c.name]), axis=0)))
            detail[c.name]["batch64_ms"] = round(bt, 3)
            detail[c.name]["batch64_gteps"] = round(float(c.ms.sum()) / (bt * 1e-3) / 1e9, 2)
            detail[c.name]["single64_ms_sum"] = round(single_ms, 3)
            detail[c.name]["batch_speedup_vs_single"] = round(single_ms / bt, 2)
            del parents, depths
        # counted HBM traffic of the batched kernel (committed counter run over
        # the same two 64-lane batches) against the measured batch times
        bt_mean = float(np.mean([detail[c.name]["batch64_ms"] for c in cases]))
        btraffic = committed_traffic("k_msbfs")
        balg = float(np.mean([detail[c.name]["batch64_alg_bytes"] for c in cases]))
        ach = balg / (bt_mean * 1e-3) / 1e9
        detail["batch_roofline"] = {
            "kernel": "k_msbfs", "bound": "hbm", "unit": "GB/s", "peak": HBM_PEAK_GBS,
            "avg_launch_ms": round(bt_mean, 3), "alg_bytes_per_launch": int(balg),
            "achieved": round(ach, 1), "frac": round(ach / HBM_PEAK_GBS, 4),
            "single_frac": roofline["frac"], "traffic": btraffic,
            "achieved_counted": (round(btraffic / (bt_mean * 1e-3) / 1e9, 1) if btraffic else None),
            "frac_counted": (round(btraffic / (bt_mean * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)
                             if btraffic else None)}

    legs = set(args.legs.split(",")) if args.legs else set()
    if "all" in legs:
        legs = {"strict", "serving", "directed", "bc", "sssp", "cc", "grid4096", "rmat24", "mixed"}
    if "strict" in legs:
        detail["strict"] = leg_strict(gb, torch, cases, stream)
    for c in cases:
        c.parent = c.depth = None
    torch.cuda.empty_cache()
    if "directed" in legs:
        detail["rmat22_directed"] = leg_directed(gb, torch, inputs, stream)
    if "bc" in legs:
        detail["bc"] = leg_bc(gb, torch, inputs, stream)
    if "sssp" in legs:
        detail["sssp"] = leg_sssp(gb, torch, inputs, stream)
    if "cc" in legs:
        detail["cc"] = leg_cc(gb, torch, inputs, stream)
    if "grid4096" in legs:
        detail["grid4096"] = leg_grid(gb, torch, inputs, stream)
    if "rmat24" in legs:
        detail["rmat24"] = leg_rmat24(gb, torch, inputs, stream)
    if "mixed" in legs:
        detail["mixed16"] = leg_mixed(gb, torch, inputs, stream)
    if "serving" in legs:
        detail["serving"] = leg_serving(gb, torch, args.serve_queries)

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline_leg(gb, torch, cases, args.cpu_seconds, stream)
        for c in cases:
            detail[c.name]["validated"] = cpu["validated"][c.name]

    out = {
        "metric": "BFS GTEPS (direction-optimizing, single-source)",
        "value": round(value, 3),
        "unit": "GTEPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32",
        "data": "synthetic",
        "config": {"workload": "rmat22+urand22: R-MAT scale 22 ef16 (a.57 b.19 c.19) and uniform "
                               "2^22 x 16*2^22 pairs, symmetrised int32 CSR, 64 random non-zero-degree "
                               "sources each, direction-optimizing single-source BFS",
                   "sources_per_graph": args.sources, "params": gb.get_params()},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "detail": detail,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
