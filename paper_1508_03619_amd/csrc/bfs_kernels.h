// Single-source direction-optimizing BFS: the per-level steps as device
// functions.  They are shared by the persistent cooperative kernel and by
// the one-launch-per-step kernels, so both schedules run the same code.
#pragma once

#include "common.h"

namespace gap {

struct StepArgs {
  DevGraph g;
  int32_t *parent;       // int32[n]: -degree (or kIsolated) while unvisited
  int32_t *depth;        // int32[n]
  const int32_t *qin;    // F_d as a vertex queue (vertices of degree <= hub)
  const int2 *cin;       // F_d hub work items: {vertex, chunk index}
  int64_t nq_in, nc_in;
  int32_t *qout;         // F_{d+1} vertex queue
  int2 *cout;            // F_{d+1} hub work items
  const uint64_t *fbm;   // F_d bitmap (bottom-up)
  uint64_t *vbm;         // visited bitmap (bottom-up), padding bits set
  uint64_t *nbm;         // F_{d+1} bitmap written by bottom-up
  LevelCounters *acc;    // totals of this level
  int32_t d;             // depth of the frontier being expanded
  int32_t hub;           // degree above which a vertex becomes chunk items
  int32_t chunk;         // edges per chunk item (multiple of 64)
};

// Per-lane totals carried through a step and flushed once per wave.
struct LaneAcc {
  unsigned long long mf = 0, nv = 0, scanned = 0, unvisited = 0;
};

// Claim v for parent u (top-down).  The parent array holds -degree for an
// unvisited vertex (Section 3, BFS), so the winner learns deg(v) from the
// value it replaced: the frontier's edge total accrues at no extra cost.
__device__ inline bool td_claim(const StepArgs &a, int32_t v, int32_t u, int64_t &degv) {
  int32_t p = a.parent[v];
  if (p >= 0) return false;
  int32_t old = atomicCAS(&a.parent[v], p, u);
  if (old != p) return false;
  a.depth[v] = a.d + 1;
  degv = (p == kIsolated) ? 0 : -(int64_t)p;
  return true;
}

// Append the vertices this wave claimed to the next frontier: vertices of
// degree <= hub go to the vertex queue, larger ones become chunk items of
// `chunk` edges each so that one hub is expanded by many waves.  One atomic
// per wave per queue.
__device__ inline void wave_append(const StepArgs &a, bool claimed, int32_t v, int64_t degv,
                                   LaneAcc &acc) {
  const uint64_t any = __ballot(claimed);
  if (any == 0) return;
  const int lane = lane_id();
  const bool big = claimed && degv > a.hub;
  const bool small = claimed && !big;
  const uint64_t ms = __ballot(small);
  if (ms) {
    const int leader = first_lane(ms);
    unsigned long long base = 0;
    if (lane == leader) base = atomicAdd(&a.acc->nq, (unsigned long long)__popcll(ms));
    base = __shfl(base, leader, kWave);
    if (small) a.qout[base + lane_rank(ms)] = v;
  }
  const uint64_t mb = __ballot(big);
  if (mb) {
    uint32_t nch = big ? (uint32_t)((degv + a.chunk - 1) / a.chunk) : 0u;
    uint32_t total;
    uint32_t off = wave_excl_scan_u32(nch, total);
    const int leader = first_lane(mb);
    unsigned long long base = 0;
    if (lane == leader) base = atomicAdd(&a.acc->nc, (unsigned long long)total);
    base = __shfl(base, leader, kWave);
    for (uint32_t k = 0; k < nch; ++k) a.cout[base + off + k] = make_int2(v, (int)k);
  }
  if (claimed) {
    acc.mf += (unsigned long long)degv;
    acc.nv += 1;
  }
}

template <bool STATS>
__device__ inline void flush_acc(const StepArgs &a, LaneAcc &acc) {
  unsigned long long mf = wave_sum_u64(acc.mf);
  unsigned long long nv = wave_sum_u64(acc.nv);
  if (lane_id() == 0) {
    if (mf) atomicAdd(&a.acc->mf, mf);
    if (nv) atomicAdd(&a.acc->nv, nv);
  }
  if (STATS) {
    unsigned long long sc = wave_sum_u64(acc.scanned);
    unsigned long long un = wave_sum_u64(acc.unvisited);
    if (lane_id() == 0) {
      if (sc) atomicAdd(&a.acc->scanned, sc);
      if (un) atomicAdd(&a.acc->unvisited, un);
    }
  }
  acc = LaneAcc();
}

// Top-down step: every edge (u, v) with u in F_d is tried once.
//  * hub chunk items: one wave walks `chunk` consecutive edges of one hub;
//  * queue vertices: a wave takes 64 queued vertices, prefix-sums their
//    degrees and then walks the combined edge range 64 edges at a time,
//    each lane finding its owner vertex by a binary search over the 64
//    offsets held in registers (no lane idles on a short list).
template <bool STATS>
__device__ void td_step(const StepArgs &a, int64_t gwave, int64_t nwaves) {
  const int lane = lane_id();
  LaneAcc acc;
  for (int64_t ci = gwave; ci < a.nc_in; ci += nwaves) {
    const int2 it = a.cin[ci];
    const int32_t u = it.x;
    const int64_t rbeg = a.g.row_ptr[u], rend = a.g.row_ptr[u + 1];
    const int64_t beg = rbeg + (int64_t)it.y * a.chunk;
    const int64_t end = beg + a.chunk < rend ? beg + a.chunk : rend;
    for (int64_t e0 = beg; e0 < end; e0 += kWave) {
      const int64_t e = e0 + lane;
      bool claimed = false;
      int32_t v = -1;
      int64_t degv = 0;
      if (e < end) {
        v = a.g.col[e];
        claimed = td_claim(a, v, u, degv);
        if (STATS) acc.scanned += 1;
      }
      wave_append(a, claimed, v, degv, acc);
    }
  }
  const int64_t ngroups = (a.nq_in + kWave - 1) / kWave;
  for (int64_t gi = gwave; gi < ngroups; gi += nwaves) {
    const int64_t idx = gi * kWave + lane;
    int32_t u = -1;
    int64_t beg = 0;
    uint32_t deg = 0;
    if (idx < a.nq_in) {
      u = a.qin[idx];
      beg = a.g.row_ptr[u];
      deg = (uint32_t)(a.g.row_ptr[u + 1] - beg);
    }
    uint32_t total;
    const uint32_t off = wave_excl_scan_u32(deg, total);
    for (uint32_t b = 0; b < total; b += kWave) {
      const uint32_t e = b + (uint32_t)lane;
      int j = 0;
#pragma unroll
      for (int step = 32; step >= 1; step >>= 1) {
        uint32_t oc = __shfl(off, j + step, kWave);
        if (oc <= e) j += step;
      }
      const int32_t uj = __shfl(u, j, kWave);
      const int64_t bj = __shfl(beg, j, kWave);
      const uint32_t oj = __shfl(off, j, kWave);
      bool claimed = false;
      int32_t v = -1;
      int64_t degv = 0;
      if (e < total) {
        v = a.g.col[bj + (int64_t)(e - oj)];
        claimed = td_claim(a, v, uj, degv);
        if (STATS) acc.scanned += 1;
      }
      wave_append(a, claimed, v, degv, acc);
    }
  }
  flush_acc<STATS>(a, acc);
}

// Bottom-up step: each unvisited vertex scans its neighbours in order and
// stops at the first one in F_d.  Lane i of a wave owns vertex 64w+i, so the
// next-frontier and visited words come from one ballot with a single writer
// (no atomics); words whose 64 vertices are all visited are skipped whole.
template <bool STATS>
__device__ void bu_step(const StepArgs &a, int64_t gwave, int64_t nwaves) {
  const int lane = lane_id();
  const int64_t nwords = (a.g.n + kWave - 1) / kWave;
  LaneAcc acc;
  for (int64_t w = gwave; w < nwords; w += nwaves) {
    const uint64_t vis = a.vbm[w];
    if (vis == ~0ull) {
      if (lane == 0) a.nbm[w] = 0ull;
      continue;
    }
    const int64_t v = w * kWave + lane;
    const bool need = ((vis >> lane) & 1ull) == 0ull;
    bool found = false;
    int32_t pu = -1;
    int64_t degv = 0;
    if (need) {
      const int64_t beg = a.g.row_ptr[v], end = a.g.row_ptr[v + 1];
      degv = end - beg;
      if (STATS) acc.unvisited += 1;
      for (int64_t e = beg; e < end; ++e) {
        const int32_t u = a.g.col[e];
        if (STATS) acc.scanned += 1;
        if ((a.fbm[u >> 6] >> (u & 63)) & 1ull) {
          found = true;
          pu = u;
          break;
        }
      }
    }
    if (found) {
      a.parent[v] = pu;
      a.depth[v] = a.d + 1;
    }
    const uint64_t b = __ballot(found);
    if (lane == 0) {
      a.nbm[w] = b;
      if (b) a.vbm[w] = vis | b;
    }
    wave_append(a, found, (int32_t)v, degv, acc);
  }
  flush_acc<STATS>(a, acc);
}

// Top-down -> bottom-up: build the frontier bitmap (depth == d) and the
// visited bitmap (parent >= 0, isolated vertices and padding count as
// visited so whole words can be skipped).
__device__ inline void convert_to_bitmaps(const DevGraph &g, const int32_t *parent,
                                          const int32_t *depth, int32_t d, uint64_t *fbm,
                                          uint64_t *vbm, int64_t gwave, int64_t nwaves) {
  const int lane = lane_id();
  const int64_t nwords = (g.n + kWave - 1) / kWave;
  for (int64_t w = gwave; w < nwords; w += nwaves) {
    const int64_t v = w * kWave + lane;
    bool visited = true, front = false;
    if (v < g.n) {
      const int32_t p = parent[v];
      visited = (p >= 0) || (p == kIsolated);
      front = depth[v] == d;
    }
    const uint64_t bv = __ballot(visited);
    const uint64_t bf = __ballot(front);
    if (lane == 0) {
      vbm[w] = bv;
      fbm[w] = bf;
    }
  }
}

// Per-search initialisation (timed, Section 2.3): parent <- -degree
// (Section 3, BFS), depth <- -1, then the source.
__device__ inline void init_vertices(const DevGraph &g, int32_t *parent, int32_t *depth,
                                     int32_t source, int64_t tid, int64_t nthreads) {
  for (int64_t v = tid; v < g.n; v += nthreads) {
    const int64_t deg = g.row_ptr[v + 1] - g.row_ptr[v];
    int32_t p = deg ? (int32_t)(-deg) : kIsolated;
    int32_t dd = -1;
    if (v == source) {
      p = source;
      dd = 0;
    }
    parent[v] = p;
    depth[v] = dd;
  }
}

// Source into F_0 plus the level -1 totals (run by one thread).
__device__ inline void init_source(const DevGraph &g, int32_t source, int32_t hub, int32_t chunk,
                                   int32_t *q0, int2 *c0, Ctl *ctl) {
  const int64_t deg = g.row_ptr[source + 1] - g.row_ptr[source];
  LevelCounters &c = ctl->cnt[2];
  c = LevelCounters();
  if (deg > hub) {
    const int64_t nch = (deg + chunk - 1) / chunk;
    for (int64_t k = 0; k < nch; ++k) c0[k] = make_int2(source, (int)k);
    c.nc = (unsigned long long)nch;
  } else {
    q0[0] = source;
    c.nq = 1;
  }
  c.nv = 1;
  c.mf = (unsigned long long)deg;
  ctl->cnt[0] = LevelCounters();
  ctl->cnt[1] = LevelCounters();
}

// Final pass (Section 3, BFS): every negative parent becomes -1.
__device__ inline void fixup_parents(int64_t n, int32_t *parent, int64_t tid, int64_t nthreads) {
  for (int64_t v = tid; v < n; v += nthreads) {
    const int32_t p = parent[v];
    if (p < -1) parent[v] = -1;
  }
}

}  // namespace gap
