// Single-source direction-optimizing BFS: the per-level steps as device
// functions, shared by the persistent cooperative kernel and by the
// one-launch-per-step kernels, so every schedule runs the same code.
#pragma once

#include "common.h"

namespace gap {

// Queue storage of one search.  The frontier F_d lives in buffer set bs =
// d & 1 as kGroups segments: vertex segment h is q[bs] + h * n, hub chunk
// segment h is c[bs] + h * ccap.  Segment sizes are published at the level
// boundary (Published::q / ::c).
struct Queues {
  int32_t *q0, *q1;  // vertex queues of buffer sets 0 and 1
  int2 *c0, *c1;     // hub chunk queues of buffer sets 0 and 1
  int64_t n;         // capacity of a vertex segment
  int64_t ccap;      // capacity of a chunk segment
  // Selected with a conditional, not an array index: a runtime index into
  // a pointer array would move the argument block to scratch memory.
  __device__ int32_t *qs(int bs) const { return bs ? q1 : q0; }
  __device__ int2 *cs(int bs) const { return bs ? c1 : c0; }
};

// Per-workgroup staging of appended vertices in LDS: a wave reserves slots
// with one LDS atomic; the workgroup copies the slots out with one device
// atomic per segment at the end of the step.  Slots beyond the capacity go
// straight to the segment (reserved with a device atomic).
// Hub claims are listed as {vertex, chunk count} and expanded into chunk
// items by the whole workgroup at the end of the step.
template <int BLOCK>
struct Stage {
  static constexpr int QCAP = BLOCK * 8;
  static constexpr int CCAP = 256;
  static constexpr int HCAP = BLOCK;
  int32_t q[QCAP];
  int2 c[CCAP];
  int32_t hv[HCAP];
  uint32_t hch[HCAP];  // chunk items of each hub claim, then their offsets
  uint32_t hwave[BLOCK / kWave];
  unsigned int qn, cn, hn;
  unsigned int hbase;
  unsigned long long hgbase;
  unsigned long long qbase, cbase;
  unsigned long long qpre[kGroups + 1];  // input segment prefix sums
  unsigned long long cpre[kGroups + 1];
  unsigned long long part[BLOCK / kWave][4];
};

struct StepArgs {
  DevGraph g;
  int32_t *parent;       // int32[n]: -degree (or kIsolated) while unvisited
  int32_t *depth;        // int32[n]
  Queues Q;
  int bs_in;             // buffer set holding F_d
  Ctl *ctl;
  const uint64_t *fbm;   // F_d bitmap (bottom-up)
  uint64_t *vbm;         // visited bitmap (bottom-up), padding bits set
  uint64_t *nbm;         // F_{d+1} bitmap written by bottom-up
  int32_t d;             // depth of the frontier being expanded
  int32_t hub;           // degree above which a vertex becomes chunk items
  int32_t chunk;         // edges per chunk item (multiple of 64)
};

struct LaneAcc {
  unsigned long long mf = 0, nv = 0, scanned = 0, unvisited = 0;
};

// Segment holding global index i of a segmented queue (prefix in LDS).
__device__ inline int seg_of(unsigned long long i, const unsigned long long *pre) {
  int h = 0;
#pragma unroll
  for (int s = kGroups / 2; s >= 1; s >>= 1)
    if (pre[h + s] <= i) h += s;
  return h;
}

// Appends the vertices with `want` set to this workgroup's staged vertex
// queue (one LDS atomic per wave; overflow goes to the group's segment).
template <int BLOCK>
__device__ inline void stage_vertices(const StepArgs &a, Stage<BLOCK> &st, bool want, int32_t v) {
  const uint64_t ms = __ballot(want);
  if (!ms) return;
  const int lane = lane_id();
  const int g = (int)(blockIdx.x % kGroups);
  const int bs_out = a.bs_in ^ 1;
  const int leader = first_lane(ms);
  const unsigned int cnt = (unsigned int)__popcll(ms);
  unsigned int base = 0;
  if (lane == leader) base = atomicAdd(&st.qn, cnt);
  base = __shfl(base, leader, kWave);
  const unsigned int cap = Stage<BLOCK>::QCAP;
  const unsigned int ov_start = base > cap ? base : cap;
  const unsigned int n_ov = base + cnt > cap ? base + cnt - ov_start : 0u;
  unsigned long long gbase = 0;
  if (n_ov) {
    if (lane == leader) gbase = atomicAdd(&a.ctl->seg[bs_out][g].q, (unsigned long long)n_ov);
    gbase = __shfl(gbase, leader, kWave);
  }
  if (want) {
    const unsigned int slot = base + lane_rank(ms);
    if (slot < cap)
      st.q[slot] = v;
    else
      a.Q.qs(bs_out)[g * a.Q.n + (int64_t)(gbase + (slot - ov_start))] = v;
  }
}

// Appends ceil(deg/chunk) chunk items {v, k | flag} for every lane with
// `want` set.  The whole wave writes them (item i belongs to the lane whose
// prefix range holds i), so a hub never leaves one lane looping alone.
template <int BLOCK>
__device__ inline void stage_chunks(const StepArgs &a, Stage<BLOCK> &st, bool want, int32_t v,
                                    int64_t degv, int flag) {
  const uint64_t mb = __ballot(want);
  if (!mb) return;
  const int lane = lane_id();
  const int g = (int)(blockIdx.x % kGroups);
  const int bs_out = a.bs_in ^ 1;
  const uint32_t nch = want ? (uint32_t)((degv + a.chunk - 1) / a.chunk) : 0u;
  uint32_t total;
  const uint32_t off = wave_excl_scan_u32(nch, total);
  const int leader = first_lane(mb);
  unsigned int base = 0;
  if (lane == leader) base = atomicAdd(&st.cn, total);
  base = __shfl(base, leader, kWave);
  const unsigned int cap = Stage<BLOCK>::CCAP;
  const unsigned int ov_start = base > cap ? base : cap;
  const unsigned int n_ov = base + total > cap ? base + total - ov_start : 0u;
  unsigned long long gbase = 0;
  if (n_ov) {
    if (lane == leader) gbase = atomicAdd(&a.ctl->seg[bs_out][g].c, (unsigned long long)n_ov);
    gbase = __shfl(gbase, leader, kWave);
  }
  for (uint32_t i0 = 0; i0 < total; i0 += kWave) {
    const uint32_t i = i0 + (uint32_t)lane;
    int j = 0;
#pragma unroll
    for (int step = 32; step >= 1; step >>= 1) {
      const uint32_t oc = __shfl(off, j + step, kWave);
      if (oc <= i) j += step;  // largest j with off_j <= i owns item i
    }
    const int32_t vj = __shfl(v, j, kWave);
    const uint32_t oj = __shfl(off, j, kWave);
    if (i < total) {
      const unsigned int slot = base + i;
      const int2 item = make_int2(vj, (int)(i - oj) | flag);
      if (slot < cap)
        st.c[slot] = item;
      else
        a.Q.cs(bs_out)[g * a.Q.ccap + (int64_t)(gbase + (slot - ov_start))] = item;
    }
  }
}

// Lists hub claims {v, chunk count} for expand_hubs; claims beyond the
// list's capacity are expanded by the wave at once.
template <int BLOCK>
__device__ inline void stage_hubs(const StepArgs &a, Stage<BLOCK> &st, bool want, int32_t v,
                                  int64_t degv) {
  const uint64_t mb = __ballot(want);
  if (!mb) return;
  const int lane = lane_id();
  const int leader = first_lane(mb);
  unsigned int base = 0;
  if (lane == leader) base = atomicAdd(&st.hn, (unsigned int)__popcll(mb));
  base = __shfl(base, leader, kWave);
  const unsigned int slot = base + lane_rank(mb);
  const bool fits = want && slot < (unsigned int)Stage<BLOCK>::HCAP;
  if (fits) {
    st.hv[slot] = v;
    st.hch[slot] = (uint32_t)((degv + a.chunk - 1) / a.chunk);
  }
  stage_chunks<BLOCK>(a, st, want && !fits, v, degv, 0);
}

// Whole workgroup, after a barrier: the listed hub claims become chunk
// items (staged like stage_chunks's, so step_end copies them out).  The
// claiming wave alone would write a hub frontier's items one after another
// (R-MAT 22's first levels claim thousands of hubs, ~10 items each).
template <int BLOCK>
__device__ inline void expand_hubs(const StepArgs &a, Stage<BLOCK> &st) {
  const unsigned int hn0 = st.hn;
  if (hn0 == 0) return;  // uniform: read after a barrier
  const unsigned int hn = hn0 < (unsigned int)Stage<BLOCK>::HCAP ? hn0 : Stage<BLOCK>::HCAP;
  const int t = threadIdx.x;
  const int wv = t / kWave;
  const uint32_t mine = (unsigned int)t < hn ? st.hch[t] : 0u;  // HCAP == BLOCK: one per thread
  uint32_t wtot = 0;
  uint32_t off = wave_excl_scan_u32(mine, wtot);
  if (lane_id() == 0) st.hwave[wv] = wtot;
  __syncthreads();
  uint32_t total = 0;
  for (int w = 0; w < BLOCK / kWave; ++w) {
    if (w < wv) off += st.hwave[w];
    total += st.hwave[w];
  }
  if ((unsigned int)t < hn) st.hch[t] = off;  // only thread t reads hch[t] above
  const int g = (int)(blockIdx.x % kGroups);
  const int bs_out = a.bs_in ^ 1;
  const unsigned int cap = Stage<BLOCK>::CCAP;
  if (t == 0) {
    const unsigned int base = atomicAdd(&st.cn, total);
    const unsigned int ov_start = base > cap ? base : cap;
    const unsigned int n_ov = base + total > cap ? base + total - ov_start : 0u;
    st.hbase = base;
    st.hgbase = n_ov ? atomicAdd(&a.ctl->seg[bs_out][g].c, (unsigned long long)n_ov) : 0ull;
    st.hn = 0;
  }
  __syncthreads();
  const unsigned int base = st.hbase;
  const unsigned int ov_start = base > cap ? base : cap;
  const unsigned long long gbase = st.hgbase;
  for (uint32_t i = (uint32_t)t; i < total; i += BLOCK) {
    uint32_t lo = 0, hi = hn;  // the claim whose range holds item i (every hub has items)
    while (hi - lo > 1) {
      const uint32_t mid = (lo + hi) / 2;
      if (st.hch[mid] <= i)
        lo = mid;
      else
        hi = mid;
    }
    const int2 item = make_int2(st.hv[lo], (int)(i - st.hch[lo]));
    const unsigned int slot = base + i;
    if (slot < cap)
      st.c[slot] = item;
    else
      a.Q.cs(bs_out)[g * a.Q.ccap + (int64_t)(gbase + (slot - ov_start))] = item;
  }
  __syncthreads();
}

// Appends this wave's newly reached vertices to F_{d+1}: degree <= hub ->
// vertex queue, larger -> chunk items so that one hub is expanded by many
// waves; accumulates the frontier totals.
template <int BLOCK>
__device__ inline void stage_append(const StepArgs &a, Stage<BLOCK> &st, bool claimed, int32_t v,
                                    int64_t degv, LaneAcc &acc) {
  if (__ballot(claimed) == 0ull) return;
  const bool big = claimed && degv > a.hub;
  stage_vertices<BLOCK>(a, st, claimed && !big, v);
  stage_hubs<BLOCK>(a, st, big, v, degv);
  if (claimed) {
    acc.mf += (unsigned long long)degv;
    acc.nv += 1;
  }
}

// Start of a step (all threads): load the input segment prefix sums of
// pub[d & 1] (only a step that reads the queues needs them: `segments`)
// and clear the staging counters.
template <int BLOCK>
__device__ inline void step_begin(const StepArgs &a, Stage<BLOCK> &st, bool segments = true) {
  if (threadIdx.x < kWave && !segments) {
    if (threadIdx.x == 0) {
      st.qn = 0;
      st.cn = 0;
      st.hn = 0;
    }
  } else if (threadIdx.x < kWave) {
    // lane h < kGroups loads segment h's sizes: one round trip, not 2*kGroups
    const int lane = threadIdx.x;
    const Published &P = a.ctl->pub[a.d & 1];
    const uint32_t q = lane < kGroups ? (uint32_t)ld_agent(&P.q[lane]) : 0u;
    const uint32_t c = lane < kGroups ? (uint32_t)ld_agent(&P.c[lane]) : 0u;
    uint32_t tq, tc;
    const uint32_t oq = wave_excl_scan_u32(q, tq);
    const uint32_t oc = wave_excl_scan_u32(c, tc);
    if (lane <= kGroups) {
      st.qpre[lane] = lane < kGroups ? oq : tq;
      st.cpre[lane] = lane < kGroups ? oc : tc;
    }
    if (lane == 0) {
      st.qn = 0;
      st.cn = 0;
      st.hn = 0;
    }
  }
  __syncthreads();
}

// End of a step (all threads): copy staged vertices to this group's
// segments (one device atomic per segment per workgroup) and reduce the
// workgroup's totals into thread 0.  HUBS: the step listed hub claims
// (stage_append does; callers that stage chunks directly pass false).
template <int BLOCK, bool HUBS = true>
__device__ inline Totals step_end(const StepArgs &a, Stage<BLOCK> &st, LaneAcc &acc) {
  const int wv = threadIdx.x / kWave;
  // a wave that counted nothing (most waves of a small level) skips the
  // cross-lane reductions
  const bool any = __ballot((acc.mf | acc.nv | acc.scanned | acc.unvisited) != 0ull) != 0ull;
  unsigned long long s0 = 0, s1 = 0, s2 = 0, s3 = 0;
  if (any) {
    s0 = wave_sum_u64(acc.mf);
    s1 = wave_sum_u64(acc.nv);
    s2 = wave_sum_u64(acc.scanned);
    s3 = wave_sum_u64(acc.unvisited);
  }
  if (lane_id() == 0) {
    st.part[wv][0] = s0;
    st.part[wv][1] = s1;
    st.part[wv][2] = s2;
    st.part[wv][3] = s3;
  }
  __syncthreads();
  if (HUBS) expand_hubs<BLOCK>(a, st);
  const int g = (int)(blockIdx.x % kGroups);
  const int bs_out = a.bs_in ^ 1;
  const unsigned int nq = st.qn < (unsigned)Stage<BLOCK>::QCAP ? st.qn : Stage<BLOCK>::QCAP;
  const unsigned int nc = st.cn < (unsigned)Stage<BLOCK>::CCAP ? st.cn : Stage<BLOCK>::CCAP;
  if (threadIdx.x == 0) {
    st.qbase = nq ? atomicAdd(&a.ctl->seg[bs_out][g].q, (unsigned long long)nq) : 0ull;
    st.cbase = nc ? atomicAdd(&a.ctl->seg[bs_out][g].c, (unsigned long long)nc) : 0ull;
  }
  __syncthreads();
  int32_t *qdst = a.Q.qs(bs_out) + g * a.Q.n + (int64_t)st.qbase;
  for (unsigned int i = threadIdx.x; i < nq; i += BLOCK) qdst[i] = st.q[i];
  int2 *cdst = a.Q.cs(bs_out) + g * a.Q.ccap + (int64_t)st.cbase;
  for (unsigned int i = threadIdx.x; i < nc; i += BLOCK) cdst[i] = st.c[i];
  Totals t = {};
  if (threadIdx.x < kWave) {  // wave 0 folds the per-wave partials, one lane per wave
    const int l = threadIdx.x;
    const bool has = l < BLOCK / kWave;
    t.mf = wave_sum_u64(has ? st.part[l][0] : 0ull);
    t.nv = wave_sum_u64(has ? st.part[l][1] : 0ull);
    t.scanned = wave_sum_u64(has ? st.part[l][2] : 0ull);
    t.unvisited = wave_sum_u64(has ? st.part[l][3] : 0ull);
  }
  acc = LaneAcc();
  return t;
}

// Tries the claims (v[k] for parent u[k], v[k] < 0 = no edge) of four edge
// batches at once: the parent probes, then the CAS claims, are issued
// back-to-back so their latencies overlap; then the winners are appended.
template <int BLOCK, bool STATS, int NK = 4>
__device__ __forceinline__ void td_claim4(const StepArgs &a, Stage<BLOCK> &st, LaneAcc &acc,
                                 const int32_t (&v)[4], const int32_t (&u)[4]) {
  // loads without branches: a load under a per-lane condition gets a block
  // of its own that waits for it before the next load issues
  int32_t p[4];
#pragma unroll
  for (int k = 0; k < NK; ++k) p[k] = a.parent[v[k] >= 0 ? v[k] : u[k]];
#pragma unroll
  for (int k = 0; k < NK; ++k) p[k] = v[k] >= 0 ? p[k] : 0;
  bool claimed[4];
#pragma unroll
  for (int k = 0; k < NK; ++k) {
    claimed[k] = false;
    if (v[k] >= 0 && p[k] < 0) claimed[k] = atomicCAS(&a.parent[v[k]], p[k], u[k]) == p[k];
  }
#pragma unroll
  for (int k = 0; k < NK; ++k) {
    int64_t degv = 0;
    if (claimed[k]) {
      a.depth[v[k]] = a.d + 1;
      degv = (p[k] == kIsolated) ? 0 : -(int64_t)p[k];
    }
    if (STATS && v[k] >= 0) acc.scanned += 1;
    stage_append<BLOCK>(a, st, claimed[k], v[k], degv, acc);
  }
}

// Plain-store claims of four edge batches: every v[k] that a probe finds
// unvisited gets parent u[k] and depth d + 1 by ordinary stores.  Several
// frontier vertices may write one v; whichever store lands is a frontier
// neighbour, so the parent is valid and the depth the same.  Nothing is
// appended: F_{d+1} is read back from the depths after the level's barrier
// (convert_to_bitmaps with totals), which also counts it exactly once.
template <bool STATS, int NK = 4>
__device__ __forceinline__ void td_plain4(const StepArgs &a, LaneAcc &acc, const int32_t (&v)[4],
                                 const int32_t (&u)[4]) {
  int32_t p[4];
#pragma unroll
  for (int k = 0; k < NK; ++k) p[k] = a.parent[v[k] >= 0 ? v[k] : u[k]];
#pragma unroll
  for (int k = 0; k < NK; ++k) {
    if (v[k] >= 0 && p[k] < 0) {
      a.parent[v[k]] = u[k];
      a.depth[v[k]] = a.d + 1;
    }
    if (STATS && v[k] >= 0) acc.scanned += 1;
  }
}

// Claims of a round of up to four edge batches, `left` edges from the
// round's first (wave-uniform): a round of at most 64 edges (the common
// case on small frontiers) probes and claims one batch, not four of which
// three are empty.
template <int BLOCK, bool STATS, bool PLAIN>
__device__ __forceinline__ void td_claims(const StepArgs &a, Stage<BLOCK> &st, LaneAcc &acc,
                                 const int32_t (&v)[4], const int32_t (&u)[4], int64_t left) {
  if (left <= kWave) {
    if constexpr (PLAIN)
      td_plain4<STATS, 1>(a, acc, v, u);
    else
      td_claim4<BLOCK, STATS, 1>(a, st, acc, v, u);
  } else {
    if constexpr (PLAIN)
      td_plain4<STATS>(a, acc, v, u);
    else
      td_claim4<BLOCK, STATS>(a, st, acc, v, u);
  }
}

// Top-down step: every edge (u, v) with u in F_d is tried once.
//  * hub chunk items: one wave walks `chunk` consecutive edges of one hub,
//    256 edges per round;
//  * queue vertices: a wave takes 64 queued vertices, prefix-sums their
//    degrees and walks the combined edge range 256 edges per round, each
//    lane finding the owner vertex of its edges by a binary search over the
//    64 offsets held in registers (no lane idles on a short list).
// SPREAD: hand the items round the workgroups first (the persistent
// kernel); the per-level kernels keep consecutive items on a workgroup's
// waves, which measured faster there (17.6 against 20.7 us per level on a
// 4096^2 grid).  PLAIN: claims by plain stores (td_plain4), no appends.
template <int BLOCK, bool STATS, bool SPREAD = false, bool PLAIN = false>
__device__ __forceinline__ void td_step(const StepArgs &a, Stage<BLOCK> &st, LaneAcc &acc, int64_t gwave,
                        int64_t nwaves) {
  const int lane = lane_id();
  const int2 *cin = a.Q.cs(a.bs_in);
  const int32_t *qin = a.Q.qs(a.bs_in);
  // Work goes round the workgroups first (item i to wave i / nblk of
  // workgroup i % nblk), so the items of a small frontier, and the claims
  // they make, spread over every workgroup's staging and hub list.
  constexpr int kWpb = BLOCK / kWave;
  const int64_t nblk = nwaves / kWpb;
  if (SPREAD) gwave = (gwave % kWpb) * nblk + gwave / kWpb;
  const unsigned long long nc = st.cpre[kGroups];
  for (unsigned long long ci = (unsigned long long)gwave; ci < nc; ci += (unsigned long long)nwaves) {
    const int h = seg_of(ci, st.cpre);
    const int2 it = cin[h * a.Q.ccap + (int64_t)(ci - st.cpre[h])];
    const int32_t uu = it.x;
    const int64_t rbeg = a.g.row_ptr[uu], rend = a.g.row_ptr[uu + 1];
    const int64_t beg = rbeg + (int64_t)it.y * a.chunk;
    const int64_t end = beg + a.chunk < rend ? beg + a.chunk : rend;
    for (int64_t e0 = beg; e0 < end; e0 += 4 * kWave) {
      int32_t v[4], u[4];
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const int64_t e = e0 + k * kWave + lane;
        const int32_t x = a.g.col[e < end ? e : beg];
        v[k] = e < end ? x : -1;
        u[k] = uu;
      }
      td_claims<BLOCK, STATS, PLAIN>(a, st, acc, v, u, end - e0);
    }
  }
  // Vertices per wave: up to 64, fewer when the frontier is small so that
  // every wave gets work (a small frontier on a few waves would run many
  // dependent rounds on each).
  const unsigned long long nq = st.qpre[kGroups];
  unsigned long long per = (nq + (unsigned long long)nwaves - 1) / (unsigned long long)nwaves;
  per = per < 1 ? 1 : (per > (unsigned long long)kWave ? (unsigned long long)kWave : per);
  const unsigned long long ngroups = (nq + per - 1) / per;
  for (unsigned long long gi = (unsigned long long)gwave; gi < ngroups;
       gi += (unsigned long long)nwaves) {
    const unsigned long long idx = gi * per + lane;
    const bool has = (unsigned long long)lane < per && idx < nq;
    const unsigned long long ix = has ? idx : gi * per;  // gi * per < nq: a valid entry
    const int h = seg_of(ix, st.qpre);
    const int32_t ur = qin[h * a.Q.n + (int64_t)(ix - st.qpre[h])];
    const int64_t b0 = a.g.row_ptr[ur], b1 = a.g.row_ptr[ur + 1];
    const int32_t uo = has ? ur : -1;
    const int64_t beg = has ? b0 : 0;
    const uint32_t deg = has ? (uint32_t)(b1 - b0) : 0u;
    uint32_t total;
    const uint32_t off = wave_excl_scan_u32(deg, total);
    // edge e of the combined range -> its owner u and its list entry (idle
    // lanes, e >= total, take the last edge's entry, encoded -entry - 1)
    auto locate = [&](uint32_t e_raw, int32_t &uk, int64_t &eak) {
      const uint32_t e = e_raw < total ? e_raw : total - 1;
      int j = 0;
#pragma unroll
      for (int step = 32; step >= 1; step >>= 1) {
        uint32_t oc = __shfl(off, j + step, kWave);
        if (oc <= e) j += step;
      }
      uk = __shfl(uo, j, kWave);
      const int64_t bj = __shfl(beg, j, kWave);
      const uint32_t oj = __shfl(off, j, kWave);
      eak = e_raw < total ? bj + (int64_t)(e - oj) : -(bj + (int64_t)(e - oj)) - 1;
    };
    for (uint32_t b = 0; b < total; b += 4 * kWave) {
      int32_t v[4], u[4];
      int64_t ea[4];
      // a round of at most 64 edges locates and loads one batch only
      const int nk = total - b <= (uint32_t)kWave ? 1 : 4;
      locate(b + (uint32_t)lane, u[0], ea[0]);
#pragma unroll
      for (int k = 1; k < 4; ++k) {
        if (nk == 4) {
          locate(b + (uint32_t)(k * kWave + lane), u[k], ea[k]);
        } else {  // idle batches: batch 0's entry, so their loads touch its lines
          u[k] = u[0];
          ea[k] = ea[0] >= 0 ? -ea[0] - 1 : ea[0];
        }
      }
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const int32_t x = a.g.col[ea[k] >= 0 ? ea[k] : -ea[k] - 1];
        v[k] = ea[k] >= 0 ? x : -1;
      }
      td_claims<BLOCK, STATS, PLAIN>(a, st, acc, v, u, (int64_t)(total - b));
    }
  }
}

// Bottom-up step: each unvisited vertex scans its neighbours in order and
// stops at the first one in F_d.  Lane i of a wave owns vertex 64w+i, so the
// next-frontier and visited words come from one ballot with a single writer
// (no atomics); words whose 64 vertices are all visited are skipped whole.
// The step is bound by load latency (visited word -> row offsets ->
// neighbours -> frontier bits), so a wave works on J words at once and
// fetches a run of neighbours per vertex per round: 4 in the first round,
// then R2 (a wave runs until its slowest vertex is done, so vertices that
// missed four times get longer runs and the wave fewer rounds).  Runs are
// read 16 bytes at a time (the column arrays are padded).  The first hit in
// list order wins.
#ifndef GAP_BU_WORDS
#define GAP_BU_WORDS 4
#endif
#ifndef GAP_BU_ROUND2
#define GAP_BU_ROUND2 4
#endif

// The frontier bitmap F_d as a bottom-up step probes it: words [0, lw) from
// the workgroup's LDS copy, the rest from global memory (the L2-held copy).
// Adjacency lists are sorted, so the first entries of a list (those a
// bottom-up search reads first, and most often stops at) are the smallest
// vertex ids: an LDS copy of the low words of the bitmap takes most of the
// probes even when the whole bitmap does not fit.
struct FrontierBits {
  const uint64_t *lds;
  int64_t lw;
  const uint64_t *g;
  int32_t spare;  // a vertex of this wave's own (see wave_spare_vertex)
  // u < 0 (no entry) tests false; the load is issued for every lane (a
  // flat load when the LDS copy is in use), with no branch around it
  __device__ __forceinline__ bool test(int32_t u) const {
    const int32_t uu = u < 0 ? spare : u;
    const int64_t w = uu >> 6;
    const uint64_t *p = w < lw ? lds + w : g + w;
    const uint64_t word = *p;
    return (u >= 0) & (((word >> (uu & 63)) & 1ull) != 0);
  }
};

// A vertex id that depends only on the wave (waves spread 1024 vertices
// apart): lanes that have nothing to load use it for their address, so the
// loads of an idle lane touch a line of their own wave's instead of one line
// every wave of the grid would share.
template <int BLOCK>
__device__ inline int32_t wave_spare_vertex(int64_t n) {
  const uint64_t w = (uint64_t)blockIdx.x * (BLOCK / kWave) + threadIdx.x / kWave;
  return (int32_t)((w * 1024ull) % (uint64_t)n);
}

// Copies the first lw words of F_d into LDS (whole workgroup, then a
// workgroup barrier); lw = 0 keeps every probe on the global copy.
template <int BLOCK>
__device__ inline FrontierBits frontier_bits(const StepArgs &a, uint64_t *lfbm, int64_t lw) {
  const int64_t nwords = (a.g.n + kWave - 1) / kWave;
  if (!lfbm) lw = 0;
  if (lw > nwords) lw = nwords;
  for (int64_t i = threadIdx.x; i < lw; i += BLOCK) lfbm[i] = a.fbm[i];
  if (lw) __syncthreads();
  return FrontierBits{lfbm, lw, a.fbm, wave_spare_vertex<BLOCK>(a.g.n)};
}

// One round over the J vertices of a lane: RR entries each from e[j] on.
// Returns whether any of them is still searching.
template <int J, int RR, bool STATS>
__device__ inline bool bu_round(const int32_t *__restrict__ col, const FrontierBits &fb, bool (&act)[J],
                                int64_t (&e)[J], int32_t (&rem)[J], int32_t (&pu)[J], LaneAcc &acc,
                                int64_t spare_e) {
  static_assert(RR % 4 == 0, "runs are read 16 bytes at a time");
  int32_t u[J][RR];
#pragma unroll
  for (int j = 0; j < J; ++j)
#pragma unroll
    for (int q = 0; q < RR / 4; ++q) {
      const bool use = act[j] && 4 * q < rem[j];
      const i32x4_a4 w = *reinterpret_cast<const i32x4_a4 *>(col + (use ? e[j] + 4 * q : spare_e));
#pragma unroll
      for (int k = 0; k < 4; ++k) u[j][4 * q + k] = (use && 4 * q + k < rem[j]) ? w[k] : -1;
    }
  bool hit[J][RR];
#pragma unroll
  for (int j = 0; j < J; ++j)
#pragma unroll
    for (int k = 0; k < RR; ++k)
      hit[j][k] = fb.test(u[j][k]);
  bool more = false;
#pragma unroll
  for (int j = 0; j < J; ++j) {
    if (!act[j]) continue;
#pragma unroll
    for (int k = RR - 1; k >= 0; --k)
      if (hit[j][k]) pu[j] = u[j][k];
    if (STATS) {  // entries up to and including the first hit
      int used = 0;
      for (int k = 0; k < RR && k < rem[j]; ++k) {
        ++used;
        if (hit[j][k]) break;
      }
      acc.scanned += used;
    }
    e[j] += RR;
    rem[j] -= RR;
    if (pu[j] >= 0 || rem[j] <= 0)
      act[j] = false;
    else
      more = true;
  }
  return more;
}

// lfbm: when not NULL, LDS room for the first lw words of the frontier
// bitmap; the step first copies them there and probes LDS for them
// instead of the L2-held copy.
// QUEUE: also append F_{d+1} to the vertex queue (and hub chunk items); a
// caller that passes false only counts the totals, and turns the bitmap
// into a queue itself when a top-down step follows (queue_from_bitmap).
template <int BLOCK, bool STATS, int J = GAP_BU_WORDS, int R2 = GAP_BU_ROUND2, bool QUEUE = true>
__device__ void bu_step(const StepArgs &a, Stage<BLOCK> &st, LaneAcc &acc, int64_t gwave,
                        int64_t nwaves, uint64_t *lfbm = nullptr, int64_t lw = 0) {
  const int lane = lane_id();
  const int64_t nwords = (a.g.n + kWave - 1) / kWave;
  const FrontierBits fb = frontier_bits<BLOCK>(a, lfbm, lw);
  // list offset an idle lane reads (a valid 16-byte run: the column array
  // has kColPad entries beyond its last list)
  const int64_t spare_e = a.g.row_ptr_in[fb.spare];
  for (int64_t base = gwave * J; base < nwords; base += nwaves * J) {
    uint64_t vis[J];
    int64_t e[J];       // next adjacency entry
    int32_t rem[J];     // entries left (a degree fits in 31 bits)
    int32_t degv[J];
    int32_t pu[J];
    bool act[J];
#pragma unroll
    for (int j = 0; j < J; ++j) vis[j] = (base + j < nwords) ? a.vbm[base + j] : ~0ull;
#pragma unroll
    for (int j = 0; j < J; ++j) {
      const int64_t v = (base + j) * kWave + lane;
      act[j] = ((vis[j] >> lane) & 1ull) == 0ull;
      e[j] = 0;
      rem[j] = 0;
      pu[j] = -1;
      if (act[j]) {
        e[j] = a.g.row_ptr_in[v];
        rem[j] = (int32_t)(a.g.row_ptr_in[v + 1] - e[j]);
        if (STATS) acc.unvisited += 1;
      }
      degv[j] = rem[j];
    }
    bool more = bu_round<J, 4, STATS>(a.g.col_in, fb, act, e, rem, pu, acc, spare_e);
    while (__ballot(more) != 0ull)
      more = bu_round<J, R2, STATS>(a.g.col_in, fb, act, e, rem, pu, acc, spare_e);
#pragma unroll
    for (int j = 0; j < J; ++j) {
      const bool found = pu[j] >= 0;
      const int64_t v = (base + j) * kWave + lane;
      if (found) {
        a.parent[v] = pu[j];
        a.depth[v] = a.d + 1;
        // the next frontier's edges are out-edges: on a directed graph the
        // in-degree read above is not the count the top-down side needs
        if (a.g.directed) degv[j] = (int32_t)(a.g.row_ptr[v + 1] - a.g.row_ptr[v]);
      }
      const uint64_t b = __ballot(found);
      if (base + j < nwords && lane == 0) {
        a.nbm[base + j] = b;
        if (b) a.vbm[base + j] = vis[j] | b;
      }
      if (QUEUE) {
        stage_append<BLOCK>(a, st, found, (int32_t)v, (int64_t)degv[j], acc);
      } else if (found) {
        acc.mf += (unsigned long long)degv[j];
        acc.nv += 1;
      }
    }
  }
}

// Position of the k-th set bit (k from 0) of x, which has more than k.
__device__ inline int nth_set_bit(uint64_t x, uint32_t k) {
  int pos = 0;
#pragma unroll
  for (int half = 32; half >= 1; half >>= 1) {
    const uint32_t c = (uint32_t)__popcll(x & ((1ull << half) - 1ull));
    if (k >= c) {
      k -= c;
      x >>= half;
      pos += half;
    }
  }
  return pos;
}

// Bottom-up step with refilled lanes (persistent schedule, no queue).
// Workgroup b owns the contiguous words [wlo, whi) of the vertex range and
// hands them to its waves kBuChunk words at a time (an LDS cursor).  A lane
// holds J vertices at once; every round reads four list entries of each held
// vertex (one 16-byte load: the vertex's head record in its first round, so
// that vertices handed out in order read consecutive records, then the
// column array) and probes the frontier bitmap for them; a vertex
// that found its parent (its first frontier neighbour in list order) or ran
// out of entries frees its slot, and the wave refills free slots from its
// chunk before the next round.  So lanes do not idle while a wave's slowest
// vertices finish, as they would if a wave kept a fixed set of vertices until
// all of them were done.  Found vertices are collected in an LDS bitmap of the
// workgroup's words (it reuses the vertex staging, which a step without a
// queue leaves empty); after the last round the workgroup writes each of its
// words of the next frontier and of the visited bitmap once.
// Requires whi - wlo <= bu_refill_words<BLOCK>().
constexpr int kBuChunk = 16;
// Vertices a lane holds at once (four keep the kernel within 128 VGPRs only
// with spills).
#ifndef GAP_BU_SLOTS
#define GAP_BU_SLOTS 3
#endif
// List entries a round reads for a vertex past its head record (a multiple
// of 4: 16-byte loads).
#ifndef GAP_BU_RUN
#define GAP_BU_RUN 4
#endif

template <int BLOCK>
__host__ __device__ constexpr int64_t bu_refill_words() {
  return (int64_t)(Stage<BLOCK>::QCAP * sizeof(int32_t) / sizeof(uint64_t));
}

template <int BLOCK, bool STATS, int J>
__device__ __forceinline__ void bu_step_refill(const StepArgs &a, Stage<BLOCK> &st, LaneAcc &acc, int64_t wlo,
                               int64_t whi, uint64_t *lfbm, int64_t lw) {
  uint64_t *found = reinterpret_cast<uint64_t *>(st.q);
  unsigned int *cursor = &st.hbase;
  const int lane = lane_id();
  const int64_t nw = whi > wlo ? whi - wlo : 0;
  for (int64_t i = threadIdx.x; i < nw; i += BLOCK) found[i] = 0ull;
  if (threadIdx.x == 0) *cursor = 0u;
  const FrontierBits fb = frontier_bits<BLOCK>(a, lfbm, lw);
  __syncthreads();
  const int32_t *__restrict__ col = a.g.col_in;
  const int64_t *__restrict__ rp = a.g.row_ptr_in;

  int32_t v[J];    // held vertex, -1 = free slot
  int64_t e[J];    // next list entry
  int32_t rem[J];  // entries left
  int32_t deg[J];  // list length (the frontier-edge count of an undirected find)
  bool fresh[J];   // the first four entries are read from the vertex's head record
#pragma unroll
  for (int j = 0; j < J; ++j) {
    v[j] = -1;
    e[j] = 0;
    rem[j] = 0;
    deg[j] = 0;
    fresh[j] = false;
  }
  uint64_t win = 0ull;  // this lane's word of the chunk: unvisited bits not yet handed out
  int64_t wbase = 0;    // first word of the chunk (wave-uniform)
  uint32_t wleft = 0;   // vertices of the chunk not yet handed out (wave-uniform)
  bool more = nw > 0;   // chunks left in the range (wave-uniform)
  for (;;) {
    // ---- refill the free slots, row by row, in vertex order ----
    for (;;) {
      uint64_t fm[J];
      uint32_t nfree = 0;
#pragma unroll
      for (int j = 0; j < J; ++j) {
        fm[j] = __ballot(v[j] < 0);
        nfree += (uint32_t)__popcll(fm[j]);
      }
      if (nfree == 0u) break;
      if (wleft == 0u) {
        if (!more) break;
        unsigned int c0 = 0;
        if (lane == 0) c0 = atomicAdd(cursor, (unsigned int)kBuChunk);
        c0 = uni((uint32_t)__shfl((int)c0, 0, kWave));
        if ((int64_t)c0 >= nw) {
          more = false;
          break;
        }
        wbase = wlo + (int64_t)c0;
        win = (lane < kBuChunk && (int64_t)c0 + lane < nw) ? ~a.vbm[wbase + lane] : 0ull;
        wleft = uni((uint32_t)wave_sum_u64((unsigned long long)__popcll(win)));
        continue;
      }
      const uint32_t cnt = (uint32_t)__popcll(win);
      uint32_t tot;
      const uint32_t off = wave_excl_scan_u32(cnt, tot);
      if (tot == 0u) {  // the chunk is used up: take the next one
        wleft = 0u;
        continue;
      }
      const uint32_t take = nfree < tot ? nfree : tot;
      uint32_t base = 0;
#pragma unroll
      for (int j = 0; j < J; ++j) {
        const bool isfree = (fm[j] >> lane) & 1ull;
        uint32_t r = base + lane_rank(fm[j]);
        base += (uint32_t)__popcll(fm[j]);
        const bool gets = isfree && r < take;
        if (!gets) r = 0;
        int jw = 0;  // the chunk word holding handed-out position r: largest jw with off <= r
#pragma unroll
        for (int step = 32; step >= 1; step >>= 1) {
          const uint32_t oc = (uint32_t)__shfl((int)off, jw + step, kWave);
          if (oc <= r && jw + step < kBuChunk) jw += step;
        }
        const uint64_t bw = (uint64_t)__shfl((long long)win, jw, kWave);
        const uint32_t ow = (uint32_t)__shfl((int)off, jw, kWave);
        // the row offsets are loaded by every lane (vertex 0 for lanes that
        // take nothing): no branch around the loads
        const int64_t vv = gets ? (wbase + jw) * kWave + nth_set_bit(bw, r - ow) : (int64_t)fb.spare;
        const int64_t r0 = rp[vv], r1 = rp[vv + 1];
        if (gets) {
          v[j] = (int32_t)vv;
          e[j] = r0;
          rem[j] = (int32_t)(r1 - r0);
          deg[j] = rem[j];
          fresh[j] = true;
          if (STATS) acc.unvisited += 1;
        }
      }
      // each chunk word drops the bits it handed out (the lowest ones)
      const int t = (int)take - (int)off;
      if (t > 0) win = t >= (int)cnt ? 0ull : (win & ~((2ull << nth_set_bit(win, (uint32_t)t - 1u)) - 1ull));
      wleft = tot - take;
    }
    bool held = false;
#pragma unroll
    for (int j = 0; j < J; ++j) held |= v[j] >= 0;
    if (__ballot(held) == 0ull) break;
    // ---- one round: the head record (four entries) of a fresh vertex,
    // RUN entries of the column array for one that missed before ----
    constexpr int RUN = GAP_BU_RUN;
    int32_t u[J][RUN];
    int32_t adv[J];
    i32x4_a4 w[J][RUN / 4];
    // every slot's loads first, then the entries (a use right after each
    // load would make the next load wait for it)
#pragma unroll
    for (int j = 0; j < J; ++j)
#pragma unroll
      for (int q = 0; q < RUN / 4; ++q) {
        const bool use = v[j] >= 0 && 4 * q < rem[j] && (q == 0 || !fresh[j]);
        const int32_t *src = !use ? reinterpret_cast<const int32_t *>(a.g.head_in + fb.spare)
                             : fresh[j] ? reinterpret_cast<const int32_t *>(a.g.head_in + v[j])
                                        : col + e[j] + 4 * q;
        w[j][q] = *reinterpret_cast<const i32x4_a4 *>(src);
      }
#pragma unroll
    for (int j = 0; j < J; ++j) {
      const bool head = fresh[j];
      adv[j] = head ? 4 : RUN;
#pragma unroll
      for (int q = 0; q < RUN / 4; ++q) {
        const bool use = v[j] >= 0 && 4 * q < rem[j] && (q == 0 || !head);
#pragma unroll
        for (int k = 0; k < 4; ++k)
          u[j][4 * q + k] = (use && 4 * q + k < rem[j] && 4 * q + k < adv[j]) ? w[j][q][k] : -1;
      }
      fresh[j] = false;
    }
    bool hit[J][RUN];
#pragma unroll
    for (int j = 0; j < J; ++j)
#pragma unroll
      for (int k = 0; k < RUN; ++k)
        hit[j][k] = fb.test(u[j][k]);
#pragma unroll
    for (int j = 0; j < J; ++j) {
      if (v[j] < 0) continue;
      int32_t pu = -1;
#pragma unroll
      for (int k = RUN - 1; k >= 0; --k)
        if (hit[j][k]) pu = u[j][k];
      if (STATS) {
        int used = 0;
        for (int k = 0; k < adv[j] && k < rem[j]; ++k) {
          ++used;
          if (hit[j][k]) break;
        }
        acc.scanned += used;
      }
      if (pu >= 0) {
        const int32_t vv = v[j];
        a.parent[vv] = pu;
        a.depth[vv] = a.d + 1;
        atomicOr((unsigned long long *)&found[(vv >> 6) - wlo], 1ull << (vv & 63));
        // the next frontier's edges are out-edges: on a directed graph the
        // in-degree held here is not the count the top-down side needs
        const int64_t dv = a.g.directed ? a.g.row_ptr[vv + 1] - a.g.row_ptr[vv] : (int64_t)deg[j];
        acc.mf += (unsigned long long)dv;
        acc.nv += 1;
        v[j] = -1;
      } else {
        e[j] += adv[j];
        rem[j] -= adv[j];
        if (rem[j] <= 0) v[j] = -1;
      }
    }
  }
  __syncthreads();
  for (int64_t i = threadIdx.x; i < nw; i += BLOCK) {
    const uint64_t b = found[i];
    a.nbm[wlo + i] = b;
    if (b) a.vbm[wlo + i] |= b;
  }
}

// Bottom-up -> top-down: F_d, held as a bitmap by the bottom-up steps
// (which do not build queues), becomes the vertex queue and hub chunk
// items of buffer set bs_out, as a top-down step would have appended them.
// A wave loads 64 bitmap words at once and hands their set bits to its
// lanes in order (prefix sums of the word popcounts), so a sparse frontier
// costs a few round trips per wave even on the small group.  Whole
// workgroups; the staged entries reach the segments in step_end, and a
// barrier that publishes bs_out must follow.
template <int BLOCK>
__device__ __forceinline__ void queue_from_bitmap(const StepArgs &a, Stage<BLOCK> &st, const uint64_t *fbm,
                                  int64_t gwave, int64_t nwaves) {
  if (threadIdx.x == 0) {
    st.qn = 0;
    st.cn = 0;
    st.hn = 0;
  }
  __syncthreads();
  LaneAcc acc;
  const int lane = lane_id();
  const int64_t nwords = (a.g.n + kWave - 1) / kWave;
  for (int64_t w0 = gwave * kWave; w0 < nwords; w0 += nwaves * kWave) {
    const uint64_t bits = w0 + lane < nwords ? fbm[w0 + lane] : 0ull;
    uint32_t total;
    const uint32_t off = wave_excl_scan_u32((uint32_t)__popcll(bits), total);
    for (uint32_t i0 = 0; i0 < total; i0 += kWave) {
      const uint32_t i = i0 + (uint32_t)lane;
      int j = 0;  // the word holding set bit i: largest j with off_j <= i
#pragma unroll
      for (int step = 32; step >= 1; step >>= 1) {
        const uint32_t oc = __shfl(off, j + step, kWave);
        if (oc <= i) j += step;
      }
      const uint64_t bj = __shfl(bits, j, kWave);
      const uint32_t oj = __shfl(off, j, kWave);
      const bool in = i < total;
      int64_t v = 0, degv = 0;
      if (in) {
        v = (w0 + j) * kWave + nth_set_bit(bj, i - oj);
        degv = a.g.row_ptr[v + 1] - a.g.row_ptr[v];
      }
      stage_append<BLOCK>(a, st, in, (int32_t)v, degv, acc);
    }
  }
  (void)step_end<BLOCK>(a, st, acc);
}

// Top-down -> bottom-up: build the frontier bitmap (depth == d) and the
// visited bitmap (parent >= 0; vertices that no edge enters and padding
// count as visited so whole words can be skipped).  Undirected, "no edge
// enters" is degree 0, which the parent encoding already holds; directed,
// it is in-degree 0, read from the in-lists.  COUNT: also count F_d into
// acc (vertices, and their out-degrees read from the row offsets) -- after
// a level of plain-store claims, the frontier's only exact count.
template <bool COUNT = false>
__device__ inline void convert_to_bitmaps(const DevGraph &g, const int32_t *parent,
                                          const int32_t *depth, int32_t d, uint64_t *fbm,
                                          uint64_t *vbm, int64_t gwave, int64_t nwaves,
                                          LaneAcc *acc = nullptr) {
  const int lane = lane_id();
  const int64_t nwords = (g.n + kWave - 1) / kWave;
  // kConvU words per pass: all their loads are issued before the first
  // ballot waits, so a wave keeps 2 * kConvU loads in flight (4 * kConvU
  // when COUNT: the row offsets that give a frontier vertex's degree are
  // loaded for every lane, not behind a per-lane test)
  constexpr int kConvU = 4;
  const int32_t spare = (int32_t)(((uint64_t)gwave * 1024ull) % (uint64_t)g.n);
  for (int64_t w0 = gwave; w0 < nwords; w0 += kConvU * nwaves) {
    int32_t p[kConvU], dv[kConvU];
    int64_t r0[kConvU], r1[kConvU];
#pragma unroll
    for (int u = 0; u < kConvU; ++u) {
      const int64_t v = (w0 + u * nwaves) * kWave + lane;
      const bool in = w0 + u * nwaves < nwords && v < g.n;
      const int64_t vl = in ? v : (int64_t)spare;
      const int32_t pr = parent[vl], dr = depth[vl];
      if (COUNT) {
        r0[u] = g.row_ptr[vl];
        r1[u] = g.row_ptr[vl + 1];
      }
      p[u] = in ? pr : 0;
      dv[u] = in ? dr : -1;
    }
#pragma unroll
    for (int u = 0; u < kConvU; ++u) {
      const int64_t w = w0 + u * nwaves;
      if (w >= nwords) break;  // wave-uniform
      const int64_t v = w * kWave + lane;
      bool visited = true;
      if (v < g.n) {
        if (g.directed)
          visited = (p[u] >= 0) || (g.row_ptr_in[v + 1] == g.row_ptr_in[v]);
        else
          visited = (p[u] >= 0) || (p[u] == kIsolated);
      }
      const bool front = v < g.n && dv[u] == d;
      const uint64_t bv = __ballot(visited);
      const uint64_t bf = __ballot(front);
      if (lane == 0) {
        vbm[w] = bv;
        fbm[w] = bf;
      }
      if (COUNT && front) {
        acc->nv += 1;
        acc->mf += (unsigned long long)(r1[u] - r0[u]);
      }
    }
  }
}

// Per-search initialisation (timed, Section 2.3): parent <- -degree
// (Section 3, BFS), depth <- -1, then the source.
// Groups of four vertices go with 16-byte stores when both outputs are
// 16-byte aligned, kInitU groups per thread per pass with every row-offset
// load issued before the first store (the compiler cannot move a load of
// row_ptr above a store to parent or depth by itself); the rest one by one.
__device__ inline int32_t initial_parent(int64_t deg) {
  return deg ? (int32_t)(-deg) : kIsolated;
}

__device__ inline void init_vertices(const DevGraph &g, int32_t *parent, int32_t *depth,
                                     int32_t source, int64_t tid, int64_t nthreads) {
  constexpr int kInitU = 4;
  const bool vec = ((reinterpret_cast<uintptr_t>(parent) | reinterpret_cast<uintptr_t>(depth) |
                     reinterpret_cast<uintptr_t>(g.row_ptr)) & 15u) == 0;
  const int64_t n4 = vec ? g.n / 4 : 0;
  for (int64_t q0 = tid; q0 < n4; q0 += kInitU * nthreads) {
    int64_t r[kInitU][5];
#pragma unroll
    for (int u = 0; u < kInitU; ++u) {
      const int64_t q = q0 + u * nthreads < n4 ? q0 + u * nthreads : q0;  // no branch around the loads
      const longlong2 a = *reinterpret_cast<const longlong2 *>(g.row_ptr + 4 * q);
      const longlong2 b = *reinterpret_cast<const longlong2 *>(g.row_ptr + 4 * q + 2);
      r[u][0] = a.x;
      r[u][1] = a.y;
      r[u][2] = b.x;
      r[u][3] = b.y;
      r[u][4] = g.row_ptr[4 * q + 4];
    }
#pragma unroll
    for (int u = 0; u < kInitU; ++u) {
      const int64_t q = q0 + u * nthreads;
      if (q >= n4) break;
      int4 p = make_int4(initial_parent(r[u][1] - r[u][0]), initial_parent(r[u][2] - r[u][1]),
                         initial_parent(r[u][3] - r[u][2]), initial_parent(r[u][4] - r[u][3]));
      int4 dd = make_int4(-1, -1, -1, -1);
      const int64_t k = (int64_t)source - 4 * q;
      if (k == 0) { p.x = source; dd.x = 0; }
      if (k == 1) { p.y = source; dd.y = 0; }
      if (k == 2) { p.z = source; dd.z = 0; }
      if (k == 3) { p.w = source; dd.w = 0; }
      reinterpret_cast<int4 *>(parent)[q] = p;
      reinterpret_cast<int4 *>(depth)[q] = dd;
    }
  }
  for (int64_t v = 4 * n4 + tid; v < g.n; v += nthreads) {
    int32_t p = initial_parent(g.row_ptr[v + 1] - g.row_ptr[v]);
    int32_t dd = -1;
    if (v == source) {
      p = source;
      dd = 0;
    }
    parent[v] = p;
    depth[v] = dd;
  }
}

// init_vertices over the vertices [lo, hi) of one workgroup (all its
// threads; lo a multiple of 4 for the 16-byte stores).
template <int BLOCK>
__device__ inline void init_vertices_range(const DevGraph &g, int32_t *parent, int32_t *depth,
                                           int32_t source, int64_t lo, int64_t hi) {
  constexpr int kInitU = 4;
  const bool vec = ((reinterpret_cast<uintptr_t>(parent) | reinterpret_cast<uintptr_t>(depth) |
                     reinterpret_cast<uintptr_t>(g.row_ptr)) & 15u) == 0 && (lo & 3) == 0;
  const int64_t q_lo = vec ? lo / 4 : 0, q_hi = vec ? hi / 4 : 0;
  for (int64_t q0 = q_lo + threadIdx.x; q0 < q_hi; q0 += kInitU * BLOCK) {
    int64_t r[kInitU][5];
#pragma unroll
    for (int u = 0; u < kInitU; ++u) {
      const int64_t q = q0 + u * BLOCK < q_hi ? q0 + u * BLOCK : q0;  // no branch around the loads
      const longlong2 x = *reinterpret_cast<const longlong2 *>(g.row_ptr + 4 * q);
      const longlong2 y = *reinterpret_cast<const longlong2 *>(g.row_ptr + 4 * q + 2);
      r[u][0] = x.x;
      r[u][1] = x.y;
      r[u][2] = y.x;
      r[u][3] = y.y;
      r[u][4] = g.row_ptr[4 * q + 4];
    }
#pragma unroll
    for (int u = 0; u < kInitU; ++u) {
      const int64_t q = q0 + u * BLOCK;
      if (q >= q_hi) break;
      int4 p = make_int4(initial_parent(r[u][1] - r[u][0]), initial_parent(r[u][2] - r[u][1]),
                         initial_parent(r[u][3] - r[u][2]), initial_parent(r[u][4] - r[u][3]));
      int4 dd = make_int4(-1, -1, -1, -1);
      const int64_t k = (int64_t)source - 4 * q;
      if (k == 0) { p.x = source; dd.x = 0; }
      if (k == 1) { p.y = source; dd.y = 0; }
      if (k == 2) { p.z = source; dd.z = 0; }
      if (k == 3) { p.w = source; dd.w = 0; }
      reinterpret_cast<int4 *>(parent)[q] = p;
      reinterpret_cast<int4 *>(depth)[q] = dd;
    }
  }
  for (int64_t v = (vec ? 4 * q_hi : lo) + threadIdx.x; v < hi; v += BLOCK) {
    int32_t p = initial_parent(g.row_ptr[v + 1] - g.row_ptr[v]);
    int32_t dd = -1;
    if (v == source) {
      p = source;
      dd = 0;
    }
    parent[v] = p;
    depth[v] = dd;
  }
}

// F_0 = {source} in buffer set 0, segment 0 (one thread).  Returns the
// totals of F_0 to feed the first level boundary.
__device__ inline Totals init_source(const DevGraph &g, const Queues &Q, Ctl *ctl, int32_t source,
                                     int32_t hub, int32_t chunk) {
  const int64_t deg = g.row_ptr[source + 1] - g.row_ptr[source];
  if (deg > hub) {
    const int64_t nch = (deg + chunk - 1) / chunk;
    for (int64_t k = 0; k < nch; ++k) Q.c0[k] = make_int2(source, (int)k);
    st_agent(&ctl->seg[0][0].c, (unsigned long long)nch);
  } else {
    Q.q0[0] = source;
    st_agent(&ctl->seg[0][0].q, 1ull);
  }
  Totals t = {};
  t.nv = 1;
  t.mf = (unsigned long long)deg;
  return t;
}

// Final pass (Section 3, BFS): every negative parent becomes -1.
// Groups of four with 16-byte accesses when `parent` is 16-byte aligned,
// kFixU loads in flight per thread before the first store.
__device__ inline void fixup_parents(int64_t n, int32_t *parent, int64_t tid, int64_t nthreads) {
  constexpr int kFixU = 4;
  const int64_t n4 = (reinterpret_cast<uintptr_t>(parent) & 15u) == 0 ? n / 4 : 0;
  int4 *p4 = reinterpret_cast<int4 *>(parent);
  for (int64_t q0 = tid; q0 < n4; q0 += kFixU * nthreads) {
    int4 x[kFixU];
#pragma unroll
    for (int u = 0; u < kFixU; ++u) x[u] = p4[q0 + u * nthreads < n4 ? q0 + u * nthreads : q0];
#pragma unroll
    for (int u = 0; u < kFixU; ++u) {
      const int64_t q = q0 + u * nthreads;
      if (q >= n4) break;
      if (x[u].x < -1 || x[u].y < -1 || x[u].z < -1 || x[u].w < -1)
        p4[q] = make_int4(x[u].x < -1 ? -1 : x[u].x, x[u].y < -1 ? -1 : x[u].y,
                          x[u].z < -1 ? -1 : x[u].z, x[u].w < -1 ? -1 : x[u].w);
    }
  }
  for (int64_t v = 4 * n4 + tid; v < n; v += nthreads) {
    const int32_t p = parent[v];
    if (p < -1) parent[v] = -1;
  }
}

}  // namespace gap
