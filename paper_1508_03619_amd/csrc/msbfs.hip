// Multi-source breadth-first search: many searches in one cooperative launch.
//
// Every (graph, source) pair of a batch is a lane.  Lanes of one graph form a
// segment; a segment keeps W 64-bit words per vertex for each of three
// bitsets: visited V (all depths so far), frontier F (depth d) and next N
// (depth d+1).  One pass over an adjacency list then serves up to 64*W
// searches: the bits of a word are the lanes.  Segments of different graphs
// are laid end to end in one virtual vertex space (each starts on a multiple
// of 64), so graphs of uneven size share one launch.
//
// Every lane's result is exactly the single-source result for its (graph,
// source): depth is the hop distance (unique) and the parent is a neighbour
// one level closer (Section 2.1).  Per level:
//   advance  (dense)  V |= F; queue the vertices with F != 0 (hubs as chunk
//                     items), queue hubs some active lane still needs as
//                     bottom-up chunk items; per-segment totals (|F|, edges
//                     of F, edges still to explore, lanes still active);
//                     clear N
//   step     top-down over the queue (F[u] & ~V[v] claimed with atomicOr on
//                     N[v]; the bits a thread turns on are its own), or
//            bottom-up over vertices still needed by an active lane (scan
//                     adjacency, gather F[u], stop when every needed lane is
//                     found); hubs are scanned chunk by chunk by whole waves
// The direction is chosen per segment with the same edge/vertex rule as the
// single-source search.
//
// Parents and depths found during the search go to vertex-major rows (the
// 64*W lanes of a vertex side by side, so the writes of one vertex share a
// few cache lines); a final kernel transposes the rows into the per-lane
// output arrays through LDS, writing every output line once and in full,
// and writes -1 for pairs that were never reached.
#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <vector>

#include "bfs_kernels.h"
#include "runtime.h"

namespace gap {

constexpr int kMaxSeg = 64;
constexpr int kMsBlock = 1024;
constexpr int kBuFlag = 1 << 30;  // chunk item is a bottom-up hub chunk
constexpr int kMsTraceLevels = 128;

struct MsSeg {
  const int64_t *row_ptr;
  const int32_t *col;
  const int4 *head;   // first four entries of every list (-1 past the end)
  int64_t n;          // vertices of the graph
  int64_t vbase;      // first virtual vertex (multiple of 64)
  int32_t lane_base;  // first lane (index into the output tables)
  int32_t lanes;      // lanes of this segment, 1..64*W
};

// Totals of one segment for one level (device atomics).
struct alignas(128) MsSegTotals {
  unsigned long long nf;    // vertices with a frontier bit
  unsigned long long mf;    // sum of their degrees
  unsigned long long mu;    // sum of degrees of vertices some lane has not reached
  unsigned long long lanes_or[4];  // OR of F over the segment
};

struct MsCtl {
  Ctl base;                        // grid barrier, queue segment counters
  MsSegTotals tot[2][kMaxSeg];     // level parity x segment
  // per level: real-time stamps (advance start, step start, step end),
  // direction of segment 0, frontier vertices and frontier edges (segment
  // 0; with statistics, every segment)
  unsigned long long trace[kMsTraceLevels][6];
  // with statistics, per level: vertices a bottom-up step searched for (some
  // lane needed them) and the adjacency entries it read
  unsigned long long lvstat[kMsTraceLevels][2];
};

struct MsArgs {
  const MsSeg *segs;
  int nseg;
  int64_t nvirt;            // virtual vertices (multiple of 64)
  uint64_t *V, *B0, *B1;    // W words per virtual vertex
  int32_t *P, *D;           // vertex-major rows: 64*W parents / depths per vertex
  int32_t *const *parents;  // per lane, int32[n of its graph]
  int32_t *const *depths;   // per lane, may hold NULL entries
  const int32_t *sources;   // per lane, local vertex ID
  int32_t nlanes;
  Queues Q;                 // virtual vertex IDs
  MsCtl *ctl;
  int *sticky;              // the stream's sticky status word
  Params p;
};

template <int W>
struct MsShared {
  int64_t vbase[kMaxSeg + 1];
  int64_t n[kMaxSeg];
  const int64_t *row_ptr[kMaxSeg];
  const int32_t *col[kMaxSeg];
  const int4 *head[kMaxSeg];
  int32_t lane_base[kMaxSeg];
  int32_t lanes[kMaxSeg];
  int32_t dir[kMaxSeg];
  int64_t nf_prev[kMaxSeg];
  uint64_t active[kMaxSeg][W];  // lanes whose frontier is not empty
  int32_t nlive;                // segments still searching
  // advance-pass accumulation (LDS atomics), flushed once per workgroup
  unsigned long long acc_nf[kMaxSeg], acc_mf[kMaxSeg], acc_mu[kMaxSeg];
  unsigned long long acc_or[kMaxSeg][W];
  Stage<kMsBlock> st;
};

__device__ inline int ms_seg_find(const int64_t *vbase, int nseg, int64_t vv) {
  int lo = 0, hi = nseg - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (vbase[mid] <= vv)
      lo = mid;
    else
      hi = mid - 1;
  }
  return lo;
}

__device__ inline uint64_t lane_mask_word(int lanes, int w) {
  const int lo = w * 64;
  if (lanes <= lo) return 0ull;
  if (lanes >= lo + 64) return ~0ull;
  return (1ull << (lanes - lo)) - 1ull;
}

// Parent/depth scratch is laid out like the outputs: for each 64-vertex word
// of the virtual space and each of its 64*W lanes, 64 consecutive int32 (one
// per vertex of the word).  Index of (virtual vertex vv, lane bit i of word w):
template <int W>
__device__ inline int64_t tile_index(int64_t vv, int w, int i) {
  return (((vv >> 6) * (64 * W) + w * 64 + i) << 6) + (vv & 63);
}

// Records parent/depth of every lane in `bits` (word w) at virtual vertex vv
// (scattered: used by top-down claims and hub chunks).
template <int W>
__device__ inline void ms_record(const MsArgs &a, int64_t vv, int w, uint64_t bits,
                                 int32_t parent, int32_t dep) {
  while (bits) {
    const int i = __builtin_ctzll(bits);
    bits &= bits - 1ull;
    const int64_t t = tile_index<W>(vv, w, i);
    a.P[t] = parent;
    a.D[t] = dep;
  }
}

__device__ inline uint64_t wave_or_u64(uint64_t x) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) x |= __shfl_xor(x, o, kWave);
  return x;
}

// OR of the lanes below this one.
__device__ inline uint64_t wave_excl_or_u64(uint64_t x) {
  const int lane = lane_id();
  uint64_t incl = x;
#pragma unroll
  for (int o = 1; o < kWave; o <<= 1) {
    const uint64_t y = __shfl_up(incl, o, kWave);
    if (lane >= o) incl |= y;
  }
  const uint64_t prev = __shfl_up(incl, 1, kWave);
  return lane == 0 ? 0ull : prev;
}

// ---- the persistent kernel ---------------------------------------------------------

template <int W, bool STATS>
__device__ __forceinline__ void msbfs(const MsArgs &a) {
  __shared__ MsShared<W> sh;
  const int64_t nthreads = (int64_t)gridDim.x * kMsBlock;
  const int64_t tid = (int64_t)blockIdx.x * kMsBlock + threadIdx.x;
  const int64_t nwaves = nthreads / kWave;
  const int64_t gwave = tid / kWave;
  const int lane = lane_id();
  const unsigned int nblocks = gridDim.x;
  const int nseg = a.nseg;
  const int hub = a.p.hub, chunk = a.p.chunk;
  Ctl *ctl = &a.ctl->base;

  for (int s = threadIdx.x; s < nseg; s += kMsBlock) {
    sh.vbase[s] = a.segs[s].vbase;
    sh.n[s] = a.segs[s].n;
    sh.row_ptr[s] = a.segs[s].row_ptr;
    sh.col[s] = a.segs[s].col;
    sh.head[s] = a.segs[s].head;
    sh.lane_base[s] = a.segs[s].lane_base;
    sh.lanes[s] = a.segs[s].lanes;
    sh.dir[s] = kTopDown;
    sh.nf_prev[s] = 0;
  }
  if (threadIdx.x == 0) sh.vbase[nseg] = a.nvirt;
  __syncthreads();

  // ---- init: clear the bitsets, then place the sources -------------------------
  uint64_t *F = a.B0, *N = a.B1;
  for (int64_t i = tid; i < a.nvirt * W; i += nthreads) {
    a.V[i] = 0ull;
    F[i] = 0ull;
  }
  if (!grid_sync(ctl, nblocks, Totals{}, -1, 0, a.p.wait)) return;
  for (int64_t l = tid; l < a.nlanes; l += nthreads) {
    int s = 0;  // lane -> segment (few segments: linear)
    while (s + 1 < nseg && sh.lane_base[s + 1] <= l) ++s;
    const int li = (int)(l - sh.lane_base[s]);
    const int32_t src = a.sources[l];
    const int64_t vv = sh.vbase[s] + src;
    atomicOr((unsigned long long *)&F[vv * W + li / 64], 1ull << (li % 64));
    a.P[tile_index<W>(vv, li / 64, li % 64)] = src;
    a.D[tile_index<W>(vv, li / 64, li % 64)] = 0;
  }
  if (!grid_sync(ctl, nblocks, Totals{}, -1, 0, a.p.wait)) return;

  const int64_t nwords = a.nvirt / kWave;
  const bool tracer = blockIdx.x == 0 && threadIdx.x == 0;
  for (int32_t d = 0;; ++d) {
    if (tracer && d < kMsTraceLevels) a.ctl->trace[d][0] = rt_clock();
    // ---- advance ----------------------------------------------------------------
    for (int s = threadIdx.x; s < nseg; s += kMsBlock) {
      sh.acc_nf[s] = sh.acc_mf[s] = sh.acc_mu[s] = 0;
      for (int w = 0; w < W; ++w) sh.acc_or[s][w] = 0;
    }
    if (threadIdx.x == 0) {
      sh.st.qn = 0;
      sh.st.cn = 0;
    }
    __syncthreads();
    StepArgs sa{};  // staging target: queue buffer set (d+1)&1
    sa.Q = a.Q;
    sa.bs_in = d & 1;
    sa.ctl = ctl;
    sa.hub = hub;
    sa.chunk = chunk;
    LaneAcc none;
    for (int64_t wd = gwave; wd < nwords; wd += nwaves) {
      const int64_t vv = wd * kWave + lane;
      const int s = ms_seg_find(sh.vbase, nseg, wd * kWave);  // one segment per wave
      const int64_t vl = vv - sh.vbase[s];
      const bool real = vl < sh.n[s];
      uint64_t f[W];
      bool any = false, incomplete = false;
#pragma unroll
      for (int w = 0; w < W; ++w) {
        f[w] = F[vv * W + w];
        any |= f[w] != 0ull;
      }
      int64_t deg = 0;
      if (real) deg = sh.row_ptr[s][vl + 1] - sh.row_ptr[s][vl];
#pragma unroll
      for (int w = 0; w < W; ++w) {
        uint64_t vis = a.V[vv * W + w];
        if (f[w]) {
          vis |= f[w];
          a.V[vv * W + w] = vis;
        }
        N[vv * W + w] = 0ull;
        incomplete |= (lane_mask_word(sh.lanes[s], w) & ~vis) != 0ull;
      }
      incomplete = incomplete && real && deg > 0;
      const unsigned long long c_nf = wave_sum_u64(any ? 1ull : 0ull);
      const unsigned long long c_mf = wave_sum_u64(any ? (unsigned long long)deg : 0ull);
      const unsigned long long c_mu = wave_sum_u64(incomplete ? (unsigned long long)deg : 0ull);
      if (lane == 0) {
        if (c_nf) atomicAdd(&sh.acc_nf[s], c_nf);
        if (c_mf) atomicAdd(&sh.acc_mf[s], c_mf);
        if (c_mu) atomicAdd(&sh.acc_mu[s], c_mu);
      }
#pragma unroll
      for (int w = 0; w < W; ++w) {
        const uint64_t o = wave_or_u64(f[w]);
        if (lane == 0 && o) atomicOr(&sh.acc_or[s][w], o);
      }
      const bool big = deg > hub;
      stage_vertices<kMsBlock>(sa, sh.st, any && !big, (int32_t)vv);
      stage_chunks<kMsBlock>(sa, sh.st, any && big, (int32_t)vv, deg, 0);
      stage_chunks<kMsBlock>(sa, sh.st, incomplete && big, (int32_t)vv, deg, kBuFlag);
    }
    (void)step_end<kMsBlock, false>(sa, sh.st, none);
    __syncthreads();
    for (int s = threadIdx.x; s < nseg; s += kMsBlock) {
      MsSegTotals &T = a.ctl->tot[d & 1][s];
      if (sh.acc_nf[s]) add_agent(&T.nf, sh.acc_nf[s]);
      if (sh.acc_mf[s]) add_agent(&T.mf, sh.acc_mf[s]);
      if (sh.acc_mu[s]) add_agent(&T.mu, sh.acc_mu[s]);
      for (int w = 0; w < W; ++w)
        if (sh.acc_or[s][w]) atomicOr(&T.lanes_or[w], sh.acc_or[s][w]);
    }
    if (!grid_sync(ctl, nblocks, Totals{}, (d + 1) & 1, (d + 1) & 1, a.p.wait)) return;

    // ---- decide per segment -----------------------------------------------------
    if (threadIdx.x == 0) sh.nlive = 0;
    __syncthreads();
    for (int s = threadIdx.x; s < nseg; s += kMsBlock) {
      MsSegTotals &T = a.ctl->tot[d & 1][s];
      const int64_t nf = (int64_t)ld_agent(&T.nf);
      const int64_t mf = (int64_t)ld_agent(&T.mf);
      const int64_t mu = (int64_t)ld_agent(&T.mu);
      for (int w = 0; w < W; ++w) sh.active[s][w] = ld_agent(&T.lanes_or[w]);
      if (nf > 0) {
        atomicAdd(&sh.nlive, 1);
        sh.dir[s] = decide_direction(sh.dir[s], nf, mf, mu, sh.nf_prev[s], sh.n[s], a.p, d);
      }
      sh.nf_prev[s] = nf;
    }
    __syncthreads();
    if (sh.nlive == 0) break;
    if (d > a.nvirt) {  // more levels than vertices: inconsistent totals
      if (tid == 0) atomicExch(&ctl->err, (int)GAP_EINTERNAL);
      return;
    }
    // the other parity's totals are free now: clear them for the next advance
    if (blockIdx.x == 0) {
      for (int s = threadIdx.x; s < nseg; s += kMsBlock) {
        MsSegTotals &T = a.ctl->tot[(d + 1) & 1][s];
        st_agent(&T.nf, 0ull);
        st_agent(&T.mf, 0ull);
        st_agent(&T.mu, 0ull);
        for (int w = 0; w < 4; ++w) st_agent(&T.lanes_or[w], 0ull);
      }
    }
    if (tracer && d < kMsTraceLevels) {
      a.ctl->trace[d][1] = rt_clock();
      a.ctl->trace[d][3] = (unsigned long long)sh.dir[0];
      unsigned long long nf = (unsigned long long)sh.nf_prev[0];
      unsigned long long mf = ld_agent(&a.ctl->tot[d & 1][0].mf);
      if (STATS) {
        for (int s = 1; s < nseg; ++s) {
          nf += (unsigned long long)sh.nf_prev[s];
          mf += ld_agent(&a.ctl->tot[d & 1][s].mf);
        }
      }
      a.ctl->trace[d][4] = nf;
      a.ctl->trace[d][5] = mf;
    }
    unsigned long long st_u = 0, st_scan = 0;  // statistics of this thread's bottom-up work

    // ---- step -------------------------------------------------------------------
    StepArgs qa{};
    qa.Q = a.Q;
    qa.bs_in = (d + 1) & 1;  // the queue built by this level's advance
    qa.ctl = ctl;
    qa.d = d + 1;            // pub[(d+1)&1] holds its segment sizes
    step_begin<kMsBlock>(qa, sh.st);
    const int32_t nd = d + 1;

    // chunk items: top-down hub chunks and bottom-up hub chunks
    {
      const unsigned long long nc = sh.st.cpre[kGroups];
      const int2 *cin = a.Q.cs(qa.bs_in);
      for (unsigned long long ci = (unsigned long long)gwave; ci < nc;
           ci += (unsigned long long)nwaves) {
        const int h = seg_of(ci, sh.st.cpre);
        const int2 it = cin[h * a.Q.ccap + (int64_t)(ci - sh.st.cpre[h])];
        const int64_t xv = it.x;
        const bool bu_item = (it.y & kBuFlag) != 0;
        const int k = it.y & ~kBuFlag;
        const int s = ms_seg_find(sh.vbase, nseg, xv);
        if (sh.dir[s] != (bu_item ? kBottomUp : kTopDown)) continue;
        const int32_t xl = (int32_t)(xv - sh.vbase[s]);
        const int64_t rbeg = sh.row_ptr[s][xl], rend = sh.row_ptr[s][xl + 1];
        const int64_t beg = rbeg + (int64_t)k * chunk;
        const int64_t end = beg + chunk < rend ? beg + chunk : rend;
        if (!bu_item) {
          // top-down: frontier hub xv pushes to its chunk of neighbours
          uint64_t fu[W];
#pragma unroll
          for (int w = 0; w < W; ++w) fu[w] = F[xv * W + w];
          for (int64_t e = beg + lane; e < end; e += kWave) {
            const int32_t vl = sh.col[s][e];
            const int64_t vv = sh.vbase[s] + vl;
#pragma unroll
            for (int w = 0; w < W; ++w) {
              if (!fu[w]) continue;
              const uint64_t nb = fu[w] & ~a.V[vv * W + w];
              if (!nb) continue;
              const uint64_t old = atomicOr((unsigned long long *)&N[vv * W + w], nb);
              const uint64_t mine = nb & ~old;
              if (mine) ms_record<W>(a, vv, w, mine, xl, nd);
            }
          }
        } else {
          // bottom-up: unfinished hub xv pulls from its chunk of neighbours;
          // each lane bit goes to the lowest wave lane that found it, then
          // one atomicOr per word settles races with the hub's other chunks
          uint64_t need[W];
          bool left = false;
#pragma unroll
          for (int w = 0; w < W; ++w) {
            need[w] = sh.active[s][w] & ~a.V[xv * W + w] &
                      ~ld_agent((const unsigned long long *)&N[xv * W + w]);
            left |= need[w] != 0ull;
          }
          if (STATS && lane == 0 && k == 0 && left) st_u += 1;
          for (int64_t e0 = beg; e0 < end && left; e0 += kWave) {
            const int64_t e = e0 + lane;
            const int32_t ul = e < end ? sh.col[s][e] : -1;
            if (STATS && ul >= 0) st_scan += 1;
            left = false;
#pragma unroll
            for (int w = 0; w < W; ++w) {
              const uint64_t hit = (ul >= 0 && need[w]) ? F[(sh.vbase[s] + ul) * W + w] & need[w]
                                                        : 0ull;
              const uint64_t uni = wave_or_u64(hit);
              if (uni) {
                const uint64_t own = hit & ~wave_excl_or_u64(hit);
                unsigned long long old = 0;
                if (lane == 0) old = atomicOr((unsigned long long *)&N[xv * W + w], uni);
                old = __shfl(old, 0, kWave);
                const uint64_t mine = own & ~old;
                if (mine) ms_record<W>(a, xv, w, mine, ul, nd);
                need[w] &= ~uni;
              }
              left |= need[w] != 0ull;
            }
          }
        }
      }
    }
    // top-down over queued vertices of top-down segments
    {
      const unsigned long long nq = sh.st.qpre[kGroups];
      const int32_t *qin = a.Q.qs(qa.bs_in);
      unsigned long long per = (nq + (unsigned long long)nwaves - 1) / (unsigned long long)nwaves;
      per = per < 1 ? 1 : (per > 64 ? 64 : per);
      const unsigned long long ngroups = (nq + per - 1) / per;
      for (unsigned long long gi = (unsigned long long)gwave; gi < ngroups;
           gi += (unsigned long long)nwaves) {
        const unsigned long long idx = gi * per + lane;
        int64_t uv = -1;
        int s = 0;
        int64_t beg = 0;
        uint32_t deg = 0;
        if ((unsigned long long)lane < per && idx < nq) {
          const int h = seg_of(idx, sh.st.qpre);
          uv = qin[h * a.Q.n + (int64_t)(idx - sh.st.qpre[h])];
          s = ms_seg_find(sh.vbase, nseg, uv);
          if (sh.dir[s] == kTopDown) {
            const int64_t ul = uv - sh.vbase[s];
            beg = sh.row_ptr[s][ul];
            deg = (uint32_t)(sh.row_ptr[s][ul + 1] - beg);
          }
        }
        uint32_t total;
        const uint32_t off = wave_excl_scan_u32(deg, total);
        for (uint32_t b = 0; b < total; b += kWave) {
          const uint32_t e = b + (uint32_t)lane;
          int j = 0;
#pragma unroll
          for (int step = 32; step >= 1; step >>= 1) {
            const uint32_t oc = __shfl(off, j + step, kWave);
            if (oc <= e) j += step;
          }
          const int64_t uj = __shfl(uv, j, kWave);
          const int sj = __shfl(s, j, kWave);
          const int64_t bj = __shfl(beg, j, kWave);
          const uint32_t oj = __shfl(off, j, kWave);
          if (e < total) {
            const int32_t vl = sh.col[sj][bj + (int64_t)(e - oj)];
            const int64_t vv = sh.vbase[sj] + vl;
            const int32_t ul = (int32_t)(uj - sh.vbase[sj]);
#pragma unroll
            for (int w = 0; w < W; ++w) {
              const uint64_t fu = F[uj * W + w];
              if (!fu) continue;
              const uint64_t nb = fu & ~a.V[vv * W + w];
              if (!nb) continue;
              const uint64_t old = atomicOr((unsigned long long *)&N[vv * W + w], nb);
              const uint64_t mine = nb & ~old;
              if (mine) ms_record<W>(a, vv, w, mine, ul, nd);
            }
          }
        }
      }
    }
    // bottom-up over the non-hub vertices of bottom-up segments
    for (int64_t wd = gwave; wd < nwords; wd += nwaves) {
      const int s = ms_seg_find(sh.vbase, nseg, wd * kWave);
      if (sh.dir[s] != kBottomUp) continue;
      const int64_t vv = wd * kWave + lane;
      const int64_t vl = vv - sh.vbase[s];
      uint64_t need[W], vis[W], got[W];
      bool want = false;
      int64_t beg = 0, end = 0;
      if (vl < sh.n[s]) {
        beg = sh.row_ptr[s][vl];
        end = sh.row_ptr[s][vl + 1];
      }
      const bool small = end - beg <= hub;
#pragma unroll
      for (int w = 0; w < W; ++w) {
        vis[w] = a.V[vv * W + w];
        need[w] = (small && vl < sh.n[s]) ? (sh.active[s][w] & ~vis[w]) : 0ull;
        got[w] = 0ull;
        want |= need[w] != 0ull;
      }
      // rounds are wave-uniform (the coalesced writes below use every lane);
      // a lane whose vertex is settled or exhausted just contributes nothing
      bool act = want;
      int64_t e = beg;
      if (STATS && want && end > beg) st_u += 1;
      bool first = true;  // the first four entries come from the head record
      while (__ballot(act) != 0ull) {
        if (STATS && act) st_scan += (unsigned long long)(end - e < 4 ? end - e : 4);
        int32_t ul[4];
        if (first) {
          int4 h = make_int4(-1, -1, -1, -1);
          if (act) h = sh.head[s][vl];
          ul[0] = h.x;
          ul[1] = h.y;
          ul[2] = h.z;
          ul[3] = h.w;
          first = false;
        } else {
#pragma unroll
          for (int k = 0; k < 4; ++k) ul[k] = (act && e + k < end) ? sh.col[s][e + k] : -1;
        }
        uint64_t fu[4][W];
#pragma unroll
        for (int k = 0; k < 4; ++k)
#pragma unroll
          for (int w = 0; w < W; ++w)
            fu[k][w] = (ul[k] >= 0 && need[w]) ? F[(sh.vbase[s] + ul[k]) * W + w] : 0ull;
        bool left = false;
#pragma unroll
        for (int w = 0; w < W; ++w) {
          uint64_t hit[4];
#pragma unroll
          for (int k = 0; k < 4; ++k) {  // first neighbour in list order wins a bit
            hit[k] = fu[k][w] & need[w];
            need[w] &= ~hit[k];
          }
          const uint64_t round = hit[0] | hit[1] | hit[2] | hit[3];
          got[w] |= round;
          // every lane bit found by some vertex of the wave: the 64 vertices
          // write that lane's slots of the word with one coalesced store
          uint64_t uni = wave_or_u64(round);
          while (uni) {
            const int i = __builtin_ctzll(uni);
            uni &= uni - 1ull;
            if ((round >> i) & 1ull) {
              const int32_t par = ((hit[0] >> i) & 1ull)   ? ul[0]
                                  : ((hit[1] >> i) & 1ull) ? ul[1]
                                  : ((hit[2] >> i) & 1ull) ? ul[2]
                                                           : ul[3];
              const int64_t t = tile_index<W>(vv, w, i);
              a.P[t] = par;
              a.D[t] = nd;
            }
          }
          left |= need[w] != 0ull;
        }
        e += 4;
        act = act && left && e < end;
      }
#pragma unroll
      for (int w = 0; w < W; ++w) {
        if (got[w]) {
          a.V[vv * W + w] = vis[w] | got[w];
          N[vv * W + w] = got[w];
        }
      }
    }
    if (STATS && d < kMsTraceLevels) {
      const unsigned long long wu = wave_sum_u64(st_u), ws = wave_sum_u64(st_scan);
      if (lane == 0 && (wu | ws)) {
        add_agent(&a.ctl->lvstat[d][0], wu);
        add_agent(&a.ctl->lvstat[d][1], ws);
      }
    }
    if (!grid_sync(ctl, nblocks, Totals{}, -1, 0, a.p.wait)) return;
    if (tracer && d < kMsTraceLevels) a.ctl->trace[d][2] = rt_clock();
    swap_ptr(F, N);
  }
}

template <int W, bool STATS>
__global__ __launch_bounds__(kMsBlock) void k_msbfs(MsArgs a) {
  msbfs<W, STATS>(a);
  note_error(a.sticky, &a.ctl->base);
}

// ---- output: scratch tiles -> per-lane arrays ------------------------------------------
// A wave takes one 64-vertex word and copies each lane's 64 slots to that
// lane's output (coalesced 256-byte reads and writes), writing -1 where the
// lane never reached the vertex.  When the search kernel recorded an error
// (a timed-out wait, an inconsistent state), every output entry becomes
// INT32_MIN instead, so a failed batch can never pass for one whose lanes
// reached nothing.

constexpr int kOutBlock = 256;

template <int W>
__global__ __launch_bounds__(kOutBlock) void k_ms_output(MsArgs a, int64_t nword_tiles,
                                                         const int64_t *tile_base) {
  __shared__ int64_t s_base[kMaxSeg + 1];
  const int nseg = a.nseg;
  for (int s = threadIdx.x; s <= nseg; s += kOutBlock) s_base[s] = tile_base[s];
  __syncthreads();
  const bool failed = __hip_atomic_load(&a.ctl->base.err, __ATOMIC_RELAXED,
                                        __HIP_MEMORY_SCOPE_AGENT) != 0;
  const int lane = lane_id();
  const int64_t nwaves = (int64_t)gridDim.x * kOutBlock / kWave;
  const int64_t gwave = ((int64_t)blockIdx.x * kOutBlock + threadIdx.x) / kWave;
  for (int64_t ti = gwave; ti < nword_tiles; ti += nwaves) {
    const int s = ms_seg_find(s_base, nseg, ti);
    const MsSeg sg = a.segs[s];
    const int64_t vl0 = (ti - s_base[s]) * kWave;
    const int64_t vv0 = sg.vbase + vl0;
    const bool real = vl0 + lane < sg.n;
    for (int w = 0; w * 64 < sg.lanes; ++w) {
      const uint64_t vis = real ? a.V[(vv0 + lane) * W + w] : 0ull;
      const int nl = min(64, sg.lanes - w * 64);
      for (int i = 0; i < nl; ++i) {
        const int l = sg.lane_base + w * 64 + i;
        const int64_t t = tile_index<W>(vv0 + lane, w, i);
        const bool hit = ((vis >> i) & 1ull) != 0ull;
        if (real) a.parents[l][vl0 + lane] = failed ? INT32_MIN : (hit ? a.P[t] : -1);
        int32_t *dp = a.depths[l];
        if (dp && real) dp[vl0 + lane] = failed ? INT32_MIN : (hit ? a.D[t] : -1);
      }
    }
  }
}

// ---- host side ------------------------------------------------------------------------

template <int W>
static gap_status launch_ms(const MsArgs &a, const DeviceInfo *di, int split, int coop, bool stats, int64_t ntiles,
                            const int64_t *tile_base, hipStream_t stream) {
  auto kern = stats ? k_msbfs<W, true> : k_msbfs<W, false>;
  int per_cu = 0;
  GAP_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, kMsBlock, 0));
  if (per_cu < 1) {
    set_error("multi-source kernel does not fit on a compute unit");
    return GAP_EDEVICE;
  }
  MsArgs args = a;
  void *kargs[] = {&args};
  // 1024-thread workgroups, one per CU
  gap_status st = launch_resident((const void *)kern, di->cus, kMsBlock, 0, kargs, split, coop, di,
                                  stream, nullptr);
  if (st != GAP_OK) return st;
  int64_t blocks = (ntiles + kOutBlock / kWave - 1) / (kOutBlock / kWave);
  if (blocks > (int64_t)di->cus * 8) blocks = (int64_t)di->cus * 8;
  if (blocks < 1) blocks = 1;
  k_ms_output<W><<<(int)blocks, kOutBlock, 0, stream>>>(a, ntiles, tile_base);
  GAP_HIP(hipGetLastError());
  return GAP_OK;
}

static size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

gap_status run_bfs_batch(const gap_graph *const *graphs, int32_t num_graphs,
                         const int32_t *graph_of_source, const int32_t *sources,
                         int32_t num_sources, int32_t *const *parents, int32_t *const *depths,
                         hipStream_t stream, const gap_params &p, gap_level_stat *stats,
                         int32_t max_levels, int32_t *num_levels) {
  const int dev = graphs[0]->device;
  const bool want_stats = stats != nullptr && max_levels > 0;
  const DeviceInfo *di = nullptr;
  gap_status st = device_info(dev, &di);
  if (st != GAP_OK) return st;
  GAP_HIP(hipSetDevice(dev));

  // lanes grouped by graph; W words per vertex from the largest group
  std::vector<std::vector<int32_t>> by_graph((size_t)num_graphs);
  for (int32_t i = 0; i < num_sources; ++i) by_graph[(size_t)graph_of_source[i]].push_back(i);
  size_t maxl = 1;
  for (auto &v : by_graph) maxl = std::max(maxl, v.size());
  const int Wneed = maxl <= 64 ? 1 : (maxl <= 128 ? 2 : 4);
  const int W = std::min(Wneed, (int)p.batch_words);
  const int lanes_per_seg = 64 * W;

  std::vector<MsSeg> segs;
  std::vector<int64_t> tile_base;
  std::vector<int32_t> lane_src;              // per lane (segment order)
  std::vector<int32_t *> lane_par, lane_dep;  // per lane (segment order)
  int64_t nvirt = 0, nnz_sum = 0, ntiles = 0;
  for (int32_t g = 0; g < num_graphs; ++g) {
    const auto &ls = by_graph[(size_t)g];
    for (size_t b = 0; b < ls.size(); b += (size_t)lanes_per_seg) {
      MsSeg s;
      s.row_ptr = graphs[g]->row_ptr;
      s.col = graphs[g]->col;
      s.head = graphs[g]->head;
      s.n = graphs[g]->n;
      s.vbase = nvirt;
      s.lane_base = (int32_t)lane_src.size();
      s.lanes = (int32_t)std::min(ls.size() - b, (size_t)lanes_per_seg);
      for (int k = 0; k < s.lanes; ++k) {
        const int32_t i = ls[b + (size_t)k];
        lane_src.push_back(sources[i]);
        lane_par.push_back(parents[i]);
        lane_dep.push_back(depths ? depths[i] : nullptr);
      }
      tile_base.push_back(ntiles);
      const int64_t words = (s.n + 63) / 64;
      ntiles += words;
      nvirt += words * 64;
      nnz_sum += graphs[g]->nnz;
      segs.push_back(s);
    }
  }
  tile_base.push_back(ntiles);
  const int nseg = (int)segs.size();
  if (nseg > kMaxSeg) {
    set_error("gap_bfs_batch: %d graph segments in one batch (at most %d)", nseg, kMaxSeg);
    return GAP_EINVAL;
  }
  if (nvirt >= (int64_t)INT32_MAX) {
    set_error("gap_bfs_batch: more than 2^31 vertices in one batch");
    return GAP_EINVAL;
  }
  // chunk items per level: top-down hub chunks plus bottom-up hub chunks,
  // each bounded by nnz/chunk + nnz/hub (one partial chunk per hub)
  const int64_t chunk_cap =
      2 * (nnz_sum / p.chunk_edges + nnz_sum / p.hub_degree) + 2 + 2 * nseg;

  size_t off = 0;
  auto take = [&](size_t bytes) {
    off = align_up(off, 256);
    const size_t at = off;
    off += bytes;
    return at;
  };
  const size_t o_ctl = take(sizeof(MsCtl));
  const size_t o_seg = take(sizeof(MsSeg) * (size_t)nseg);
  const size_t o_tb = take(sizeof(int64_t) * tile_base.size());
  const size_t o_par = take(sizeof(int32_t *) * lane_src.size());
  const size_t o_dep = take(sizeof(int32_t *) * lane_src.size());
  const size_t o_src = take(sizeof(int32_t) * lane_src.size());
  const size_t meta_end = off;
  const size_t o_V = take(sizeof(uint64_t) * (size_t)nvirt * W);
  const size_t o_B0 = take(sizeof(uint64_t) * (size_t)nvirt * W);
  const size_t o_B1 = take(sizeof(uint64_t) * (size_t)nvirt * W);
  const size_t o_P = take(sizeof(int32_t) * (size_t)nvirt * 64 * W);
  const size_t o_D = take(sizeof(int32_t) * (size_t)nvirt * 64 * W);
  const size_t o_q0 = take(sizeof(int32_t) * (size_t)nvirt * kGroups);
  const size_t o_q1 = take(sizeof(int32_t) * (size_t)nvirt * kGroups);
  const size_t o_c0 = take(sizeof(int2) * (size_t)chunk_cap * kGroups);
  const size_t o_c1 = take(sizeof(int2) * (size_t)chunk_cap * kGroups);
  const size_t total = off;

  Workspace *ws = workspace_for(dev, stream);
  if (!ws) {
    set_error("workspace allocation failed");
    return GAP_ENOMEM;
  }
  st = workspace_reserve_ms(ws, total, meta_end);
  if (st != GAP_OK) return st;
  char *base = reinterpret_cast<char *>(ws->ms_buf);
  char *host = reinterpret_cast<char *>(ws->ms_host);
  // the pinned staging may still feed a previous batch's copy on this stream
  GAP_HIP(hipStreamSynchronize(stream));
  memset(host, 0, meta_end);
  memcpy(host + o_seg, segs.data(), sizeof(MsSeg) * (size_t)nseg);
  memcpy(host + o_tb, tile_base.data(), sizeof(int64_t) * tile_base.size());
  memcpy(host + o_par, lane_par.data(), sizeof(int32_t *) * lane_par.size());
  memcpy(host + o_dep, lane_dep.data(), sizeof(int32_t *) * lane_dep.size());
  memcpy(host + o_src, lane_src.data(), sizeof(int32_t) * lane_src.size());
  GAP_HIP(hipMemcpyAsync(base, host, meta_end, hipMemcpyHostToDevice, stream));

  MsArgs a{};
  a.segs = reinterpret_cast<const MsSeg *>(base + o_seg);
  a.nseg = nseg;
  a.nvirt = nvirt;
  a.V = reinterpret_cast<uint64_t *>(base + o_V);
  a.B0 = reinterpret_cast<uint64_t *>(base + o_B0);
  a.B1 = reinterpret_cast<uint64_t *>(base + o_B1);
  a.P = reinterpret_cast<int32_t *>(base + o_P);
  a.D = reinterpret_cast<int32_t *>(base + o_D);
  a.parents = reinterpret_cast<int32_t *const *>(base + o_par);
  a.depths = reinterpret_cast<int32_t *const *>(base + o_dep);
  a.sources = reinterpret_cast<const int32_t *>(base + o_src);
  a.nlanes = (int32_t)lane_src.size();
  a.Q.q0 = reinterpret_cast<int32_t *>(base + o_q0);
  a.Q.q1 = reinterpret_cast<int32_t *>(base + o_q1);
  a.Q.c0 = reinterpret_cast<int2 *>(base + o_c0);
  a.Q.c1 = reinterpret_cast<int2 *>(base + o_c1);
  a.Q.n = nvirt;
  a.Q.ccap = chunk_cap;
  a.ctl = reinterpret_cast<MsCtl *>(base + o_ctl);
  // bottom-up cannot stop early while any lane still misses a vertex, so the
  // batch has its own switching thresholds
  a.p = Params{p.batch_alpha, p.batch_beta, p.direction, p.hub_degree, p.chunk_edges, 0, 0, 0, 0, 0};
  set_wait_limits(a.p, p.wait_limit_us);
  a.sticky = ws->sticky;
  const int64_t *d_tile_base = reinterpret_cast<const int64_t *>(base + o_tb);

  CoopOrder order;
  st = coop_begin(dev, stream, p.grid_split, &order);
  if (st != GAP_OK) return st;
  switch (W) {
    case 1: st = launch_ms<1>(a, di, p.grid_split, p.coop_launch, want_stats, ntiles, d_tile_base, stream); break;
    case 2: st = launch_ms<2>(a, di, p.grid_split, p.coop_launch, want_stats, ntiles, d_tile_base, stream); break;
    default: st = launch_ms<4>(a, di, p.grid_split, p.coop_launch, want_stats, ntiles, d_tile_base, stream); break;
  }
  gap_status st2 = coop_end(dev, stream, &order);
  if (st != GAP_OK) return st;
  if (st2 != GAP_OK) return st2;
  if (want_stats) {
    GAP_HIP(hipStreamSynchronize(stream));
    int err = 0;
    GAP_HIP(hipMemcpy(&err, &a.ctl->base.err, sizeof(int), hipMemcpyDeviceToHost));
    if (err != 0) {
      set_error(err == GAP_ETIMEOUT ? "device-side wait timed out (grid barrier)"
                                    : "batch ran more levels than vertices");
      return err;
    }
    static_assert(offsetof(MsCtl, lvstat) == offsetof(MsCtl, trace) +
                                                 sizeof(unsigned long long) * kMsTraceLevels * 6,
                  "trace and lvstat are copied together");
    std::vector<unsigned long long> tr((size_t)kMsTraceLevels * 8);
    GAP_HIP(hipMemcpy(tr.data(), reinterpret_cast<char *>(a.ctl) + offsetof(MsCtl, trace),
                      tr.size() * sizeof(unsigned long long), hipMemcpyDeviceToHost));
    const unsigned long long *T = tr.data();
    const unsigned long long *LS = tr.data() + (size_t)kMsTraceLevels * 6;
    int levels = 0;
    while (levels < kMsTraceLevels && T[levels * 6 + 2] != 0ull) ++levels;
    const int nrec = std::min(levels, max_levels);
    for (int d = 0; d < nrec; ++d) {
      gap_level_stat &r = stats[d];
      r.level = d;
      r.direction = (int32_t)T[d * 6 + 3];
      r.frontier = (int64_t)T[d * 6 + 4];
      r.frontier_edges = (int64_t)T[d * 6 + 5];
      r.claimed = d + 1 < levels ? (int64_t)T[(d + 1) * 6 + 4] : 0;
      r.unvisited = r.direction == kBottomUp ? (int64_t)LS[d * 2 + 0] : 0;
      r.scanned = r.direction == kBottomUp ? (int64_t)LS[d * 2 + 1] : r.frontier_edges;
      r.time_ns = T[d * 6 + 2] > T[d * 6 + 0] ? (int64_t)((T[d * 6 + 2] - T[d * 6 + 0]) * 10ull) : 0;
    }
    if (num_levels) *num_levels = levels;
  }
  if (getenv("GAP_MS_TRACE")) {  // development aid: per-level timing of segment 0
    GAP_HIP(hipStreamSynchronize(stream));
    static unsigned long long tr[kMsTraceLevels][6];
    GAP_HIP(hipMemcpy(tr, reinterpret_cast<char *>(a.ctl) + offsetof(MsCtl, trace), sizeof(tr),
                      hipMemcpyDeviceToHost));
    for (int d = 0; d < kMsTraceLevels && tr[d][0] && tr[d][2]; ++d)
      fprintf(stderr, "[ms] W=%d level %d dir %llu nf %llu mf %llu advance %.1f us step %.1f us\n",
              W, d, tr[d][3], tr[d][4], tr[d][5], (tr[d][1] - tr[d][0]) / 100.0,
              (tr[d][2] - tr[d][1]) / 100.0);
  }
  return GAP_OK;
}

}  // namespace gap
