// Single-source direction-optimizing BFS on gfx950: kernels and the three
// level schedules.
//  * persistent: one cooperative kernel runs every level; levels are
//    separated by a reducing grid barrier;
//  * levels: one launch per step, device-side decisions, the host waits for
//    each level's "done" flag;
//  * graph: the same per-level kernels captured into a hipGraph of K levels
//    that is replayed until the device reports the search done.
#include <algorithm>
#include <mutex>
#include <vector>

#include "bfs_kernels.h"
#include "runtime.h"

namespace gap {

struct SearchArgs {
  DevGraph g;
  int32_t *parent;
  int32_t *depth;
  int32_t source;
  Queues Q;
  uint64_t *bm0, *bm1;  // frontier bitmaps (current / next alternate)
  uint64_t *vbm;
  Ctl *ctl;
  Ctl *ctl_clear;  // persistent kernel: the next search's control block, cleared at start
  int *sticky;     // the stream's sticky status word (persistent kernel)
  Params p;
  DevLevelRec *recs;
  int32_t max_recs;
  int64_t lds_words;  // frontier bitmap words held in each workgroup's dynamic LDS (0: none)
};

// ---- persistent cooperative kernel -------------------------------------------

// Small levels: a top-down level whose frontier and frontier edges are both
// at most p.small runs on the first GAP_SMALL_GROUP workgroups only, which
// meet at a barrier of their own (a barrier's cost grows with the number of arriving
// workgroups, and such a level has too little work to need the whole grid).
// The other workgroups park until the small group hands the search back:
// the last arriver of each level's barrier decides whether the next level
// is small and sends the answer with the release; when the small group
// stops (a large level next, or the search done) it stores its state in
// ctl->park and the level to rejoin at in ctl->resume.
// Longest source list whose level 0 is folded into the initialisation.
#ifndef GAP_FOLD_DEGREE
#define GAP_FOLD_DEGREE 4096
#endif
constexpr int64_t kFoldDegree = GAP_FOLD_DEGREE;

// Workgroups (of the block size in use) that run the small levels.
// Measured on the 4096^2 grid, whose ~5,100 levels are nearly all small:
// 1, 2, 4, 8, 16, 32, 64, 128 workgroups gave 250, 176, 131, 95, 74.2,
// 71.0, 71.1, 74.6 ms per search (R-MAT and uniform scale 22 unchanged).
#ifndef GAP_SMALL_GROUP
#define GAP_SMALL_GROUP 32
#endif

struct SmallDecision {
  int64_t n, mu, nv, small_limit;
  int32_t dir, d, have_bm, fsel_next;
  Params p;
  bool in_small, enabled;
  __device__ BarrierDecision operator()(Ctl *ctl, const Totals &all) const {
    const int64_t nv1 = (int64_t)all.nv, mf1 = (int64_t)all.mf;
    int small_next = 0;
    if (enabled && nv1 > 0 && nv1 <= small_limit && mf1 <= small_limit) {
      const int32_t nd = decide_direction(dir, nv1, mf1, mu - mf1, nv, n, p, d + 1);
      small_next = (nd == kTopDown);
    }
    if (in_small && !small_next) {
      ParkState ps;
      ps.level = d + 1;
      ps.dir = dir;
      ps.have_bm = have_bm;
      ps.fsel = fsel_next;
      ps.mu = mu;
      ps.nf_prev = nv;
      ctl->park = ps;
      return {0, d + 1};
    }
    return {small_next, -1};
  }
};

// Level 0 folded into the initialisation (whole workgroup, after it has
// initialised [lo, hi)): the source's neighbours in [lo, hi) get parent
// `source` and depth 1 and are appended to F_1 (buffer set 1) as a top-down
// step would append them; returns the workgroup's totals in thread 0.  Kept
// out of line: it runs once per search, and inlined its registers would
// count against the level loop's.
template <int BLOCK, bool STATS>
__device__ __forceinline__ Totals fold_level0(const SearchArgs &a, Stage<BLOCK> &st, int64_t lo, int64_t hi,
                                           int64_t s_beg, int64_t s_end) {
  __syncthreads();  // this workgroup's vertices are initialised
  StepArgs s{a.g, a.parent, a.depth, a.Q, 0, a.ctl, nullptr, nullptr, nullptr, 0, a.p.hub, a.p.chunk};
  step_begin<BLOCK>(s, st, false);
  LaneAcc acc;
  for (int64_t e0 = s_beg; e0 < s_end; e0 += BLOCK) {  // the same trip count on every thread
    const int64_t e = e0 + threadIdx.x;
    const int32_t v = e < s_end ? a.g.col[e] : -1;
    const bool mine = v >= lo && v < hi;
    int64_t degv = 0;
    if (mine) {
      degv = a.g.row_ptr[v + 1] - a.g.row_ptr[v];
      a.parent[v] = a.source;
      a.depth[v] = 1;
    }
    stage_append<BLOCK>(s, st, mine, v, degv, acc);
  }
  if (STATS && blockIdx.x == 0 && threadIdx.x == 0) acc.scanned += (unsigned long long)(s_end - s_beg);
  return step_end<BLOCK>(s, st, acc);
}

template <int BLOCK, bool STATS>
__device__ __forceinline__ void bfs_persistent(const SearchArgs &a) {
  __shared__ Stage<BLOCK> st;
  extern __shared__ uint64_t lds_fbm[];  // frontier bitmap words [0, lds_words)
  const int64_t nthreads = (int64_t)gridDim.x * BLOCK;
  const int64_t tid = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
  const int64_t nwaves = nthreads / kWave;
  const int64_t gwave = uni(tid / kWave);
  const unsigned int nblocks = gridDim.x;
  const unsigned int nsmall = nblocks < (unsigned)GAP_SMALL_GROUP ? nblocks : (unsigned)GAP_SMALL_GROUP;
  const bool small_enabled = a.p.small > 0 && nblocks > nsmall;
  const int64_t nwords_all = (a.g.n + kWave - 1) / kWave;

  // Level 0 expands F_0 = {source}.  When the source's list is short it is
  // folded into the initialisation: workgroup b initialises the vertices of
  // its own range [lo, hi) and then claims the source's neighbours in that
  // range (no other workgroup writes them), appending F_1 as a top-down
  // step would; the first barrier then ends level 0.
  const int64_t s_beg = a.g.row_ptr[a.source], s_end = a.g.row_ptr[a.source + 1];
  const bool fold = a.p.direction != GAP_DIR_BOTTOMUP && s_end > s_beg && s_end - s_beg <= kFoldDegree;
  const unsigned long long t_init = (STATS || a.recs) ? rt_clock() : 0ull;
  const int64_t per = ((a.g.n + 3) / 4 + nblocks - 1) / nblocks * 4;
  const int64_t lo = (int64_t)blockIdx.x * per < a.g.n ? (int64_t)blockIdx.x * per : a.g.n;
  const int64_t hi = lo + per < a.g.n ? lo + per : a.g.n;
  init_vertices_range<BLOCK>(a.g, a.parent, a.depth, a.source, lo, hi);
  if (a.ctl_clear) {  // no search uses it now: the one before this has finished with it
    uint32_t *w = reinterpret_cast<uint32_t *>(a.ctl_clear);
    for (int64_t i = tid; i < (int64_t)(sizeof(Ctl) / sizeof(uint32_t)); i += nthreads) w[i] = 0u;
  }
  Totals part = {};
  int32_t d = 0, dir = kTopDown;
  bool have_bm = false;
  int64_t mu = a.g.nnz, nf_prev = 0;
  int fsel = 0;
  bool small = false;     // this level runs on the small group
  bool bm_ready = false;  // F_d's bitmaps were read back at the end of a plain-claim level
  if (fold) {
    part = fold_level0<BLOCK, STATS>(a, st, lo, hi, s_beg, s_end);
    if ((STATS || a.recs) && tid == 0 && a.max_recs > 0) {
      DevLevelRec r = {};
      r.level = 0;
      r.direction = kTopDown;
      r.frontier = 1;
      r.frontier_edges = (unsigned long long)(s_end - s_beg);
      r.t_start = t_init;
      a.recs[0] = r;
    }
    mu -= s_end - s_beg;
    const SmallDecision dec{a.g.n, mu, 1, (int64_t)a.p.small, kTopDown, 0, 0, 0,
                            a.p, false, small_enabled};
    int small_next = 0;
    if (!grid_sync_x(a.ctl, main_barrier(a.ctl, a.p.wait), nblocks, part, 1, 1, dec, small_next))
      return;
    small_next = uni(small_next);
    d = 1;
    nf_prev = 1;
    if (small_next && blockIdx.x >= nsmall) {
      ParkState ps;
      if (!park_wait(a.ctl, (unsigned int)d, ps, a.p.wait_park)) return;
      d = uni(ps.level);
      dir = uni(ps.dir);
      have_bm = uni(ps.have_bm) != 0;
      fsel = uni(ps.fsel);
      mu = uni((int64_t)ps.mu);
      nf_prev = uni((int64_t)ps.nf_prev);
    } else {
      small = small_next != 0;
    }
  } else {
    if (tid == 0) part = init_source(a.g, a.Q, a.ctl, a.source, a.p.hub, a.p.chunk);
    if (!grid_sync(a.ctl, nblocks, part, 0, 0, a.p.wait)) return;
  }
  for (;;) {
    const Published &P = a.ctl->pub[d & 1];
    const int64_t nv = uni((int64_t)ld_agent(&P.t.nv));
    const int64_t mf = uni((int64_t)ld_agent(&P.t.mf));
    if (STATS && tid == 0 && d > 0 && d - 1 < a.max_recs) {
      a.recs[d - 1].claimed = (unsigned long long)nv;
      a.recs[d - 1].scanned = ld_agent(&P.t.scanned);
      a.recs[d - 1].unvisited = ld_agent(&P.t.unvisited);
      a.recs[d - 1].t_end = rt_clock();
    }
    if (nv == 0) break;
    if (d > a.g.n) {  // more levels than vertices: inconsistent counters
      if (tid == 0) atomicExch(&a.ctl->err, (int)GAP_EINTERNAL);
      return;
    }
    const unsigned long long level_t0 = STATS ? rt_clock() : 0ull;
    mu -= mf;
    const int32_t ndir = decide_direction(dir, nv, mf, mu, nf_prev, a.g.n, a.p, d);
    if (ndir == kBottomUp && !bm_ready && !(dir == kBottomUp && have_bm)) {
      convert_to_bitmaps(a.g, a.parent, a.depth, d, (fsel ? a.bm1 : a.bm0), a.vbm, gwave, nwaves);
      if (!grid_sync(a.ctl, nblocks, Totals{}, -1, 0, a.p.wait)) return;
    }
    if (ndir == kBottomUp) have_bm = true;
    if ((dir == kBottomUp || bm_ready) && ndir == kTopDown) {
      // the bottom-up steps (or the read-back after plain claims) left F_d
      // as a bitmap only: queue it for this top-down step (buffer set
      // d & 1), on the workgroups that run it
      StepArgs c{a.g, a.parent, a.depth, a.Q, (d & 1) ^ 1, a.ctl, nullptr, nullptr, nullptr,
                 d, a.p.hub, a.p.chunk};
      queue_from_bitmap<BLOCK>(c, st, (fsel ? a.bm1 : a.bm0), gwave,
                               small ? (int64_t)nsmall * (BLOCK / kWave) : nwaves);
      int unused = 0;
      if (!grid_sync_x(a.ctl, small ? small_barrier(a.ctl, a.p.wait) : main_barrier(a.ctl, a.p.wait),
                       small ? nsmall : nblocks, Totals{}, d & 1, d & 1, NoDecision{}, unused))
        return;
    }
    if (ndir == kTopDown) have_bm = false;
    bm_ready = false;
    dir = ndir;
    // a large top-down level claims by plain stores (never on the small
    // group, whose parked workgroups would not know that F_{d+1} comes back
    // as bitmaps)
    const bool plain = dir == kTopDown && !small && a.p.td_plain > 0 &&
                       mf > a.g.n / (int64_t)a.p.td_plain;
    if (STATS && tid == 0 && d < a.max_recs) {
      DevLevelRec r = {};
      r.level = d;
      r.direction = dir;
      r.frontier = (unsigned long long)nv;
      r.frontier_edges = (unsigned long long)mf;
      r.t_start = level_t0;
      a.recs[d] = r;
    }
    StepArgs s{a.g, a.parent, a.depth, a.Q, d & 1, a.ctl, (fsel ? a.bm1 : a.bm0), a.vbm, (fsel ? a.bm0 : a.bm1),
               d, a.p.hub, a.p.chunk};
    step_begin<BLOCK>(s, st, dir == kTopDown);  // a bottom-up step reads no queue
    // the LDS copy of the frontier bitmap pays when a workgroup has more
    // list entries left to probe (mu bounds them) than words to copy
    const int64_t lw = (mu / (int64_t)nblocks >= a.lds_words) ? a.lds_words : 0;
    LaneAcc acc;
    if (dir == kTopDown && plain)
      td_step<BLOCK, STATS, true, true>(s, st, acc, gwave, nwaves);
    else if (dir == kTopDown)
      td_step<BLOCK, STATS, true>(s, st, acc, gwave, small ? (int64_t)nsmall * (BLOCK / kWave) : nwaves);
    else if (a.p.bu_mapping == 0 && (nwords_all + nblocks - 1) / nblocks <= bu_refill_words<BLOCK>()) {
      // never on the small group: every workgroup takes its share of the words
      const int64_t per = (nwords_all + nblocks - 1) / nblocks;
      const int64_t wlo = (int64_t)blockIdx.x * per < nwords_all ? (int64_t)blockIdx.x * per : nwords_all;
      const int64_t whi = wlo + per < nwords_all ? wlo + per : nwords_all;
      bu_step_refill<BLOCK, STATS, GAP_BU_SLOTS>(s, st, acc, wlo, whi, lds_fbm, lw);
    } else
      bu_step<BLOCK, STATS, GAP_BU_WORDS, GAP_BU_ROUND2, false>(s, st, acc, gwave,
                                                                nwaves,  // never on the small group
                                                                lds_fbm, lw);
    Totals t = step_end<BLOCK>(s, st, acc);
    if (plain) {
      // F_{d+1} is every vertex at depth d + 1: after the claims' barrier,
      // build its bitmaps (in the current slot: a top-down step keeps fsel)
      // and count it, for the barrier below and the next level
      const unsigned long long scanned = t.scanned;  // thread 0's
      if (!grid_sync(a.ctl, nblocks, Totals{}, -1, 0, a.p.wait)) return;
      step_begin<BLOCK>(s, st, false);
      convert_to_bitmaps<true>(a.g, a.parent, a.depth, d + 1, (fsel ? a.bm1 : a.bm0), a.vbm, gwave,
                               nwaves, &acc);
      t = step_end<BLOCK>(s, st, acc);
      t.scanned += scanned;
    }
    const int fsel_next = (dir == kBottomUp) ? (fsel ^ 1) : fsel;
    const SmallDecision dec{a.g.n, mu, nv, (int64_t)a.p.small, dir, d, have_bm ? 1 : 0, fsel_next,
                            a.p, small, small_enabled};
    int small_next = 0;
    const BarrierSet bar = small ? small_barrier(a.ctl, a.p.wait) : main_barrier(a.ctl, a.p.wait);
    if (!grid_sync_x(a.ctl, bar, small ? nsmall : nblocks, t, (d + 1) & 1, (d + 1) & 1, dec,
                     small_next))
      return;
    small_next = uni(small_next);
    fsel = fsel_next;
    nf_prev = nv;
    bm_ready = plain;
    ++d;
    if (small_next && !small && blockIdx.x >= nsmall) {
      // park until the small group hands the search back
      ParkState ps;
      if (!park_wait(a.ctl, (unsigned int)d, ps, a.p.wait_park)) return;
      d = uni(ps.level);
      dir = uni(ps.dir);
      have_bm = uni(ps.have_bm) != 0;
      fsel = uni(ps.fsel);
      mu = uni((int64_t)ps.mu);
      nf_prev = uni((int64_t)ps.nf_prev);
      bm_ready = false;  // the small group (which never claims by plain stores) hands over
      continue;
    }
    small = small_next != 0;
  }
  // every vertex with an out-list was reached (the frontiers' edges add up
  // to nnz) and there is no other: no parent is left negative
  if (!(mu == 0 && a.g.n_sinks == 0)) fixup_parents(a.g.n, a.parent, tid, nthreads);
  if (tid == 0) a.ctl->levels = d;
}

template <int BLOCK, bool STATS>
__global__ __launch_bounds__(BLOCK) void k_bfs_persistent(SearchArgs a) {
  bfs_persistent<BLOCK, STATS>(a);
  note_error(a.sticky, a.ctl);
}

// ---- device-driven per-level kernels (levels and graph schedules) -------------
// The search state lives in Ctl (level, dir, done, have_bm, mu, nf_prev) and
// the per-search arguments in device memory, so a captured graph can be
// replayed for any source and output buffers.

constexpr int kLevelBlock = 256;

struct alignas(64) DDArgs {
  SearchArgs s;
  int fsel;          // 1 when bm1 holds the current frontier bitmap
  int need_convert;  // the next step is bottom-up and needs the bitmaps
};
static_assert(sizeof(DDArgs) <= 1024, "argument block must fit the workspace slot");

__global__ __launch_bounds__(kLevelBlock) void k_dd_init(DDArgs *A) {
  const SearchArgs a = A->s;
  const int64_t nthreads = (int64_t)gridDim.x * blockDim.x;
  const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  init_vertices(a.g, a.parent, a.depth, a.source, tid, nthreads);
  if (tid == 0) {
    const Totals t = init_source(a.g, a.Q, a.ctl, a.source, a.p.hub, a.p.chunk);
    add_totals(a.ctl->grp[0], t);
    a.ctl->level = -1;
    a.ctl->dir = kTopDown;
    a.ctl->have_bm = 0;
    a.ctl->mu = a.g.nnz;
    a.ctl->nf_prev = 0;
    a.ctl->done = 0;
    A->fsel = 0;
    A->need_convert = 0;
  }
}

// Closes level L = ctl->level (L = -1 after init): reduces the level's
// totals, publishes F_{L+1}, and decides how level L+1 runs.  One wave:
// lane h handles group h, lane 0 decides.
template <bool STATS>
__global__ __launch_bounds__(64) void k_dd_publish(DDArgs *A) {
  const int lane = threadIdx.x;
  const SearchArgs &a = A->s;
  Ctl *ctl = a.ctl;
  if (ctl->done) return;
  const int L = ctl->level;
  const int d = L + 1;
  Totals p = {};
  if (lane < kGroups) {
    p = take_totals(ctl->grp[lane]);
    publish_segment(ctl, d & 1, d & 1, lane);
  }
  Totals t;
  t.nv = wave_sum_u64(p.nv);
  t.mf = wave_sum_u64(p.mf);
  t.scanned = wave_sum_u64(p.scanned);
  t.unvisited = wave_sum_u64(p.unvisited);
  if (lane != 0) return;
  publish_totals(ctl, d & 1, t);
  if (STATS && L >= 0 && L < a.max_recs) {
    a.recs[L].claimed = t.nv;
    a.recs[L].scanned = t.scanned;
    a.recs[L].unvisited = t.unvisited;
    a.recs[L].t_end = rt_clock();
  }
  if (L >= 0 && ctl->dir == kBottomUp) A->fsel ^= 1;
  const int64_t nv = (int64_t)t.nv, mf = (int64_t)t.mf;
  if (nv == 0) {
    ctl->done = 1;
    ctl->levels = d;
    return;
  }
  if (d > a.g.n) {
    ctl->err = GAP_EINTERNAL;
    ctl->done = 1;
    return;
  }
  ctl->mu -= mf;
  const int32_t dir = ctl->dir;
  const int32_t ndir = decide_direction(dir, nv, mf, ctl->mu, ctl->nf_prev, a.g.n, a.p, d);
  A->need_convert = (ndir == kBottomUp && !(dir == kBottomUp && ctl->have_bm)) ? 1 : 0;
  ctl->have_bm = (ndir == kBottomUp) ? 1 : 0;
  ctl->dir = ndir;
  ctl->nf_prev = nv;
  ctl->level = d;
  if (STATS && d < a.max_recs) {
    DevLevelRec r = {};
    r.level = d;
    r.direction = ndir;
    r.frontier = (unsigned long long)nv;
    r.frontier_edges = (unsigned long long)mf;
    r.t_start = rt_clock();
    a.recs[d] = r;
  }
}

__global__ __launch_bounds__(kLevelBlock) void k_dd_convert(DDArgs *A) {
  const SearchArgs &a = A->s;
  if (a.ctl->done || !A->need_convert) return;
  const int64_t nwaves = (int64_t)gridDim.x * blockDim.x / kWave;
  const int64_t gwave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
  convert_to_bitmaps(a.g, a.parent, a.depth, a.ctl->level, (A->fsel ? a.bm1 : a.bm0), a.vbm, gwave, nwaves);
}

template <bool STATS>
__global__ __launch_bounds__(kLevelBlock) void k_dd_step(DDArgs *A) {
  __shared__ Stage<kLevelBlock> st;
  const SearchArgs &a = A->s;
  if (a.ctl->done) return;
  const int d = a.ctl->level;
  const int fsel = A->fsel;
  const int64_t nwaves = (int64_t)gridDim.x * blockDim.x / kWave;
  const int64_t gwave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
  StepArgs s{a.g, a.parent, a.depth, a.Q, d & 1, a.ctl, (fsel ? a.bm1 : a.bm0), a.vbm, (fsel ? a.bm0 : a.bm1),
             d, a.p.hub, a.p.chunk};
  step_begin<kLevelBlock>(s, st);
  LaneAcc acc;
  if (a.ctl->dir == kTopDown)
    td_step<kLevelBlock, STATS>(s, st, acc, gwave, nwaves);
  else
    bu_step<kLevelBlock, STATS>(s, st, acc, gwave, nwaves);
  const Totals t = step_end<kLevelBlock>(s, st, acc);
  if (threadIdx.x == 0) add_totals(a.ctl->grp[blockIdx.x % kGroups], t);
}

__global__ __launch_bounds__(kLevelBlock) void k_dd_fixup(DDArgs *A) {
  const SearchArgs &a = A->s;
  const int64_t nthreads = (int64_t)gridDim.x * blockDim.x;
  const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  fixup_parents(a.g.n, a.parent, tid, nthreads);
}

// ---- host side ----------------------------------------------------------------

template <int BLOCK, bool STATS>
static gap_status launch_persistent(const SearchArgs &a, const DeviceInfo *di, int blocks_per_cu,
                                    int split, int coop, int lds_bitmap, hipStream_t stream) {
  auto kern = k_bfs_persistent<BLOCK, STATS>;
  SearchArgs args = a;
  // the frontier bitmap goes to LDS next to the static staging: all of it
  // when it fits, else as many of its low words as the LDS left to each of
  // the workgroups that share a compute unit holds (at least kMinLdsWords)
  constexpr int64_t kMinLdsWords = 1024;
  size_t shmem = 0;
  args.lds_words = 0;
  if (lds_bitmap) {
    hipFuncAttributes attr{};
    int fit0 = 0;
    if (hipFuncGetAttributes(&attr, (const void *)kern) == hipSuccess &&
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&fit0, kern, BLOCK, 0) == hipSuccess &&
        fit0 > 0) {
      const int want = blocks_per_cu > 0 && blocks_per_cu < fit0 ? blocks_per_cu : fit0;
      const int64_t room = std::min<int64_t>(di->lds_per_block, di->lds_per_cu / want) -
                           (int64_t)attr.sharedSizeBytes - 1024;
      const int64_t nwords = (a.g.n + kWave - 1) / kWave;
      const int64_t words = std::min<int64_t>(nwords, room / (int64_t)sizeof(uint64_t));
      if (words >= std::min<int64_t>(nwords, kMinLdsWords) && words > 0) {
        shmem = (size_t)words * sizeof(uint64_t);
        args.lds_words = words;
      }
    }
    (void)hipGetLastError();
  }
  int per_cu = 0;
  GAP_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, BLOCK, shmem));
  if (per_cu < 1) {
    set_error("persistent kernel does not fit on a compute unit");
    return GAP_EDEVICE;
  }
  if (blocks_per_cu > 0 && blocks_per_cu < per_cu) per_cu = blocks_per_cu;
  void *kargs[] = {&args};
  return launch_resident((const void *)kern, per_cu * di->cus, BLOCK, shmem, kargs, split, coop,
                         di, stream, nullptr);
}

template <bool STATS>
static gap_status dispatch_persistent(const SearchArgs &a, const DeviceInfo *di,
                                      const gap_params &p, hipStream_t stream) {
  switch (p.block) {
    case 256:
      return launch_persistent<256, STATS>(a, di, p.blocks_per_cu, p.grid_split, p.coop_launch, p.lds_bitmap,
                                           stream);
    case 512:
      return launch_persistent<512, STATS>(a, di, p.blocks_per_cu, p.grid_split, p.coop_launch, p.lds_bitmap,
                                           stream);
    default:
      return launch_persistent<1024, STATS>(a, di, p.blocks_per_cu, p.grid_split, p.coop_launch, p.lds_bitmap,
                                            stream);
  }
}

// Grid of the per-level kernels: enough waves to cover the largest step
// (one wave per 64-vertex word), capped so the launch stays cheap.
static int level_grid(const DeviceInfo *di, int64_t n) {
  const int64_t words = (n + kWave - 1) / kWave;
  const int64_t wpb = kLevelBlock / kWave;
  int64_t b = (words + wpb - 1) / wpb;
  const int64_t cap = (int64_t)di->cus * 8;
  if (b > cap) b = cap;
  if (b < 1) b = 1;
  return (int)b;
}

static gap_status enqueue_level(DDArgs *dA, int grid, bool stats, hipStream_t stream) {
  k_dd_convert<<<grid, kLevelBlock, 0, stream>>>(dA);
  if (stats) {
    k_dd_step<true><<<grid, kLevelBlock, 0, stream>>>(dA);
    k_dd_publish<true><<<1, 64, 0, stream>>>(dA);
  } else {
    k_dd_step<false><<<grid, kLevelBlock, 0, stream>>>(dA);
    k_dd_publish<false><<<1, 64, 0, stream>>>(dA);
  }
  GAP_HIP(hipGetLastError());
  return GAP_OK;
}

// Reads err, levels and done from the device (synchronous).
static gap_status read_flags(Workspace *ws, const Ctl *ctl, hipStream_t stream, int *done,
                             int *levels, int *err) {
  static_assert(offsetof(Ctl, levels) == offsetof(Ctl, err) + sizeof(int), "Ctl layout");
  static_assert(offsetof(Ctl, done) == offsetof(Ctl, err) + 2 * sizeof(int), "Ctl layout");
  static_assert(sizeof(Ctl) % sizeof(uint32_t) == 0, "Ctl is cleared word by word");
  GAP_HIP(hipMemcpyAsync(ws->h_flags, &ctl->err, 3 * sizeof(int), hipMemcpyDeviceToHost,
                         stream));
  GAP_HIP(hipStreamSynchronize(stream));
  *err = ws->h_flags[0];
  *levels = ws->h_flags[1];
  *done = ws->h_flags[2];
  return GAP_OK;
}

static gap_status run_device_driven(const SearchArgs &a, const gap_params &p, bool stats,
                                    Workspace *ws, const DeviceInfo *di, hipStream_t stream,
                                    int32_t *levels_out) {
  DDArgs *dA = reinterpret_cast<DDArgs *>(ws->dd_args);
  // the arguments travel through pinned memory so the copy is truly async;
  // wait first: the previous search on this stream may still read it
  GAP_HIP(hipStreamSynchronize(stream));
  DDArgs *pin = reinterpret_cast<DDArgs *>(ws->h_args);
  *pin = DDArgs{};
  pin->s = a;
  GAP_HIP(hipMemcpyAsync(dA, pin, sizeof(DDArgs), hipMemcpyHostToDevice, stream));
  GAP_HIP(hipMemsetAsync(ws->ctl, 0, sizeof(Ctl), stream));
  const int grid = level_grid(di, a.g.n);
  k_dd_init<<<grid, kLevelBlock, 0, stream>>>(dA);
  if (stats)
    k_dd_publish<true><<<1, 64, 0, stream>>>(dA);
  else
    k_dd_publish<false><<<1, 64, 0, stream>>>(dA);
  GAP_HIP(hipGetLastError());
  int done = 0, levels = 0, err = 0;
  if (p.mode == GAP_MODE_LEVELS) {
    for (int64_t it = 0;; ++it) {
      gap_status st = read_flags(ws, ws->ctl, stream, &done, &levels, &err);
      if (st != GAP_OK) return st;
      if (done || err) break;
      if (it > a.g.n + 1) {
        set_error("search ran more levels than vertices");
        return GAP_EINTERNAL;
      }
      st = enqueue_level(dA, grid, stats, stream);
      if (st != GAP_OK) return st;
    }
  } else {
    // hipGraph of K levels, captured once per workspace, chunk size and grid
    const int K = p.graph_chunk;
    const int key = K * 4 + (stats ? 2 : 0) + 1;
    if (!ws->graph_exec || ws->graph_key != key || ws->graph_grid != grid) {
      if (ws->graph_exec) (void)hipGraphExecDestroy((hipGraphExec_t)ws->graph_exec);
      ws->graph_exec = nullptr;
      hipStream_t cap = nullptr;
      GAP_HIP(hipStreamCreateWithFlags(&cap, hipStreamNonBlocking));
      hipGraph_t graph = nullptr;
      hipError_t e = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal);
      if (e == hipSuccess) {
        for (int k = 0; k < K; ++k) (void)enqueue_level(dA, grid, stats, cap);
        e = hipStreamEndCapture(cap, &graph);
      }
      hipGraphExec_t exec = nullptr;
      if (e == hipSuccess) e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
      if (graph) (void)hipGraphDestroy(graph);
      (void)hipStreamDestroy(cap);
      if (e != hipSuccess) return hip_fail(e, "capturing the level graph");
      ws->graph_exec = exec;
      ws->graph_key = key;
      ws->graph_grid = grid;
    }
    for (int64_t it = 0;; ++it) {
      gap_status st = read_flags(ws, ws->ctl, stream, &done, &levels, &err);
      if (st != GAP_OK) return st;
      if (done || err) break;
      if (it * K > a.g.n + 1) {
        set_error("search ran more levels than vertices");
        return GAP_EINTERNAL;
      }
      GAP_HIP(hipGraphLaunch((hipGraphExec_t)ws->graph_exec, stream));
    }
  }
  if (err) {
    set_error("device reported an inconsistent search state");
    return GAP_EINTERNAL;
  }
  k_dd_fixup<<<grid, kLevelBlock, 0, stream>>>(dA);
  GAP_HIP(hipGetLastError());
  *levels_out = levels;
  return GAP_OK;
}

gap_status run_bfs(const gap_graph *g, int32_t source, int32_t *parent, int32_t *depth,
                   hipStream_t stream, const gap_params &p, gap_level_stat *stats,
                   int32_t max_levels, int32_t *num_levels) {
  const DeviceInfo *di = nullptr;
  gap_status st = device_info(g->device, &di);
  if (st != GAP_OK) return st;
  GAP_HIP(hipSetDevice(g->device));
  Workspace *ws = workspace_for(g->device, stream);
  if (!ws) {
    set_error("workspace allocation failed");
    return GAP_ENOMEM;
  }
  st = workspace_reserve_single(ws, g->n, g->nnz, p);
  if (st != GAP_OK) return st;
  const bool want_stats = stats != nullptr && max_levels > 0;
  if (want_stats) {
    st = workspace_reserve_recs(ws, max_levels);
    if (st != GAP_OK) return st;
  }
  SearchArgs a{};
  a.g = DevGraph{g->row_ptr, g->col, g->row_ptr_in, g->col_in, g->head_in, g->n, g->nnz,
                 g->directed, g->n_sinks};
  a.parent = parent;
  a.depth = depth ? depth : ws->depth_scratch;
  a.source = source;
  a.Q.q0 = ws->q[0];
  a.Q.q1 = ws->q[1];
  a.Q.c0 = ws->cq[0];
  a.Q.c1 = ws->cq[1];
  a.Q.n = ws->cap_n;
  a.Q.ccap = ws->cap_chunks;
  a.bm0 = ws->bm[0];
  a.bm1 = ws->bm[1];
  a.vbm = ws->bm[2];
  a.ctl = ws->ctl;
  a.p = Params{p.alpha, p.beta, p.direction, p.hub_degree, p.chunk_edges, p.small_frontier,
               p.bu_mapping, p.td_plain, 0, 0};
  set_wait_limits(a.p, p.wait_limit_us);
  a.sticky = ws->sticky;
  a.recs = want_stats ? ws->recs : nullptr;
  a.max_recs = want_stats ? max_levels : 0;

  int32_t levels = -1;
  const bool device_driven = p.mode == GAP_MODE_LEVELS || p.mode == GAP_MODE_GRAPH;
  Ctl *used = ws->ctl;
  if (device_driven) {
    ws->ctl_next_clean = false;  // ctl[0] is left as this schedule leaves it
    a.ctl_clear = nullptr;
    st = run_device_driven(a, p, want_stats, ws, di, stream, &levels);
    if (st != GAP_OK) return st;
  } else {
    // the device's launch lock (held from coop_begin to coop_end) also
    // keeps the choice of control block consistent between host threads
    CoopOrder order;
    st = coop_begin(g->device, stream, p.grid_split, &order);
    if (st != GAP_OK) return st;
    used = ws->ctl + (ws->ctl_seq & 1);
    if (!ws->ctl_next_clean) GAP_HIP(hipMemsetAsync(used, 0, sizeof(Ctl), stream));
    ws->ctl_next_clean = false;  // until this search's kernel is queued
    a.ctl = used;
    a.ctl_clear = ws->ctl + ((ws->ctl_seq + 1) & 1);
    st = want_stats ? dispatch_persistent<true>(a, di, p, stream)
                    : dispatch_persistent<false>(a, di, p, stream);
    if (st == GAP_OK) {
      ws->ctl_seq += 1;
      ws->ctl_next_clean = true;
    }
    gap_status st2 = coop_end(g->device, stream, &order);
    if (st != GAP_OK) return st;
    if (st2 != GAP_OK) return st2;
  }
  if (want_stats) {
    int done = 0, err = 0, lv = 0;
    st = read_flags(ws, used, stream, &done, &lv, &err);
    if (st != GAP_OK) return st;
    if (err != 0) {
      set_error(err == GAP_ETIMEOUT ? "device-side wait timed out (grid barrier)"
                                    : "search ran more levels than vertices");
      return err;
    }
    levels = lv;
    std::vector<DevLevelRec> recs((size_t)std::max(0, std::min(levels, max_levels)));
    if (!recs.empty())
      GAP_HIP(hipMemcpy(recs.data(), ws->recs, recs.size() * sizeof(DevLevelRec),
                        hipMemcpyDeviceToHost));
    for (size_t i = 0; i < recs.size(); ++i) {
      stats[i].level = recs[i].level;
      stats[i].direction = recs[i].direction;
      stats[i].frontier = (int64_t)recs[i].frontier;
      stats[i].frontier_edges = (int64_t)recs[i].frontier_edges;
      stats[i].claimed = (int64_t)recs[i].claimed;
      stats[i].scanned = (int64_t)recs[i].scanned;
      stats[i].unvisited = (int64_t)recs[i].unvisited;
      stats[i].time_ns = recs[i].t_end > recs[i].t_start
                             ? (int64_t)((recs[i].t_end - recs[i].t_start) * 10ull)
                             : 0;
    }
  }
  if (num_levels) *num_levels = levels;
  return GAP_OK;
}

// ---- a search that allocates nothing ------------------------------------------------
// For callers that cannot allocate device memory (work queued under stream
// capture, serving loops, harnesses that forbid allocation): the per-search
// scratch of the persistent schedule lives in one file-scope device array.
// Each GPU holds its own copy (zero-initialised data of the code object)
// until the process ends.  Host code names the array only to look up its
// device address, once per device; kernels get that address as an argument.
constexpr size_t kNoAllocBytes = (size_t)GAP_NOALLOC_SCRATCH_BYTES;
static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];

constexpr int kNoAllocMaxDevices = 64;
static std::mutex g_na_mu;
static unsigned char *g_na_ptr[kNoAllocMaxDevices];  // device address of `scratch`, per device

__global__ __launch_bounds__(256) void k_fill_u32(uint32_t *p, int64_t words, uint32_t v) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < words; i += stride) p[i] = v;
}

static size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// Offsets into the array for one search: [0, 256) holds the status word.
struct NoAllocLayout {
  size_t ctl, bm0, bm1, vbm, depth, q0, q1, c0, c1, total;
  int64_t ccap;
};

static NoAllocLayout noalloc_layout(int64_t n, int64_t nnz, const gap_params &p, bool need_depth) {
  NoAllocLayout L{};
  const size_t words = (size_t)((n + kWave - 1) / kWave + 1);
  L.ccap = nnz / p.chunk_edges + nnz / p.hub_degree + 2;  // as the pooled workspace
  size_t o = 256;
  L.ctl = o;
  o = align256(o + sizeof(Ctl));
  L.bm0 = o;
  o = align256(o + sizeof(uint64_t) * words);
  L.bm1 = o;
  o = align256(o + sizeof(uint64_t) * words);
  L.vbm = o;
  o = align256(o + sizeof(uint64_t) * words);
  L.depth = o;
  if (need_depth) o = align256(o + sizeof(int32_t) * (size_t)n);
  L.q0 = o;
  o = align256(o + sizeof(int32_t) * (size_t)n * kGroups);
  L.q1 = o;
  o = align256(o + sizeof(int32_t) * (size_t)n * kGroups);
  L.c0 = o;
  o = align256(o + sizeof(int2) * (size_t)L.ccap * kGroups);
  L.c1 = o;
  o = align256(o + sizeof(int2) * (size_t)L.ccap * kGroups);
  L.total = o;
  return L;
}

// Device address of the array on `dev` (current), looked up on the first
// call for that device; the status word is cleared then, on `stream`.
static gap_status noalloc_base(int dev, hipStream_t stream, unsigned char **out) {
  if (dev < 0 || dev >= kNoAllocMaxDevices) {
    set_error("gap_bfs_noalloc: device %d beyond the %d supported", dev, kNoAllocMaxDevices);
    return GAP_EINVAL;
  }
  std::lock_guard<std::mutex> lk(g_na_mu);
  if (!g_na_ptr[dev]) {
    void *ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
    if (!ptr) {
      set_error("hipGetSymbolAddress(scratch) returned NULL");
      return GAP_EDEVICE;
    }
    k_fill_u32<<<1, 64, 0, stream>>>(reinterpret_cast<uint32_t *>(ptr), 64, 0u);
    GAP_HIP(hipGetLastError());
    coop_prepare(dev);  // the launch-order bookkeeping entry of the device
    g_na_ptr[dev] = reinterpret_cast<unsigned char *>(ptr);
  }
  *out = g_na_ptr[dev];
  return GAP_OK;
}

gap_status run_bfs_noalloc(const gap_graph *g, int32_t source, int32_t *parent, int32_t *depth,
                           hipStream_t stream) {
  const DeviceInfo *di = nullptr;
  gap_status st = device_info(g->device, &di);
  if (st != GAP_OK) return st;
  GAP_HIP(hipSetDevice(g->device));
  gap_params p = params_current();
  const NoAllocLayout L = noalloc_layout(g->n, g->nnz, p, depth == nullptr);
  if (L.total > kNoAllocBytes) {
    set_error("gap_bfs_noalloc: the graph (n = %lld, %lld entries) needs %zu bytes of scratch; "
              "the array holds %zu",
              (long long)g->n, (long long)g->nnz, L.total, kNoAllocBytes);
    return GAP_EINVAL;
  }
  unsigned char *base = nullptr;
  st = noalloc_base(g->device, stream, &base);
  if (st != GAP_OK) return st;
  SearchArgs a{};
  a.g = DevGraph{g->row_ptr, g->col, g->row_ptr_in, g->col_in, g->head_in, g->n, g->nnz,
                 g->directed, g->n_sinks};
  a.parent = parent;
  a.depth = depth ? depth : reinterpret_cast<int32_t *>(base + L.depth);
  a.source = source;
  a.Q.q0 = reinterpret_cast<int32_t *>(base + L.q0);
  a.Q.q1 = reinterpret_cast<int32_t *>(base + L.q1);
  a.Q.c0 = reinterpret_cast<int2 *>(base + L.c0);
  a.Q.c1 = reinterpret_cast<int2 *>(base + L.c1);
  a.Q.n = g->n;
  a.Q.ccap = L.ccap;
  a.bm0 = reinterpret_cast<uint64_t *>(base + L.bm0);
  a.bm1 = reinterpret_cast<uint64_t *>(base + L.bm1);
  a.vbm = reinterpret_cast<uint64_t *>(base + L.vbm);
  a.ctl = reinterpret_cast<Ctl *>(base + L.ctl);
  a.ctl_clear = nullptr;
  a.sticky = reinterpret_cast<int *>(base);
  a.p = Params{p.alpha, p.beta, p.direction, p.hub_degree, p.chunk_edges, p.small_frontier,
               p.bu_mapping, p.td_plain, 0, 0};
  set_wait_limits(a.p, p.wait_limit_us);
  a.recs = nullptr;
  a.max_recs = 0;
  // one cooperative launch (grid_split 1), ordered after the persistent
  // launches of the device's existing ring; no event is created
  p.grid_split = 1;
  CoopOrder order;
  st = coop_begin_existing(g->device, stream, &order);
  if (st != GAP_OK) return st;
  static_assert(sizeof(Ctl) % sizeof(uint32_t) == 0, "Ctl is cleared word by word");
  k_fill_u32<<<8, 256, 0, stream>>>(reinterpret_cast<uint32_t *>(a.ctl),
                                    (int64_t)(sizeof(Ctl) / sizeof(uint32_t)), 0u);
  hipError_t e = hipGetLastError();
  st = e == hipSuccess ? dispatch_persistent<false>(a, di, p, stream) : hip_fail(e, "k_fill_u32");
  const gap_status st2 = coop_end_existing(g->device, stream, &order);
  if (st != GAP_OK) return st;
  return st2;
}

// The no-allocation search's status word on every device where it ran,
// read after waiting for `stream`: the first non-zero one is returned and
// cleared.
gap_status noalloc_status(hipStream_t stream) {
  gap_status first = GAP_OK;
  std::lock_guard<std::mutex> lk(g_na_mu);
  for (int dev = 0; dev < kNoAllocMaxDevices; ++dev) {
    if (!g_na_ptr[dev]) continue;
    GAP_HIP(hipSetDevice(dev));
    GAP_HIP(hipStreamSynchronize(stream));
    int code = 0;
    GAP_HIP(hipMemcpy(&code, g_na_ptr[dev], sizeof(int), hipMemcpyDeviceToHost));
    if (code != 0) {
      const int zero = 0;
      GAP_HIP(hipMemcpy(g_na_ptr[dev], &zero, sizeof(int), hipMemcpyHostToDevice));
      if (first == GAP_OK) first = code;
    }
  }
  return first;
}

}  // namespace gap
