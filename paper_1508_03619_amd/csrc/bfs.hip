// Single-source direction-optimizing BFS on gfx950: kernels and the two
// level schedules (persistent cooperative kernel; one launch per step).
#include <algorithm>

#include "bfs_kernels.h"
#include "runtime.h"

namespace gap {

struct PersistArgs {
  DevGraph g;
  int32_t *parent;
  int32_t *depth;
  int32_t source;
  int32_t *q0, *q1;
  int2 *c0, *c1;
  uint64_t *fa, *fb, *vbm;
  Ctl *ctl;
  Params p;
  DevLevelRec *recs;
  int32_t max_recs;
};

__device__ inline unsigned long long ld_agent(const unsigned long long *p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// The whole search in one cooperative launch.  Every workgroup runs the same
// level loop and takes the same decisions from the same device counters;
// levels are separated by grid barriers.
template <int BLOCK, bool STATS>
__global__ __launch_bounds__(BLOCK) void k_bfs_persistent(PersistArgs a) {
  const int64_t nthreads = (int64_t)gridDim.x * BLOCK;
  const int64_t tid = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
  const int64_t nwaves = nthreads / kWave;
  const int64_t gwave = tid / kWave;
  const unsigned int nblocks = gridDim.x;

  init_vertices(a.g, a.parent, a.depth, a.source, tid, nthreads);
  if (tid == 0) init_source(a.g, a.source, a.p.hub, a.p.chunk, a.q0, a.c0, a.ctl);
  if (!grid_barrier(a.ctl, nblocks)) return;

  int32_t d = 0, dir = kTopDown;
  bool have_bm = false;
  int64_t mu = a.g.nnz, nf_prev = 0;
  int32_t *qin = a.q0, *qout = a.q1;
  int2 *cin = a.c0, *cout = a.c1;
  uint64_t *fb = a.fa, *nb = a.fb;
  for (;;) {
    LevelCounters *prev = &a.ctl->cnt[(d + 2) % 3];
    const int64_t nq = (int64_t)ld_agent(&prev->nq);
    const int64_t nc = (int64_t)ld_agent(&prev->nc);
    const int64_t nv = (int64_t)ld_agent(&prev->nv);
    const int64_t mf = (int64_t)ld_agent(&prev->mf);
    if (STATS && tid == 0 && d > 0 && d - 1 < a.max_recs) {
      a.recs[d - 1].claimed = (unsigned long long)nv;
      a.recs[d - 1].scanned = ld_agent(&prev->scanned);
      a.recs[d - 1].unvisited = ld_agent(&prev->unvisited);
    }
    if (nv == 0) break;
    if (d > a.g.n) {  // more levels than vertices: inconsistent counters
      if (tid == 0) atomicExch(&a.ctl->err, (int)GAP_EINTERNAL);
      return;
    }
    mu -= mf;
    const int32_t ndir = decide_direction(dir, nv, mf, mu, nf_prev, a.g.n, a.p, d);
    if (ndir == kBottomUp && !(dir == kBottomUp && have_bm)) {
      convert_to_bitmaps(a.g, a.parent, a.depth, d, fb, a.vbm, gwave, nwaves);
      if (!grid_barrier(a.ctl, nblocks)) return;
      have_bm = true;
    }
    if (ndir == kTopDown) have_bm = false;
    dir = ndir;
    if (tid == 0) {
      a.ctl->cnt[(d + 1) % 3] = LevelCounters();
      if (STATS && d < a.max_recs) {
        DevLevelRec r = {};
        r.level = d;
        r.direction = dir;
        r.frontier = (unsigned long long)nv;
        r.frontier_edges = (unsigned long long)mf;
        a.recs[d] = r;
      }
    }
    StepArgs s{a.g, a.parent, a.depth, qin, cin, nq, nc, qout, cout, fb, a.vbm, nb,
               &a.ctl->cnt[d % 3], d, a.p.hub, a.p.chunk};
    if (dir == kTopDown)
      td_step<STATS>(s, gwave, nwaves);
    else
      bu_step<STATS>(s, gwave, nwaves);
    if (!grid_barrier(a.ctl, nblocks)) return;
    swap_ptr(qin, qout);
    swap_ptr(cin, cout);
    if (dir == kBottomUp) swap_ptr(fb, nb);
    nf_prev = nv;
    ++d;
  }
  fixup_parents(a.g.n, a.parent, tid, nthreads);
  if (tid == 0) a.ctl->levels = d;
}

// ---- one launch per step ----------------------------------------------------

struct InitArgs {
  DevGraph g;
  int32_t *parent, *depth;
  int32_t source, hub, chunk;
  int32_t *q0;
  int2 *c0;
  Ctl *ctl;
};

__global__ __launch_bounds__(256) void k_init(InitArgs a) {
  const int64_t nthreads = (int64_t)gridDim.x * blockDim.x;
  const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  init_vertices(a.g, a.parent, a.depth, a.source, tid, nthreads);
  if (tid == 0) init_source(a.g, a.source, a.hub, a.chunk, a.q0, a.c0, a.ctl);
}

__global__ __launch_bounds__(256) void k_convert(DevGraph g, const int32_t *parent,
                                                 const int32_t *depth, int32_t d, uint64_t *fbm,
                                                 uint64_t *vbm) {
  const int64_t nwaves = (int64_t)gridDim.x * blockDim.x / kWave;
  const int64_t gwave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
  convert_to_bitmaps(g, parent, depth, d, fbm, vbm, gwave, nwaves);
}

template <bool STATS>
__global__ __launch_bounds__(256) void k_td(StepArgs a) {
  const int64_t nwaves = (int64_t)gridDim.x * blockDim.x / kWave;
  const int64_t gwave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
  td_step<STATS>(a, gwave, nwaves);
}

template <bool STATS>
__global__ __launch_bounds__(256) void k_bu(StepArgs a) {
  const int64_t nwaves = (int64_t)gridDim.x * blockDim.x / kWave;
  const int64_t gwave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
  bu_step<STATS>(a, gwave, nwaves);
}

__global__ __launch_bounds__(256) void k_fixup(int64_t n, int32_t *parent) {
  const int64_t nthreads = (int64_t)gridDim.x * blockDim.x;
  const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  fixup_parents(n, parent, tid, nthreads);
}

// ---- host side ----------------------------------------------------------------

static int grid_for_waves(int64_t waves, int block) {
  const int64_t wpb = block / kWave;
  int64_t b = (waves + wpb - 1) / wpb;
  if (b < 1) b = 1;
  if (b > 65536) b = 65536;
  return (int)b;
}

template <int BLOCK, bool STATS>
static gap_status launch_persistent(const PersistArgs &a, const DeviceInfo *di, int blocks_per_cu,
                                    hipStream_t stream) {
  auto kern = k_bfs_persistent<BLOCK, STATS>;
  int per_cu = 0;
  GAP_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, BLOCK, 0));
  if (per_cu < 1) {
    set_error("persistent kernel does not fit on a compute unit");
    return GAP_EDEVICE;
  }
  if (blocks_per_cu > 0 && blocks_per_cu < per_cu) per_cu = blocks_per_cu;
  const int grid = per_cu * di->cus;
  PersistArgs args = a;
  void *kargs[] = {&args};
  GAP_HIP(hipLaunchCooperativeKernel((const void *)kern, dim3(grid), dim3(BLOCK), kargs, 0,
                                     stream));
  return GAP_OK;
}

template <bool STATS>
static gap_status dispatch_persistent(const PersistArgs &a, const DeviceInfo *di,
                                      const gap_params &p, hipStream_t stream) {
  switch (p.block) {
    case 256: return launch_persistent<256, STATS>(a, di, p.blocks_per_cu, stream);
    case 512: return launch_persistent<512, STATS>(a, di, p.blocks_per_cu, stream);
    default: return launch_persistent<1024, STATS>(a, di, p.blocks_per_cu, stream);
  }
}

static gap_status run_levels(const PersistArgs &a, bool stats, Workspace *ws, hipStream_t stream,
                             int32_t *levels_out, std::vector<DevLevelRec> *host_recs) {
  const int block = 256;
  const int64_t n = a.g.n;
  const int64_t nwords = (n + kWave - 1) / kWave;
  InitArgs ia{a.g, a.parent, a.depth, a.source, a.p.hub, a.p.chunk, a.q0, a.c0, a.ctl};
  k_init<<<grid_for_waves((n + kWave - 1) / kWave, block), block, 0, stream>>>(ia);
  GAP_HIP(hipGetLastError());
  int32_t d = 0, dir = kTopDown;
  bool have_bm = false;
  int64_t mu = a.g.nnz, nf_prev = 0;
  int32_t *qin = a.q0, *qout = a.q1;
  int2 *cin = a.c0, *cout = a.c1;
  uint64_t *fb = a.fa, *nb = a.fb;
  for (;;) {
    GAP_HIP(hipMemcpyAsync(ws->h_cnt, &a.ctl->cnt[(d + 2) % 3], sizeof(LevelCounters),
                           hipMemcpyDeviceToHost, stream));
    GAP_HIP(hipStreamSynchronize(stream));
    const LevelCounters c = *ws->h_cnt;
    if (stats && d > 0 && d - 1 < (int32_t)host_recs->size()) {
      DevLevelRec &h = (*host_recs)[d - 1];
      h.claimed = c.nv;
      h.scanned = c.scanned;
      h.unvisited = c.unvisited;
    }
    const int64_t nv = (int64_t)c.nv, mf = (int64_t)c.mf;
    if (nv == 0) break;
    if (d > n) {
      set_error("search ran more levels than vertices (inconsistent counters)");
      return GAP_EINTERNAL;
    }
    mu -= mf;
    const int32_t ndir = decide_direction(dir, nv, mf, mu, nf_prev, n, a.p, d);
    if (ndir == kBottomUp && !(dir == kBottomUp && have_bm)) {
      k_convert<<<grid_for_waves(nwords, block), block, 0, stream>>>(a.g, a.parent, a.depth, d, fb,
                                                                     a.vbm);
      GAP_HIP(hipGetLastError());
      have_bm = true;
    }
    if (ndir == kTopDown) have_bm = false;
    dir = ndir;
    GAP_HIP(hipMemsetAsync(&a.ctl->cnt[(d + 1) % 3], 0, sizeof(LevelCounters), stream));
    if (stats && d < a.max_recs) {
      DevLevelRec h = {};
      h.level = d;
      h.direction = dir;
      h.frontier = (unsigned long long)nv;
      h.frontier_edges = (unsigned long long)mf;
      host_recs->push_back(h);
    }
    StepArgs s{a.g, a.parent, a.depth, qin, cin, (int64_t)c.nq, (int64_t)c.nc, qout, cout, fb,
               a.vbm, nb, &a.ctl->cnt[d % 3], d, a.p.hub, a.p.chunk};
    if (dir == kTopDown) {
      const int64_t waves = std::max<int64_t>((int64_t)c.nc, ((int64_t)c.nq + kWave - 1) / kWave);
      if (stats)
        k_td<true><<<grid_for_waves(waves, block), block, 0, stream>>>(s);
      else
        k_td<false><<<grid_for_waves(waves, block), block, 0, stream>>>(s);
    } else {
      if (stats)
        k_bu<true><<<grid_for_waves(nwords, block), block, 0, stream>>>(s);
      else
        k_bu<false><<<grid_for_waves(nwords, block), block, 0, stream>>>(s);
    }
    GAP_HIP(hipGetLastError());
    swap_ptr(qin, qout);
    swap_ptr(cin, cout);
    if (dir == kBottomUp) swap_ptr(fb, nb);
    nf_prev = nv;
    ++d;
  }
  k_fixup<<<grid_for_waves(nwords, block), block, 0, stream>>>(n, a.parent);
  GAP_HIP(hipGetLastError());
  *levels_out = d;
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
  PersistArgs a{};
  a.g = DevGraph{g->row_ptr, g->col, g->n, g->nnz};
  a.parent = parent;
  a.depth = depth ? depth : ws->depth_scratch;
  a.source = source;
  a.q0 = ws->q[0];
  a.q1 = ws->q[1];
  a.c0 = ws->cq[0];
  a.c1 = ws->cq[1];
  a.fa = ws->bm[0];
  a.fb = ws->bm[1];
  a.vbm = ws->bm[2];
  a.ctl = ws->ctl;
  a.p = Params{p.alpha, p.beta, p.direction, p.hub_degree, p.chunk_edges};
  a.recs = want_stats ? ws->recs : nullptr;
  a.max_recs = want_stats ? max_levels : 0;

  int32_t levels = 0;
  std::vector<DevLevelRec> recs;
  const bool host_loop = p.mode == GAP_MODE_LEVELS || p.mode == GAP_MODE_GRAPH;
  if (host_loop) {
    st = run_levels(a, want_stats, ws, stream, &levels, &recs);
    if (st != GAP_OK) return st;
  } else {
    GAP_HIP(hipMemsetAsync(ws->ctl, 0, sizeof(Ctl), stream));
    st = want_stats ? dispatch_persistent<true>(a, di, p, stream)
                    : dispatch_persistent<false>(a, di, p, stream);
    if (st != GAP_OK) return st;
  }
  if (want_stats) {
    GAP_HIP(hipStreamSynchronize(stream));
    if (!host_loop) {
      Ctl h;
      GAP_HIP(hipMemcpy(&h, ws->ctl, sizeof(Ctl), hipMemcpyDeviceToHost));
      if (h.err != 0) {
        set_error(h.err == GAP_ETIMEOUT ? "device-side wait timed out (grid barrier)"
                                         : "search ran more levels than vertices");
        return h.err;
      }
      levels = h.levels;
      recs.resize((size_t)std::min(levels, max_levels));
      if (!recs.empty())
        GAP_HIP(hipMemcpy(recs.data(), ws->recs, recs.size() * sizeof(DevLevelRec),
                          hipMemcpyDeviceToHost));
    }
    for (size_t i = 0; i < recs.size(); ++i) {
      stats[i].level = recs[i].level;
      stats[i].direction = recs[i].direction;
      stats[i].frontier = (int64_t)recs[i].frontier;
      stats[i].frontier_edges = (int64_t)recs[i].frontier_edges;
      stats[i].claimed = (int64_t)recs[i].claimed;
      stats[i].scanned = (int64_t)recs[i].scanned;
      stats[i].unvisited = (int64_t)recs[i].unvisited;
    }
    if (num_levels) *num_levels = levels;
  } else if (num_levels) {
    *num_levels = host_loop ? levels : -1;
  }
  return GAP_OK;
}

}  // namespace gap
