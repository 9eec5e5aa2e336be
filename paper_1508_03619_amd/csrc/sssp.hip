// Single-source shortest paths (Section 2.1, "SSSP") by Delta-stepping (the
// method of the paper's reference code, Section 3), as one persistent kernel.
//
// Buckets of width delta are kept as two structures, as GPU Delta-stepping
// usually does: a near queue for the current bucket [bucket_end - delta,
// bucket_end) and one far pile for everything beyond it (the paper keeps
// thread-local bins plus one shared bin for the current range; here the
// near queue is that shared bin and the far pile stands for all later bins
// at once).  Phases, separated by grid barriers:
//   relax:   every item of the near queue relaxes its entries:
//            nd = dist[v] + w; atomicMin(dist[x], nd); a lowered x goes to
//            the next near queue if nd < bucket_end, else to the far pile;
//            repeated until the near queue stays empty (the bucket is
//            settled, since weights are positive);
//   findmin: the smallest live distance in the far pile;
//   compact: the bucket moves to the one holding that distance; far entries
//            inside it become near items, later ones move to the other far
//            pile, settled ones are dropped.
// The last workgroup to reach a barrier does the bookkeeping (counts,
// swaps, the next phase) before releasing the others.  A vertex is put in a
// near queue at most once per relax phase and in a far pile at most once
// per compaction (claim stamps), which bounds both.  A near item is a
// vertex and a slice of up to kSlice entries of its list, so a hub is
// relaxed by many lanes; four lanes share an item.  Claims of a workgroup
// round are staged in LDS and appended with one atomic per queue.

#include "runtime.h"

namespace gap {
namespace {

// The persistent grid: one workgroup of 1024 threads per CU (16 waves, as
// in the search kernel).  Every phase ends at a grid barrier, and its cost
// grows with the number of arriving workgroups: 4 workgroups of 256 per CU
// put a floor of about 27 us under every phase, and 1024-thread groups cut
// a search by 4-16 % (more where the bucket width is small and phases are
// many).  Cooperative grids must be resident as a whole: the occupancy
// query reported 7 workgroups of 256 per CU once, but with 7 the first
// barrier timed out, so the count is capped, never taken from the query.
#ifndef GAP_SSSP_BLOCKS_PER_CU
#define GAP_SSSP_BLOCKS_PER_CU 1
#endif
#ifndef GAP_SSSP_BLOCK
#define GAP_SSSP_BLOCK 1024
#endif
constexpr int kSpBlock = GAP_SSSP_BLOCK;
constexpr int kSlice = 16;      // list entries per near item
constexpr int kItemLanes = 4;   // lanes per item (kSlice / kItemLanes entries each)
constexpr uint32_t kInf = 0xFFFFFFFFu;

enum Phase : unsigned int { kRelax = 0, kFindMin = 1, kCompact = 2, kDone = 3 };

// Written by the last arriver of each barrier, read by everyone after it.
struct alignas(128) SpState {
  unsigned int phase;
  unsigned int cur;         // near queue being read (0/1)
  unsigned int ncur;        // its items
  unsigned int fcur;        // far pile being filled / read (0/1)
  unsigned int nfar;        // entries of far[fcur] (findmin, compact)
  unsigned int bucket_end;  // current bucket is [bucket_end - delta, bucket_end)
  unsigned int next_end;    // bucket after a compaction
  unsigned int stamp;       // near claims of the running phase use this value (new per phase)
  unsigned int epoch;       // far claims use this value
  unsigned int iters;       // relax phases run (statistics)
};

struct alignas(128) SpCounter {
  unsigned int v;
};

struct SpCtl {
  SpState st;
  SpCounter qtail[2];  // items appended to near queue 0 / 1
  SpCounter ftail[2];  // entries appended to far pile 0 / 1
  SpCounter minfar;    // findmin reduction
};

struct SpArgs {
  int64_t n;
  const int64_t *rp;
  const int32_t *col;
  const int32_t *wt;  // NULL: every weight is 1
  uint32_t *dist;
  uint32_t *near_stamp;
  uint32_t *far_stamp;
  int2 *q[2];
  int32_t *far[2];
  SpCtl *sc;
  Ctl *ctl;
  int *sticky;  // the stream's sticky status word
  int32_t source;
  uint32_t delta;
};

__device__ inline uint32_t items_of(int64_t deg) {
  return (uint32_t)((deg + kSlice - 1) / kSlice);
}

// Claim of x for the running phase (a near queue) or epoch (a far pile):
// true for exactly one caller.
__device__ inline bool claim(uint32_t *stamps, int32_t x, uint32_t stamp) {
  // a plain read first: most repeat claims in a phase stop here without an
  // atomic (atomics are carried out at the memory side)
  if (stamps[x] >= stamp) return false;
  return atomicMax(&stamps[x], stamp) < stamp;
}

// Claims of one workgroup round, staged in LDS and appended with one
// atomic per queue (same-address atomics are carried out one at a time at
// the memory side, so one per lane or per wave would serialise).
constexpr int kStage = kSpBlock * (kSlice / kItemLanes);  // at most one claim per lane and round
struct Stage {
  int32_t near_v[kStage];
  uint32_t near_ni[kStage];   // items of each near claim, then their offsets
  int32_t far_v[kStage];
  uint32_t nn, nf, nitems;
  uint32_t near_base, far_base;
};

__device__ inline void stage_claim(Stage &st, int32_t x, uint32_t ni, bool to_near, bool to_far) {
  if (to_near && ni > 0) {
    const uint32_t k = atomicAdd(&st.nn, 1u);
    st.near_v[k] = x;
    st.near_ni[k] = ni;
  }
  if (to_far) st.far_v[atomicAdd(&st.nf, 1u)] = x;
}

// Appends the staged claims (whole workgroup; ends with the stage empty).
__device__ inline void stage_flush(Stage &st, int2 *q, unsigned int *qtail, int32_t *far,
                                   unsigned int *ftail) {
  __syncthreads();
  const uint32_t nn = st.nn, nf = st.nf;
  // item offsets of the near claims: exclusive scan, four claims per thread
  constexpr int kPer = kStage / kSpBlock;
  __shared__ uint32_t wave_total[kSpBlock / kWave];
  uint32_t loc[kPer];
  uint32_t sum = 0;
#pragma unroll
  for (int j = 0; j < kPer; ++j) {
    const uint32_t k = threadIdx.x * kPer + j;
    loc[j] = k < nn ? st.near_ni[k] : 0u;
    sum += loc[j];
  }
  uint32_t wtot = 0;
  uint32_t off = wave_excl_scan_u32(sum, wtot);
  if (lane_id() == 0) wave_total[threadIdx.x / kWave] = wtot;
  __syncthreads();
  uint32_t total = 0;
  for (int w = 0; w < kSpBlock / kWave; ++w) {
    if (w < (int)(threadIdx.x / kWave)) off += wave_total[w];
    total += wave_total[w];
  }
#pragma unroll
  for (int j = 0; j < kPer; ++j) {
    const uint32_t k = threadIdx.x * kPer + j;
    if (k < nn) st.near_ni[k] = off;
    off += loc[j];
  }
  if (threadIdx.x == 0) {
    st.nitems = total;
    st.near_base = total ? atomicAdd(qtail, total) : 0u;
    st.far_base = nf ? atomicAdd(ftail, nf) : 0u;
  }
  __syncthreads();
  for (uint32_t k = threadIdx.x; k < nf; k += kSpBlock) far[st.far_base + k] = st.far_v[k];
  // item j of the round belongs to the claim whose offset range holds it
  for (uint32_t j = threadIdx.x; j < total; j += kSpBlock) {
    uint32_t lo = 0, hi = nn;  // last k with near_ni[k] <= j
    while (hi - lo > 1) {
      const uint32_t mid = (lo + hi) / 2;
      if (st.near_ni[mid] <= j)
        lo = mid;
      else
        hi = mid;
    }
    q[st.near_base + j] = make_int2(st.near_v[lo], (int)(j - st.near_ni[lo]));
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    st.nn = 0;
    st.nf = 0;
  }
  __syncthreads();
}

struct SpDecide {
  SpCtl *sc;
  uint32_t delta;
  __device__ BarrierDecision operator()(Ctl *, const Totals &) const {
    SpState s;
    s.phase = ld_agent(&sc->st.phase);
    s.cur = ld_agent(&sc->st.cur);
    s.fcur = ld_agent(&sc->st.fcur);
    s.bucket_end = ld_agent(&sc->st.bucket_end);
    s.next_end = ld_agent(&sc->st.next_end);
    s.stamp = ld_agent(&sc->st.stamp);
    s.epoch = ld_agent(&sc->st.epoch);
    s.iters = ld_agent(&sc->st.iters);
    s.ncur = 0;
    s.nfar = 0;
    if (s.phase == kFindMin) {
      const uint32_t mf = ld_agent(&sc->minfar.v);
      if (mf == kInf) {
        s.phase = kDone;
      } else {
        const uint64_t e = ((uint64_t)mf / delta + 1) * (uint64_t)delta;
        s.next_end = e > (uint64_t)kInf ? kInf : (uint32_t)e;
        s.phase = kCompact;
        s.nfar = ld_agent(&sc->ftail[s.fcur].v);
        s.stamp += 1;
        s.epoch += 1;
      }
    } else {
      // after a relax or a compaction: the other near queue is next
      const uint32_t nxt = s.cur ^ 1u;
      const uint32_t nn = ld_agent(&sc->qtail[nxt].v);
      st_agent(&sc->qtail[s.cur].v, 0u);  // the queue just read is free again
      if (s.phase == kCompact) {
        st_agent(&sc->ftail[s.fcur].v, 0u);  // the pile just read is free again
        s.fcur ^= 1u;
        s.bucket_end = s.next_end;
      }
      s.cur = nxt;
      if (nn > 0) {
        s.phase = kRelax;
        s.ncur = nn;
        s.stamp += 1;
        s.iters += 1;
      } else {
        const uint32_t nf = ld_agent(&sc->ftail[s.fcur].v);
        if (nf == 0) {
          s.phase = kDone;
        } else {
          s.phase = kFindMin;
          s.nfar = nf;
          st_agent(&sc->minfar.v, kInf);
        }
      }
    }
    st_agent(&sc->st.phase, s.phase);
    st_agent(&sc->st.cur, s.cur);
    st_agent(&sc->st.ncur, s.ncur);
    st_agent(&sc->st.fcur, s.fcur);
    st_agent(&sc->st.nfar, s.nfar);
    st_agent(&sc->st.bucket_end, s.bucket_end);
    st_agent(&sc->st.next_end, s.next_end);
    st_agent(&sc->st.stamp, s.stamp);
    st_agent(&sc->st.epoch, s.epoch);
    st_agent(&sc->st.iters, s.iters);
    return {0, -1};
  }
};

__device__ __forceinline__ void sssp_body(const SpArgs &a) {
  const unsigned int nblocks = gridDim.x;
  const int64_t tid = blockIdx.x * (int64_t)kSpBlock + threadIdx.x;
  const int64_t nthreads = (int64_t)nblocks * kSpBlock;
  const int lane = lane_id();
  const SpDecide decide{a.sc, a.delta};
  int flag = 0;
  __shared__ Stage sg;
  if (threadIdx.x == 0) {
    sg.nn = 0;
    sg.nf = 0;
  }
  for (int64_t v = tid; v < a.n; v += nthreads) {
    a.dist[v] = kInf;
    a.near_stamp[v] = 0;
    a.far_stamp[v] = 0;
  }
  if (!grid_sync(a.ctl, nblocks, Totals{}, -1, 0)) return;
  // the source's items go to near queue 1 (the decide below makes it current)
  if (blockIdx.x == 0) {
    const int32_t s = a.source;
    const int64_t deg = a.rp[s + 1] - a.rp[s];
    const uint32_t ni = items_of(deg);
    for (uint32_t k = threadIdx.x; k < ni; k += kSpBlock) a.q[1][k] = make_int2(s, (int)k);
    if (threadIdx.x == 0) {
      a.dist[s] = 0;
      a.near_stamp[s] = 1;
      st_agent(&a.sc->qtail[1].v, ni);
    }
  }
  if (!grid_sync_x(a.ctl, main_barrier(a.ctl), nblocks, Totals{}, -1, 0, decide, flag)) return;

  for (;;) {
    const unsigned int phase = ld_agent(&a.sc->st.phase);
    if (phase == kDone) break;
    const unsigned int cur = ld_agent(&a.sc->st.cur);
    const unsigned int fcur = ld_agent(&a.sc->st.fcur);
    const uint32_t bend = ld_agent(&a.sc->st.bucket_end);
    const uint32_t stamp = ld_agent(&a.sc->st.stamp);
    const uint32_t epoch = ld_agent(&a.sc->st.epoch);
    int2 *qn = a.q[cur ^ 1u];
    unsigned int *qn_tail = &a.sc->qtail[cur ^ 1u].v;
    if (phase == kRelax) {
      const uint32_t ncur = ld_agent(&a.sc->st.ncur);
      const int2 *qc = a.q[cur];
      int32_t *fp = a.far[fcur];
      unsigned int *fp_tail = &a.sc->ftail[fcur].v;
      constexpr int kItemsPerRound = kSpBlock / kItemLanes;
      const int gl = lane & (kItemLanes - 1);
      // every workgroup runs the same number of rounds (barriers inside)
      for (int64_t base = (int64_t)blockIdx.x * kItemsPerRound; base < (int64_t)ncur;
           base += (int64_t)nblocks * kItemsPerRound) {
        const int64_t i = base + threadIdx.x / kItemLanes;
        int32_t v = -1;
        int64_t beg = 0, end = 0;
        uint32_t du = kInf;
        if (i < (int64_t)ncur) {
          const int2 it = qc[i];
          v = it.x;
          const int64_t rb = a.rp[v];
          beg = rb + (int64_t)it.y * kSlice;
          end = min(beg + (int64_t)kSlice, a.rp[v + 1]);
          du = a.dist[v];
        }
#pragma unroll
        for (int r = 0; r < kSlice / kItemLanes; ++r) {
          const int64_t e = beg + gl + r * kItemLanes;
          int32_t x = -1;
          uint32_t nd = kInf;
          if (e < end) {
            x = a.col[e];
            nd = du + (a.wt ? (uint32_t)a.wt[e] : 1u);
          }
          if (x >= 0 && nd < a.dist[x]) {
            const uint32_t old = atomicMin(&a.dist[x], nd);
            if (nd < old) {
              if (nd < bend) {
                if (claim(a.near_stamp, x, stamp))
                  stage_claim(sg, x, items_of(a.rp[x + 1] - a.rp[x]), true, false);
              } else if (claim(a.far_stamp, x, epoch)) {
                stage_claim(sg, x, 0, false, true);
              }
            }
          }
        }
        stage_flush(sg, qn, qn_tail, fp, fp_tail);
      }
    } else if (phase == kFindMin) {
      const uint32_t nf = ld_agent(&a.sc->st.nfar);
      const int32_t *fp = a.far[fcur];
      uint32_t m = kInf;
      for (int64_t i = tid; i < (int64_t)nf; i += nthreads) {
        const uint32_t dx = a.dist[fp[i]];
        if (dx >= bend && dx < m) m = dx;  // entries below bucket_end are settled
      }
      for (int o = 32; o >= 1; o >>= 1) m = min(m, (uint32_t)__shfl_xor(m, o, kWave));
      // skip the atomic unless it can lower the published minimum
      if (lane == 0 && m != kInf && m < ld_agent(&a.sc->minfar.v)) atomicMin(&a.sc->minfar.v, m);
    } else {  // kCompact
      const uint32_t nf = ld_agent(&a.sc->st.nfar);
      const uint32_t nend = ld_agent(&a.sc->st.next_end);
      const int32_t *fp = a.far[fcur];
      int32_t *fo = a.far[fcur ^ 1u];
      unsigned int *fo_tail = &a.sc->ftail[fcur ^ 1u].v;
      for (int64_t base = (int64_t)blockIdx.x * kSpBlock; base < (int64_t)nf;
           base += (int64_t)nblocks * kSpBlock) {
        const int64_t i = base + threadIdx.x;
        if (i < (int64_t)nf) {
          const int32_t x = fp[i];
          const uint32_t dx = a.dist[x];
          if (dx >= bend) {  // below: settled in an earlier bucket
            if (dx < nend) {
              if (claim(a.near_stamp, x, stamp))
                stage_claim(sg, x, items_of(a.rp[x + 1] - a.rp[x]), true, false);
            } else if (claim(a.far_stamp, x, epoch)) {
              stage_claim(sg, x, 0, false, true);
            }
          }
        }
        stage_flush(sg, qn, qn_tail, fo, fo_tail);
      }
    }
    if (!grid_sync_x(a.ctl, main_barrier(a.ctl), nblocks, Totals{}, -1, 0, decide, flag)) return;
  }
}

__global__ __launch_bounds__(kSpBlock) void k_sssp(SpArgs a) {
  sssp_body(a);
  note_error(a.sticky, a.ctl);
}

// Control state before a search: the first barrier's bookkeeping treats
// the source's items (near queue 1) like the output of a compaction into
// the first bucket [0, delta).
__global__ void k_sp_init(SpCtl *sc, uint32_t delta) {
  SpCtl c{};
  c.st.phase = kCompact;
  c.st.cur = 0;
  c.st.fcur = 1;
  c.st.next_end = delta;
  c.st.stamp = 1;  // the source's claim
  c.st.epoch = 1;
  *sc = c;
}

template <class T>
T *carve(char *&p, size_t count) {
  T *r = reinterpret_cast<T *>(p);
  p += (sizeof(T) * count + 255) & ~(size_t)255;
  return r;
}

}  // namespace

gap_status run_sssp(const gap_graph *g, int32_t source, uint32_t *dist, uint32_t delta,
                    hipStream_t stream, int32_t *phases) {
  const DeviceInfo *di = nullptr;
  gap_status st = device_info(g->device, &di);
  if (st != GAP_OK) return st;
  Workspace *ws = workspace_for(g->device, stream);
  if (!ws) {
    set_error("gap_sssp: no workspace for the stream");
    return GAP_ENOMEM;
  }
  const int64_t n = g->n;
  // near items of one phase: at most one claim per vertex, items_of(deg) each
  const int64_t cap_items = g->nnz / kSlice + n + 1;
  const size_t bytes = 8 * 256 + sizeof(uint32_t) * 2 * (size_t)n + sizeof(int2) * 2 * (size_t)cap_items +
                       sizeof(int32_t) * 2 * (size_t)n + sizeof(SpCtl) + sizeof(Ctl);
  st = workspace_reserve_sssp(ws, bytes);
  if (st != GAP_OK) return st;
  char *p = reinterpret_cast<char *>(ws->sp_buf);
  SpArgs a{};
  a.n = n;
  a.rp = g->row_ptr;
  a.col = g->col;
  a.wt = g->wt;
  a.dist = dist;
  a.near_stamp = carve<uint32_t>(p, n);
  a.far_stamp = carve<uint32_t>(p, n);
  a.q[0] = carve<int2>(p, cap_items);
  a.q[1] = carve<int2>(p, cap_items);
  a.far[0] = carve<int32_t>(p, n);
  a.far[1] = carve<int32_t>(p, n);
  a.sc = carve<SpCtl>(p, 1);
  a.ctl = carve<Ctl>(p, 1);
  a.sticky = ws->sticky;
  a.source = source;
  a.delta = delta;
  k_sp_init<<<1, 1, 0, stream>>>(a.sc, delta);
  GAP_HIP(hipGetLastError());
  GAP_HIP(hipMemsetAsync(a.ctl, 0, sizeof(Ctl), stream));
  auto kern = k_sssp;
  int per_cu = 0;
  GAP_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, kSpBlock, 0));
  if (per_cu < 1) {
    set_error("shortest-path kernel does not fit on a compute unit");
    return GAP_EDEVICE;
  }
  per_cu = std::min(per_cu, GAP_SSSP_BLOCKS_PER_CU);
  void *kargs[] = {&a};
  CoopOrder order;
  st = coop_begin(g->device, stream, 1, &order);
  if (st != GAP_OK) return st;
  st = launch_resident((const void *)kern, per_cu * di->cus, kSpBlock, 0, kargs, 1,
                       params_current().coop_launch, di, stream, nullptr);
  gap_status st2 = coop_end(g->device, stream, &order);
  if (st != GAP_OK) return st;
  if (st2 != GAP_OK) return st2;
  if (phases) {
    GAP_HIP(hipMemcpyAsync(ws->sp_host, &a.sc->st.iters, sizeof(unsigned int),
                           hipMemcpyDeviceToHost, stream));
    GAP_HIP(hipMemcpyAsync(reinterpret_cast<char *>(ws->sp_host) + 4, &a.ctl->err, sizeof(int),
                           hipMemcpyDeviceToHost, stream));
    GAP_HIP(hipStreamSynchronize(stream));
    const int err = reinterpret_cast<int *>(ws->sp_host)[1];
    if (err != 0) {
      set_error("device-side wait timed out (grid barrier)");
      return err;
    }
    *phases = (int32_t) reinterpret_cast<unsigned int *>(ws->sp_host)[0];
  }
  return GAP_OK;
}

}  // namespace gap
