// Continuous batching of single-source searches on one resident graph.
//
// One persistent launch holds up to 64 searches as the bits of a 64-bit word
// per vertex (visited V, frontier F, next frontier N), as the batched search
// does, and takes new searches while it runs:
//  * the host writes a request (query id, source, output arrays) into a ring
//    in pinned host memory and advances `posted`;
//  * after every level's step, the last workgroup to reach the barrier moves
//    waiting requests into free lanes: the lane's bit is set in N at the
//    source, so the lane's frontier at the next level is {source}, and the
//    lane's depths count from that level (depth = level - joining level);
//  * the next level's dense advance pass writes the new lane's outputs (-1
//    everywhere, the source as its own parent at depth 0) before any record
//    of that lane is written;
//  * after an advance, a lane whose frontier is empty has finished: its query
//    id goes to the host's completion ring, and the next advance clears its
//    visited bits, so the lane can take a new search at once.
// Lanes are independent: a bit is set only by its own lane's search (claims
// and gathers work bit by bit), so every lane's result is exactly the
// single-source result for its source (Section 2.1), whichever searches run
// beside it and whenever it joined.
// A launch stops taking requests once it has run for serve_window_us, or
// when it holds no search; it then finishes its lanes and exits.  The host
// launches again when it posts a request and finds no launch taking requests
// (`accepting`): the launch gives up `accepting` before its last look at
// `posted`, and the host posts before it looks at `accepting`, so one of the
// two always sees the other and no request is stranded.
#include <algorithm>
#include <atomic>
#include <cstring>
#include <mutex>

#include "bfs_kernels.h"
#include "runtime.h"

namespace gap {

constexpr int kSrvBlock = 1024;
constexpr int kSrvLanes = 64;
constexpr int kSrvRing = 256;
constexpr int kSrvBuFlag = 1 << 30;  // chunk item of a hub that some lane still needs (bottom-up)

// One request, written by the host.
struct ServeReq {
  long long qid;
  long long source;  // in the low 32 bits
  int32_t *parent;
  int32_t *depth;  // may be NULL
};

// Shared between the host and the launches (pinned, coherent host memory).
// Counters only grow; the host writes `posted` and req[], a launch writes
// `taken`, `completed`, done[] and `accepting`.
struct ServeMailbox {
  unsigned long long posted;
  unsigned long long pad0[7];
  unsigned long long taken;
  unsigned long long completed;
  unsigned long long pad1[6];
  unsigned int accepting;  // generation of the launch taking requests, 0 = none
  int err;                 // first device-side failure of a launch
  unsigned int pad2[14];
  ServeReq req[kSrvRing];
  long long done[kSrvRing];  // query id of completion record k at done[k % kSrvRing]
};

struct ServeLane {
  int32_t *parent;
  int32_t *depth;
  long long qid;
  int32_t source;
  int32_t inj;  // level at which the lane's frontier is {source}
};

struct alignas(128) SrvTot {
  unsigned long long nf;   // vertices with a frontier bit
  unsigned long long mf;   // their degrees
  unsigned long long mu;   // degrees of vertices some searching lane has not reached
  unsigned long long lor;  // lanes with a frontier bit
};

// Device-resident state of one launch (cleared before the launch).
struct ServeCtl {
  Ctl base;
  SrvTot tot[2];             // level parity
  unsigned long long active;  // lanes searching
  unsigned long long fresh;   // lanes whose outputs the next advance writes
  unsigned long long clear;   // lanes whose visited bits the next advance clears
  unsigned long long t0;      // real-time clock at the first boundary
  long long nf_prev;
  int dir;
  int stopped;  // this launch takes no more requests
  ServeLane lane[kSrvLanes];
};

struct SrvArgs {
  const int64_t *row_ptr;
  const int32_t *col;
  int64_t n;
  uint64_t *V, *B0, *B1;
  Queues Q;
  ServeCtl *ctl;
  ServeMailbox *mb;  // device address of the pinned mailbox
  int *sticky;
  Params p;
  unsigned int gen;
  unsigned long long window;  // real-time ticks after which no request is taken
};

__device__ inline unsigned long long ld_sys(const void *p) {
  return __hip_atomic_load(reinterpret_cast<const unsigned long long *>(p), __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_SYSTEM);
}
__device__ inline void st_sys(void *p, unsigned long long v) {
  __hip_atomic_store(reinterpret_cast<unsigned long long *>(p), v, __ATOMIC_RELAXED,
                     __HIP_MEMORY_SCOPE_SYSTEM);
}

// Moves waiting requests into free lanes (lanes joining after level d start
// at level d + 1).  One thread.
__device__ inline void srv_take(const SrvArgs &a, int32_t d, uint64_t *N, unsigned long long &act,
                                unsigned long long &fresh, unsigned long long &taken) {
  ServeMailbox *mb = a.mb;
  const unsigned long long posted = __hip_atomic_load(&mb->posted, __ATOMIC_ACQUIRE,
                                                      __HIP_MEMORY_SCOPE_SYSTEM);
  while (taken < posted && act != ~0ull) {
    const int i = __builtin_ctzll(~act);
    const ServeReq *r = &mb->req[taken % kSrvRing];
    ServeLane L;
    L.qid = (long long)ld_sys(&r->qid);
    L.source = (int32_t)(uint32_t)ld_sys(&r->source);
    L.parent = reinterpret_cast<int32_t *>(ld_sys(&r->parent));
    L.depth = reinterpret_cast<int32_t *>(ld_sys(&r->depth));
    L.inj = d + 1;
    a.ctl->lane[i] = L;
    atomicOr(reinterpret_cast<unsigned long long *>(&N[L.source]), 1ull << i);
    act |= 1ull << i;
    fresh |= 1ull << i;
    ++taken;
  }
}

// Boundary after a step (or before the first level, d = -1): takes requests
// into free lanes, and stops taking them once the window has passed or no
// lane is searching.  Flag 1: no lane is searching, every workgroup leaves.
struct SrvTake {
  const SrvArgs *a;
  int32_t d;
  uint64_t *N;
  __device__ BarrierDecision operator()(Ctl *, const Totals &) const {
    ServeCtl *c = a->ctl;
    ServeMailbox *mb = a->mb;
    unsigned long long act = ld_agent(&c->active);
    unsigned long long fresh = 0;
    const unsigned long long now = rt_clock();
    unsigned long long t0 = ld_agent(&c->t0);
    if (t0 == 0ull) {
      t0 = now;
      st_agent(&c->t0, t0);
    }
    if (__hip_atomic_load(&c->stopped, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0) {
      unsigned long long taken = ld_sys(&mb->taken);
      const bool expired = now - t0 > a->window;
      if (!expired) srv_take(*a, d, N, act, fresh, taken);
      if (expired || act == 0ull) {
        // give up `accepting`; a request posted after this finds it 0 (the
        // host launches again) or is seen by the look below
        unsigned int expected = a->gen;
        __hip_atomic_compare_exchange_strong(&mb->accepting, &expected, 0u, __ATOMIC_SEQ_CST,
                                             __ATOMIC_SEQ_CST, __HIP_MEMORY_SCOPE_SYSTEM);
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "");
        __hip_atomic_store(&c->stopped, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (!expired) {
          // about to leave with no search: one last look at `posted`
          srv_take(*a, d, N, act, fresh, taken);
          if (act != 0ull) {  // it found work: keep taking, unless the host has launched again
            expected = 0u;
            if (__hip_atomic_compare_exchange_strong(&mb->accepting, &expected, a->gen,
                                                     __ATOMIC_SEQ_CST, __ATOMIC_SEQ_CST,
                                                     __HIP_MEMORY_SCOPE_SYSTEM))
              __hip_atomic_store(&c->stopped, 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          }
        }
      }
      __hip_atomic_store(&mb->taken, taken, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
    }
    st_agent(&c->active, act);
    st_agent(&c->fresh, fresh);
    return {act == 0ull ? 1 : 0, -1};
  }
};

// Boundary after an advance: lanes without a frontier have finished (their
// completion records go to the host); the direction of this level's step.
struct SrvRetire {
  const SrvArgs *a;
  int32_t d;
  __device__ BarrierDecision operator()(Ctl *, const Totals &) const {
    ServeCtl *c = a->ctl;
    ServeMailbox *mb = a->mb;
    SrvTot &T = c->tot[d & 1];
    const unsigned long long lor = ld_agent(&T.lor);
    const unsigned long long act = ld_agent(&c->active);
    const unsigned long long done = act & ~lor;
    if (done) {
      // every record of these lanes was written before this barrier; the
      // system-scope fence orders them before the completion records
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "");
      unsigned long long k = ld_sys(&mb->completed);
      for (unsigned long long b = done; b; b &= b - 1ull) {
        const int i = __builtin_ctzll(b);
        st_sys(&mb->done[k % kSrvRing], (unsigned long long)c->lane[i].qid);
        ++k;
      }
      __hip_atomic_store(&mb->completed, k, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
    }
    st_agent(&c->active, act & ~done);
    st_agent(&c->clear, done);
    st_agent(&c->fresh, 0ull);
    const int64_t nf = (int64_t)ld_agent(&T.nf);
    const int64_t mf = (int64_t)ld_agent(&T.mf);
    const int64_t mu = (int64_t)ld_agent(&T.mu);
    const int dir0 = __hip_atomic_load(&c->dir, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const int dir = decide_direction(dir0 == 0 ? kTopDown : dir0, nf, mf, mu,
                                     (int64_t)ld_agent((const unsigned long long *)&c->nf_prev), a->n,
                                     a->p, d);
    __hip_atomic_store(&c->dir, dir, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    st_agent((unsigned long long *)&c->nf_prev, (unsigned long long)nf);
    SrvTot &U = c->tot[(d + 1) & 1];  // feeds the next advance
    st_agent(&U.nf, 0ull);
    st_agent(&U.mf, 0ull);
    st_agent(&U.mu, 0ull);
    st_agent(&U.lor, 0ull);
    return {0, -1};
  }
};

// Writes parent/depth of every lane in `bits` at vertex v (lanes from LDS).
__device__ inline void srv_record(const ServeLane *lanes, int64_t v, unsigned long long bits,
                                  int32_t parent, int32_t level) {
  for (; bits; bits &= bits - 1ull) {
    const ServeLane &L = lanes[__builtin_ctzll(bits)];
    L.parent[v] = parent;
    if (L.depth) L.depth[v] = level - L.inj;
  }
}

__device__ inline uint64_t srv_wave_or(uint64_t x) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) x |= __shfl_xor(x, o, kWave);
  return x;
}

__device__ inline uint64_t srv_wave_excl_or(uint64_t x) {
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

__device__ __forceinline__ void serve_body(const SrvArgs &a) {
  __shared__ Stage<kSrvBlock> st;
  __shared__ ServeLane s_lane[kSrvLanes];
  __shared__ unsigned long long s_acc[4];
  const int64_t nthreads = (int64_t)gridDim.x * kSrvBlock;
  const int64_t tid = (int64_t)blockIdx.x * kSrvBlock + threadIdx.x;
  const int64_t nwaves = nthreads / kWave;
  const int64_t gwave = tid / kWave;
  const int lane = lane_id();
  const unsigned int nblocks = gridDim.x;
  const int hub = a.p.hub, chunk = a.p.chunk;
  Ctl *ctl = &a.ctl->base;
  const int64_t nwords = (a.n + kWave - 1) / kWave;
  const int64_t nv = nwords * kWave;
  const int64_t *__restrict__ rp = a.row_ptr;
  const int32_t *__restrict__ col = a.col;
  uint64_t *V = a.V, *F = a.B0, *N = a.B1;

  for (int64_t i = tid; i < nv; i += nthreads) {
    V[i] = 0ull;
    F[i] = 0ull;
    N[i] = 0ull;
  }
  if (!grid_sync(ctl, nblocks, Totals{}, -1, 0, a.p.wait)) return;
  {
    int flag = 0;
    const SrvTake first{&a, -1, N};
    if (!grid_sync_x(ctl, main_barrier(ctl, a.p.wait), nblocks, Totals{}, -1, 0, first, flag)) return;
    if (uni(flag)) return;
  }
  swap_ptr(F, N);

  for (int32_t d = 0;; ++d) {
    if ((int64_t)d > a.n + 1000000) {  // guard: far more levels than any search needs
      if (tid == 0) atomicExch(&ctl->err, (int)GAP_EINTERNAL);
      return;
    }
    const unsigned long long active = uni((int64_t)ld_agent(&a.ctl->active));
    const unsigned long long fresh = uni((int64_t)ld_agent(&a.ctl->fresh));
    const unsigned long long clear = uni((int64_t)ld_agent(&a.ctl->clear));
    for (int i = threadIdx.x; i < kSrvLanes; i += kSrvBlock) s_lane[i] = a.ctl->lane[i];
    if (threadIdx.x == 0) {
      st.qn = 0;
      st.cn = 0;
      st.hn = 0;
      s_acc[0] = s_acc[1] = s_acc[2] = s_acc[3] = 0ull;
    }
    __syncthreads();
    // ---- advance: V |= F (after clearing finished lanes), queue F, clear N,
    // write the outputs of lanes that joined at the last boundary ----
    StepArgs sa{};
    sa.Q = a.Q;
    sa.bs_in = d & 1;  // staged into buffer set (d + 1) & 1
    sa.ctl = ctl;
    sa.hub = hub;
    sa.chunk = chunk;
    LaneAcc none;
    for (int64_t wd = gwave; wd < nwords; wd += nwaves) {
      const int64_t v = wd * kWave + lane;
      const bool real = v < a.n;
      const uint64_t f = F[v];
      uint64_t vis = V[v];
      vis = (vis & ~clear) | f;
      V[v] = vis;
      N[v] = 0ull;
      const int64_t deg = real ? rp[v + 1] - rp[v] : 0;
      const bool incomplete = real && deg > 0 && (active & ~vis) != 0ull;
      if (fresh && real) {
        for (unsigned long long b = fresh; b; b &= b - 1ull) {
          const ServeLane &L = s_lane[__builtin_ctzll(b)];
          const bool is_src = v == (int64_t)L.source;
          L.parent[v] = is_src ? (int32_t)v : -1;
          if (L.depth) L.depth[v] = is_src ? 0 : -1;
        }
      }
      const unsigned long long c_nf = wave_sum_u64(f ? 1ull : 0ull);
      const unsigned long long c_mf = wave_sum_u64(f ? (unsigned long long)deg : 0ull);
      const unsigned long long c_mu = wave_sum_u64(incomplete ? (unsigned long long)deg : 0ull);
      const uint64_t c_or = srv_wave_or(f);
      if (lane == 0) {
        if (c_nf) atomicAdd(&s_acc[0], c_nf);
        if (c_mf) atomicAdd(&s_acc[1], c_mf);
        if (c_mu) atomicAdd(&s_acc[2], c_mu);
        if (c_or) atomicOr(&s_acc[3], c_or);
      }
      const bool big = deg > hub;
      stage_vertices<kSrvBlock>(sa, st, f && !big, (int32_t)v);
      stage_chunks<kSrvBlock>(sa, st, f && big, (int32_t)v, deg, 0);
      stage_chunks<kSrvBlock>(sa, st, incomplete && big, (int32_t)v, deg, kSrvBuFlag);
    }
    (void)step_end<kSrvBlock, false>(sa, st, none);
    __syncthreads();
    if (threadIdx.x == 0) {
      SrvTot &T = a.ctl->tot[d & 1];
      add_agent(&T.nf, s_acc[0]);
      add_agent(&T.mf, s_acc[1]);
      add_agent(&T.mu, s_acc[2]);
      if (s_acc[3]) atomicOr(&T.lor, s_acc[3]);
    }
    {
      int unused = 0;
      const SrvRetire dec{&a, d};
      if (!grid_sync_x(ctl, main_barrier(ctl, a.p.wait), nblocks, Totals{}, (d + 1) & 1, (d + 1) & 1,
                       dec, unused))
        return;
    }
    const unsigned long long live = uni((int64_t)ld_agent(&a.ctl->active));
    const int dir = uni(__hip_atomic_load(&a.ctl->dir, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));

    // ---- step ----
    StepArgs qa{};
    qa.Q = a.Q;
    qa.bs_in = (d + 1) & 1;  // the queue built by this level's advance
    qa.ctl = ctl;
    qa.d = d + 1;            // pub[(d + 1) & 1] holds its segment sizes
    step_begin<kSrvBlock>(qa, st);
    const int32_t nd = d + 1;
    if (live) {
      // chunk items: top-down hub chunks (push) and bottom-up hub chunks (pull)
      const unsigned long long nc = st.cpre[kGroups];
      const int2 *cin = a.Q.cs(qa.bs_in);
      for (unsigned long long ci = (unsigned long long)gwave; ci < nc;
           ci += (unsigned long long)nwaves) {
        const int h = seg_of(ci, st.cpre);
        const int2 it = cin[h * a.Q.ccap + (int64_t)(ci - st.cpre[h])];
        const int64_t x = it.x;
        const bool bu_item = (it.y & kSrvBuFlag) != 0;
        const int k = it.y & ~kSrvBuFlag;
        if (dir != (bu_item ? kBottomUp : kTopDown)) continue;
        const int64_t rbeg = rp[x], rend = rp[x + 1];
        const int64_t beg = rbeg + (int64_t)k * chunk;
        const int64_t end = beg + chunk < rend ? beg + chunk : rend;
        if (!bu_item) {
          const uint64_t fu = F[x];
          for (int64_t e = beg + lane; e < end; e += kWave) {
            const int32_t v = col[e];
            const uint64_t nb = fu & ~V[v];
            if (!nb) continue;
            const uint64_t old = atomicOr(reinterpret_cast<unsigned long long *>(&N[v]), nb);
            const uint64_t mine = nb & ~old;
            if (mine) srv_record(s_lane, v, mine, (int32_t)x, nd);
          }
        } else {
          // each lane bit goes to the lowest wave lane that found it; one
          // atomicOr per round settles races with the hub's other chunks
          uint64_t need = live & ~V[x] & ~ld_agent(reinterpret_cast<const unsigned long long *>(&N[x]));
          for (int64_t e0 = beg; e0 < end && need; e0 += kWave) {
            const int64_t e = e0 + lane;
            const int32_t u = e < end ? col[e] : -1;
            const uint64_t hit = u >= 0 ? F[u] & need : 0ull;
            const uint64_t all = srv_wave_or(hit);
            if (all) {
              const uint64_t own = hit & ~srv_wave_excl_or(hit);
              unsigned long long old = 0;
              if (lane == 0) old = atomicOr(reinterpret_cast<unsigned long long *>(&N[x]), all);
              old = __shfl(old, 0, kWave);
              const uint64_t mine = own & ~old;
              if (mine) srv_record(s_lane, x, mine, u, nd);
              need &= ~all;
            }
          }
        }
      }
      if (dir == kTopDown) {
        // top-down over queued (non-hub) frontier vertices: a wave walks the
        // combined edge range of up to 64 of them
        const unsigned long long nq = st.qpre[kGroups];
        const int32_t *qin = a.Q.qs(qa.bs_in);
        unsigned long long per = (nq + (unsigned long long)nwaves - 1) / (unsigned long long)nwaves;
        per = per < 1 ? 1 : (per > 64 ? 64 : per);
        const unsigned long long ngroups = (nq + per - 1) / per;
        for (unsigned long long gi = (unsigned long long)gwave; gi < ngroups;
             gi += (unsigned long long)nwaves) {
          const unsigned long long idx = gi * per + lane;
          int32_t u = -1;
          int64_t beg = 0;
          uint32_t deg = 0;
          if ((unsigned long long)lane < per && idx < nq) {
            const int h = seg_of(idx, st.qpre);
            u = qin[h * a.Q.n + (int64_t)(idx - st.qpre[h])];
            beg = rp[u];
            deg = (uint32_t)(rp[u + 1] - beg);
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
            const int32_t uj = __shfl(u, j, kWave);
            const int64_t bj = __shfl(beg, j, kWave);
            const uint32_t oj = __shfl(off, j, kWave);
            if (e < total) {
              const int32_t v = col[bj + (int64_t)(e - oj)];
              const uint64_t nb = F[uj] & ~V[v];
              if (nb) {
                const uint64_t old = atomicOr(reinterpret_cast<unsigned long long *>(&N[v]), nb);
                const uint64_t mine = nb & ~old;
                if (mine) srv_record(s_lane, v, mine, uj, nd);
              }
            }
          }
        }
      } else {
        // bottom-up over non-hub vertices: lane i owns vertex 64w+i and is the
        // only writer of its V and N words
        for (int64_t wd = gwave; wd < nwords; wd += nwaves) {
          const int64_t v = wd * kWave + lane;
          int64_t beg = 0, end = 0;
          if (v < a.n) {
            beg = rp[v];
            end = rp[v + 1];
          }
          const uint64_t vis = V[v];
          uint64_t need = (v < a.n && end > beg && end - beg <= hub) ? (live & ~vis) : 0ull;
          uint64_t got = 0ull;
          bool act = need != 0ull;
          int64_t e = beg;
          while (__ballot(act) != 0ull) {
            int32_t u[4];
#pragma unroll
            for (int k = 0; k < 4; ++k) u[k] = (act && e + k < end) ? col[e + k] : -1;
            uint64_t fu[4];
#pragma unroll
            for (int k = 0; k < 4; ++k) fu[k] = u[k] >= 0 ? F[u[k]] : 0ull;
#pragma unroll
            for (int k = 0; k < 4; ++k) {  // the first neighbour in list order wins a lane
              const uint64_t hit = fu[k] & need;
              if (hit) {
                srv_record(s_lane, v, hit, u[k], nd);
                need &= ~hit;
                got |= hit;
              }
            }
            e += 4;
            act = act && need != 0ull && e < end;
          }
          if (got) {
            V[v] = vis | got;
            N[v] = got;
          }
        }
      }
    }
    {
      int flag = 0;
      const SrvTake dec{&a, d, N};
      if (!grid_sync_x(ctl, main_barrier(ctl, a.p.wait), nblocks, Totals{}, -1, 0, dec, flag)) return;
      if (uni(flag)) break;
    }
    swap_ptr(F, N);
  }
}

__global__ __launch_bounds__(kSrvBlock) void k_serve(SrvArgs a) {
  serve_body(a);
  note_error(a.sticky, &a.ctl->base);
  if (threadIdx.x == 0) {
    const int e = __hip_atomic_load(&a.ctl->base.err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (e != 0) {
      int expected = 0;
      __hip_atomic_compare_exchange_strong(&a.mb->err, &expected, e, __ATOMIC_RELAXED,
                                           __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    }
  }
}

__global__ __launch_bounds__(256) void k_srv_clear(uint32_t *p, int64_t words) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < words; i += stride) p[i] = 0u;
}

}  // namespace gap

// ---- host side ---------------------------------------------------------------------

using namespace gap;

struct gap_server {
  int device = -1;
  hipStream_t stream = nullptr;
  int64_t cap_n = 0, cap_nnz = 0;
  char *buf = nullptr;
  size_t o_V = 0, o_B0 = 0, o_B1 = 0, o_q0 = 0, o_q1 = 0, o_c0 = 0, o_c1 = 0, o_ctl = 0;
  int64_t ccap = 0;
  ServeMailbox *mb = nullptr;      // host address (pinned)
  ServeMailbox *mb_dev = nullptr;  // device address of the same memory
  hipEvent_t last = nullptr;       // recorded after the latest launch
  bool launched = false;
  const gap_graph *g = nullptr;  // graph of the requests in flight
  unsigned long long posted = 0, reaped = 0;
  unsigned int gen = 0;
  std::mutex mu;
};

namespace {

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

void release_server(gap_server *s) {
  if (s->stream) (void)hipStreamSynchronize(s->stream);
  if (s->buf) (void)hipFree(s->buf);
  if (s->mb) (void)hipHostFree(s->mb);
  if (s->last) (void)hipEventDestroy(s->last);
  (void)hipGetLastError();
  delete s;
}

gap_status server_launch(gap_server *s) {
  const DeviceInfo *di = nullptr;
  gap_status st = device_info(s->device, &di);
  if (st != GAP_OK) return st;
  const gap_params p = params_current();
  s->gen = s->gen + 1u == 0u ? 1u : s->gen + 1u;
  __atomic_store_n(&s->mb->accepting, s->gen, __ATOMIC_SEQ_CST);
  const gap_graph *g = s->g;
  SrvArgs a{};
  a.row_ptr = g->row_ptr;
  a.col = g->col;
  a.n = g->n;
  a.V = reinterpret_cast<uint64_t *>(s->buf + s->o_V);
  a.B0 = reinterpret_cast<uint64_t *>(s->buf + s->o_B0);
  a.B1 = reinterpret_cast<uint64_t *>(s->buf + s->o_B1);
  a.Q.q0 = reinterpret_cast<int32_t *>(s->buf + s->o_q0);
  a.Q.q1 = reinterpret_cast<int32_t *>(s->buf + s->o_q1);
  a.Q.c0 = reinterpret_cast<int2 *>(s->buf + s->o_c0);
  a.Q.c1 = reinterpret_cast<int2 *>(s->buf + s->o_c1);
  a.Q.n = ((s->cap_n + kWave - 1) / kWave) * kWave;
  a.Q.ccap = s->ccap;
  a.ctl = reinterpret_cast<ServeCtl *>(s->buf + s->o_ctl);
  a.mb = s->mb_dev;
  Workspace *ws = workspace_for(s->device, s->stream);
  if (!ws) {
    set_error("workspace allocation failed");
    return GAP_ENOMEM;
  }
  a.sticky = ws->sticky;
  a.p = Params{p.batch_alpha, p.batch_beta, p.direction, p.hub_degree, p.chunk_edges, 0, 0, 0, 0, 0};
  set_wait_limits(a.p, p.wait_limit_us);
  a.gen = s->gen;
  a.window = (unsigned long long)(p.serve_window_us > 0 ? p.serve_window_us : 1) * kTicksPerUs;

  static_assert(sizeof(ServeCtl) % sizeof(uint32_t) == 0, "cleared word by word");
  CoopOrder order;
  st = coop_begin(s->device, s->stream, p.grid_split, &order);
  if (st != GAP_OK) return st;
  k_srv_clear<<<8, 256, 0, s->stream>>>(reinterpret_cast<uint32_t *>(a.ctl),
                                          (int64_t)(sizeof(ServeCtl) / sizeof(uint32_t)));
  hipError_t e = hipGetLastError();
  if (e == hipSuccess) {
    int per_cu = 0;
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void *)k_serve, kSrvBlock, 0);
    if (e == hipSuccess && per_cu < 1) {
      set_error("serving kernel does not fit on a compute unit");
      st = GAP_EDEVICE;
    } else if (e == hipSuccess) {
      void *kargs[] = {&a};
      st = launch_resident((const void *)k_serve, di->cus, kSrvBlock, 0, kargs, p.grid_split, p.coop_launch, di,
                           s->stream, nullptr);
    }
  }
  if (e != hipSuccess) st = hip_fail(e, "serving launch");
  const gap_status st2 = coop_end(s->device, s->stream, &order);
  if (st == GAP_OK) {
    const hipError_t er = hipEventRecord(s->last, s->stream);
    if (er != hipSuccess) st = hip_fail(er, "hipEventRecord");
    s->launched = true;
  }
  if (st != GAP_OK) {
    __atomic_store_n(&s->mb->accepting, 0u, __ATOMIC_SEQ_CST);
    return st;
  }
  return st2;
}

}  // namespace

extern "C" {

gap_status gap_serve_open(int64_t max_vertices, int64_t max_entries, void *stream,
                          gap_server **out) {
  clear_error();
  if (!out) {
    set_error("gap_serve_open: NULL out");
    return GAP_EINVAL;
  }
  *out = nullptr;
  if (max_vertices < 1 || max_vertices > 2147483647ll || max_entries < 0) {
    set_error("gap_serve_open: sizes out of range");
    return GAP_EINVAL;
  }
  int dev = 0;
  GAP_HIP(hipGetDevice(&dev));
  const gap_params p = params_current();
  gap_server *s = new (std::nothrow) gap_server();
  if (!s) {
    set_error("gap_serve_open: out of host memory");
    return GAP_ENOMEM;
  }
  s->device = dev;
  s->stream = (hipStream_t)stream;
  s->cap_n = max_vertices;
  s->cap_nnz = max_entries;
  const int64_t nv = ((max_vertices + kWave - 1) / kWave) * kWave;
  // chunk items per level: top-down and bottom-up hub chunks, each bounded
  // by entries/chunk + entries/hub (one partial chunk per hub)
  s->ccap = 2 * (max_entries / p.chunk_edges + max_entries / p.hub_degree) + 4;
  size_t o = 0;
  auto take = [&](size_t bytes) {
    o = align256(o);
    const size_t at = o;
    o += bytes;
    return at;
  };
  s->o_ctl = take(sizeof(ServeCtl));
  s->o_V = take(sizeof(uint64_t) * (size_t)nv);
  s->o_B0 = take(sizeof(uint64_t) * (size_t)nv);
  s->o_B1 = take(sizeof(uint64_t) * (size_t)nv);
  s->o_q0 = take(sizeof(int32_t) * (size_t)nv * kGroups);
  s->o_q1 = take(sizeof(int32_t) * (size_t)nv * kGroups);
  s->o_c0 = take(sizeof(int2) * (size_t)s->ccap * kGroups);
  s->o_c1 = take(sizeof(int2) * (size_t)s->ccap * kGroups);
  hipError_t e = hipMalloc(&s->buf, o);
  if (e == hipSuccess) e = hipHostMalloc(&s->mb, sizeof(ServeMailbox), hipHostMallocCoherent);
  if (e == hipSuccess) {
    memset(s->mb, 0, sizeof(ServeMailbox));
    e = hipHostGetDevicePointer(reinterpret_cast<void **>(&s->mb_dev), s->mb, 0);
  }
  if (e == hipSuccess) e = hipEventCreateWithFlags(&s->last, hipEventDisableTiming);
  if (e != hipSuccess) {
    const gap_status st = hip_fail(e, "gap_serve_open");
    release_server(s);
    return st;
  }
  *out = s;
  return GAP_OK;
}

gap_status gap_serve_submit(gap_server *s, const gap_graph *g, int64_t qid, int32_t source,
                            int32_t *parent, int32_t *depth) {
  clear_error();
  if (!s || !g || !parent) {
    set_error("gap_serve_submit: NULL %s", !s ? "server" : (!g ? "graph" : "parent"));
    return GAP_EINVAL;
  }
  std::lock_guard<std::mutex> lk(s->mu);
  if (g->device != s->device || g->directed) {
    set_error("gap_serve_submit: the graph must be undirected and on the server's device");
    return GAP_EINVAL;
  }
  if (g->n > s->cap_n || g->nnz > s->cap_nnz) {
    set_error("gap_serve_submit: graph (n = %lld, %lld entries) exceeds the server's sizes",
              (long long)g->n, (long long)g->nnz);
    return GAP_EINVAL;
  }
  if (source < 0 || (int64_t)source >= g->n) {
    set_error("gap_serve_submit: source %d outside [0, %lld)", source, (long long)g->n);
    return GAP_EINVAL;
  }
  const unsigned long long outstanding = s->posted - s->reaped;
  if (outstanding >= (unsigned long long)kSrvRing) {
    set_error("gap_serve_submit: %d requests in flight (poll first)", kSrvRing);
    return GAP_EBUSY;
  }
  if (s->g != g) {
    if (outstanding > 0) {
      set_error("gap_serve_submit: the server holds requests on another graph");
      return GAP_EBUSY;
    }
    // the previous graph's launch has no lane left and is about to leave
    GAP_HIP(hipSetDevice(s->device));
    GAP_HIP(hipStreamSynchronize(s->stream));
    __atomic_store_n(&s->mb->accepting, 0u, __ATOMIC_SEQ_CST);
    s->g = g;
  }
  ServeReq &r = s->mb->req[s->posted % kSrvRing];
  r.qid = qid;
  r.source = source;
  r.parent = parent;
  r.depth = depth;
  __atomic_store_n(&s->mb->posted, s->posted + 1, __ATOMIC_SEQ_CST);
  s->posted += 1;
  __atomic_thread_fence(__ATOMIC_SEQ_CST);
  if (__atomic_load_n(&s->mb->accepting, __ATOMIC_SEQ_CST) == 0u) {
    GAP_HIP(hipSetDevice(s->device));
    return server_launch(s);
  }
  return GAP_OK;
}

gap_status gap_serve_poll(gap_server *s, int64_t *qids, int32_t max, int32_t *count) {
  clear_error();
  if (!s || !count || (max > 0 && !qids) || max < 0) {
    set_error("gap_serve_poll: bad arguments");
    return GAP_EINVAL;
  }
  std::lock_guard<std::mutex> lk(s->mu);
  *count = 0;
  const unsigned long long done = __atomic_load_n(&s->mb->completed, __ATOMIC_ACQUIRE);
  int32_t c = 0;
  while (s->reaped < done && c < max) {
    qids[c++] = s->mb->done[s->reaped % kSrvRing];
    s->reaped += 1;
  }
  *count = c;
  const int err = __atomic_exchange_n(&s->mb->err, 0, __ATOMIC_SEQ_CST);
  if (err != 0) {
    set_error("a serving launch failed on the device (%s); requests in flight are lost",
              err == GAP_ETIMEOUT ? "a bounded wait gave up" : "inconsistent state");
    return err;
  }
  // requests that no launch will take (the last one has left): launch again
  if (s->launched && __atomic_load_n(&s->mb->taken, __ATOMIC_ACQUIRE) < s->posted &&
      hipEventQuery(s->last) == hipSuccess) {
    GAP_HIP(hipSetDevice(s->device));
    return server_launch(s);
  }
  (void)hipGetLastError();
  return GAP_OK;
}

gap_status gap_serve_close(gap_server *s) {
  clear_error();
  if (!s) return GAP_OK;
  (void)hipSetDevice(s->device);
  release_server(s);
  return GAP_OK;
}

}  // extern "C"
