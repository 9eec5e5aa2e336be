// Shared device/host definitions of libgapbfs (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "gapbfs.h"

namespace gap {

constexpr int kWave = 64;
// Parent-array encoding of an unvisited vertex (Section 3, BFS): -degree.
// A degree-0 vertex would encode as 0, which is a vertex ID, so it gets the
// most negative int32 instead; it can only be reached as the source.
constexpr int32_t kIsolated = INT32_MIN;

// Workgroups are split into kGroups groups (blockIdx % kGroups).  Same-address
// device atomics serialise (about 12 ns each on MI355X), so every shared
// counter is per group: a group's workgroups contend on their own cache line,
// and queues are segmented per group (each segment can hold n vertices).
constexpr int kGroups = 16;

// Column arrays are allocated kColPad entries longer than nnz, so a 16-byte
// read of four list entries that starts at any entry stays inside the
// allocation (entries past a list's end are read, then ignored).
constexpr int kColPad = 4;

// Four consecutive int32 with 4-byte alignment: one global_load_dwordx4.
typedef int32_t i32x4_a4 __attribute__((ext_vector_type(4), aligned(4)));

struct DevGraph {
  const int64_t *row_ptr;     // int64[n+1], out-lists (top-down)
  const int32_t *col;         // int32[nnz], each row ascending
  const int64_t *row_ptr_in;  // in-lists (bottom-up); the same arrays when undirected
  const int32_t *col_in;
  const int4 *head_in;        // first four in-list entries of every vertex (-1 past the end)
  int64_t n;
  int64_t nnz;
  int32_t directed;
  int64_t n_sinks;            // vertices with no out-list entry
};

// Level totals reduced across the grid.
struct Totals {
  unsigned long long nv;         // vertices claimed: |F_{d+1}|
  unsigned long long mf;         // sum of degrees over F_{d+1}
  unsigned long long scanned;    // adjacency entries read (statistics only)
  unsigned long long unvisited;  // bottom-up vertices still searching (stats)
};

struct alignas(128) GroupSlot {
  Totals part;          // partial totals of this group for the current level
  unsigned int arrive;  // barrier arrivals of this group
  unsigned int pad;
};

struct alignas(128) GenFlag {
  unsigned int gen;
  unsigned int pad;
};

struct alignas(128) SegCount {
  unsigned long long q;  // vertices appended to this group's queue segment
  unsigned long long c;  // hub chunk items appended to this group's segment
};

// What the grid learns at a level boundary: totals of the new frontier and
// the size of every queue segment that holds it.
struct alignas(128) Published {
  Totals t;
  unsigned long long q[kGroups];
  unsigned long long c[kGroups];
};

// Search state handed from the small group to the parked workgroups when
// every workgroup rejoins (single-source persistent kernel).
struct ParkState {
  int level, dir, have_bm, fsel;
  long long mu, nf_prev;
};

// Device-resident control block of one workspace (zeroed before a search).
struct Ctl {
  GroupSlot grp[kGroups];    // barrier of the whole grid
  GroupSlot top;
  GenFlag gen[kGroups];
  GroupSlot sgrp[kGroups];   // barrier of the small group (its first workgroups)
  GroupSlot stop;
  GenFlag sgen[kGroups];
  ParkState park;
  unsigned int resume;       // level at which parked workgroups rejoin
  SegCount seg[2][kGroups];  // live append counters, per queue buffer set
  Published pub[2];          // frontier of level d lives in pub[d & 1]
  int err;                   // GAP_ETIMEOUT / GAP_EINTERNAL
  int levels;                // levels run by the last search
  int done;                  // device-driven schedules: search finished
  int dir;                   // device-driven schedules: direction of next step
  int level;                 // device-driven schedules: next level
  int have_bm;               // device-driven schedules: bitmaps are current
  long long mu;              // device-driven schedules: unexplored edges
  long long nf_prev;         // device-driven schedules: previous frontier size
};

struct Params {
  int32_t alpha, beta, direction, hub, chunk;
  int32_t small;  // top-down levels with |F| and m_f at most this run on the small group
  int32_t bu_mapping;  // persistent bottom-up steps: 0 refilled lanes, 1 fixed words per wave
  int32_t td_plain;    // persistent top-down levels with m_f > n / td_plain claim by plain stores (0: never)
  uint64_t wait;       // bound of one barrier wait (real-time ticks)
  uint64_t wait_park;  // bound of a parked workgroup's wait without progress
};

// Device-side wait bounds from gap_params::wait_limit_us (0: the defaults).
inline void set_wait_limits(Params &p, int32_t wait_limit_us);

enum Dir : int32_t { kTopDown = 1, kBottomUp = 2 };

// Direction rule (Section 3 cites the direction-optimizing search: switch to
// bottom-up once the frontier is large enough).  Top-down -> bottom-up when
// the frontier's edges exceed the unexplored edges / alpha; bottom-up ->
// top-down when the frontier is small (< n / beta) and shrinking.
__host__ __device__ inline int32_t decide_direction(int32_t dir, int64_t nf, int64_t mf, int64_t mu,
                                                    int64_t nf_prev, int64_t n, const Params &p,
                                                    int32_t level) {
  if (p.direction == GAP_DIR_TOPDOWN) return kTopDown;
  if (p.direction == GAP_DIR_BOTTOMUP) return kBottomUp;
  if (level == 0) return kTopDown;
  if (dir == kTopDown) {
    return (mf > mu / (int64_t)p.alpha) ? kBottomUp : kTopDown;
  }
  return (nf < n / (int64_t)p.beta && nf < nf_prev) ? kTopDown : kBottomUp;
}

// ---- wave helpers ---------------------------------------------------------

__device__ inline int lane_id() { return __lane_id(); }

// Number of set bits of `mask` below this lane.
__device__ inline uint32_t lane_rank(uint64_t mask) {
  return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                   __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

__device__ inline uint32_t wave_excl_scan_u32(uint32_t x, uint32_t &total) {
  const int lane = lane_id();
  uint32_t s = x;
#pragma unroll
  for (int o = 1; o < kWave; o <<= 1) {
    uint32_t y = __shfl_up(s, o, kWave);
    if (lane >= o) s += y;
  }
  total = __shfl(s, kWave - 1, kWave);
  return s - x;
}

__device__ inline unsigned long long wave_sum_u64(unsigned long long x) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) x += __shfl_xor(x, o, kWave);
  return x;
}

template <class T>
__host__ __device__ inline void swap_ptr(T &a, T &b) {
  T t = a;
  a = b;
  b = t;
}

__device__ inline int first_lane(uint64_t mask) { return __builtin_ctzll(mask); }

// A value that is the same in every lane, moved to a scalar register (the
// compiler cannot prove that a loaded value is wave-uniform; keeping loop
// state in SGPRs leaves the VGPRs to the steps).
__device__ inline int32_t uni(int32_t x) { return __builtin_amdgcn_readfirstlane(x); }
__device__ inline uint32_t uni(uint32_t x) { return (uint32_t)__builtin_amdgcn_readfirstlane((int32_t)x); }
__device__ inline int64_t uni(int64_t x) {
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int32_t)(uint32_t)x);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int32_t)(uint32_t)((uint64_t)x >> 32));
  return (int64_t)(((uint64_t)hi << 32) | lo);
}

// Real-time clock (100 MHz constant clock on CDNA).
__device__ inline uint64_t rt_clock() { return __builtin_amdgcn_s_memrealtime(); }

constexpr uint64_t kBarrierTimeoutTicks = 300000000ull;  // ~3 s at 100 MHz
constexpr uint64_t kTicksPerUs = 100ull;

__device__ inline unsigned long long ld_agent(const unsigned long long *p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline unsigned int ld_agent(const unsigned int *p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline void st_agent(unsigned long long *p, unsigned long long v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline void st_agent(unsigned int *p, unsigned int v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline void add_agent(unsigned long long *p, unsigned long long v) {
  if (v) __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ inline int group_size(int g, unsigned int nblocks) {
  return (int)(nblocks / kGroups) + ((unsigned)g < nblocks % kGroups ? 1 : 0);
}

// Publishes group h's queue segment sizes of buffer set `bs` into
// pub[publish] and clears the live counters (one thread per group).
__device__ inline void publish_segment(Ctl *ctl, int publish, int bs, int h) {
  Published &P = ctl->pub[publish];
  const unsigned long long q = ld_agent(&ctl->seg[bs][h].q);
  const unsigned long long c = ld_agent(&ctl->seg[bs][h].c);
  st_agent(&P.q[h], q);
  st_agent(&P.c[h], c);
  st_agent(&ctl->seg[bs][h].q, 0ull);
  st_agent(&ctl->seg[bs][h].c, 0ull);
}

__device__ inline void publish_totals(Ctl *ctl, int publish, const Totals &t) {
  Published &P = ctl->pub[publish];
  st_agent(&P.t.nv, t.nv);
  st_agent(&P.t.mf, t.mf);
  st_agent(&P.t.scanned, t.scanned);
  st_agent(&P.t.unvisited, t.unvisited);
}

__device__ inline void add_totals(GroupSlot &s, const Totals &t) {
  add_agent(&s.part.nv, t.nv);
  add_agent(&s.part.mf, t.mf);
  add_agent(&s.part.scanned, t.scanned);
  add_agent(&s.part.unvisited, t.unvisited);
}

__device__ inline Totals take_totals(GroupSlot &s) {
  Totals t;
  t.nv = ld_agent(&s.part.nv);
  t.mf = ld_agent(&s.part.mf);
  t.scanned = ld_agent(&s.part.scanned);
  t.unvisited = ld_agent(&s.part.unvisited);
  st_agent(&s.part.nv, 0ull);
  st_agent(&s.part.mf, 0ull);
  st_agent(&s.part.scanned, 0ull);
  st_agent(&s.part.unvisited, 0ull);
  return t;
}

// The counters and flags of one barrier: the whole grid's or the small
// group's.
// `limit` bounds one wait for the release, in real-time ticks.
struct BarrierSet {
  GroupSlot *grp;
  GroupSlot *top;
  GenFlag *gen;
  uint64_t limit;
};
__device__ inline BarrierSet main_barrier(Ctl *c, uint64_t limit = kBarrierTimeoutTicks) {
  return {c->grp, &c->top, c->gen, limit};
}
__device__ inline BarrierSet small_barrier(Ctl *c, uint64_t limit = kBarrierTimeoutTicks) {
  return {c->sgrp, &c->stop, c->sgen, limit};
}

// What the last arriver decides for everyone: a flag delivered with the
// release (bit 0 of the generation word) and, when resume >= 0, a value
// stored to ctl->resume after the release fence.
struct BarrierDecision {
  int flag;
  int resume;
};
struct NoDecision {
  __device__ BarrierDecision operator()(Ctl *, const Totals &) const { return {0, -1}; }
};

// Grid-wide barrier with a reduction.  Every participating workgroup calls
// it the same number of times, with its partial totals in thread 0.
// Arrival is two-level (workgroup -> its group -> top) so that no address
// sees more than ~nblocks/kGroups atomics (same-address atomics serialise).
// The last workgroup of each group folds the group's totals into the top
// slot and, when `publish` >= 0, publishes its group's queue segment sizes
// of buffer set `bs`; the last group publishes the totals, runs `decide` on
// them, and releases everyone with one release fence and plain flag stores
// (a release store per flag would write the L2 back once per flag).  The
// generation word advances by 2 and carries the decision's flag in bit 0;
// `flag` returns it to every participant.
// Bounded: a workgroup that waits longer than B.limit records GAP_ETIMEOUT
// in ctl->err.  Returns false when this wait saw an error recorded (before
// the release, or by this workgroup's own time-out); an error recorded
// after the release is seen at the next wait.
template <class Decide>
__device__ inline bool grid_sync_x(Ctl *ctl, BarrierSet B, unsigned int nblocks, const Totals &part,
                                   int publish, int bs, const Decide &decide, int &flag) {
  __syncthreads();
  __shared__ int s_ok, s_flag;
  if (threadIdx.x == 0) {
    int ok = 1, fl = 0;
    const int g = (int)(blockIdx.x % kGroups);
    const unsigned int gen0 = ld_agent(&B.gen[g].gen);
    GroupSlot &gs = B.grp[g];
    add_totals(gs, part);
    const unsigned int a =
        __hip_atomic_fetch_add(&gs.arrive, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
    bool released = false;
    if ((int)a == group_size(g, nblocks) - 1) {
      // last of the group: fold the group into the top slot
      const Totals t = take_totals(gs);
      if (publish >= 0) publish_segment(ctl, publish, bs, g);
      st_agent(&gs.arrive, 0u);
      add_totals(*B.top, t);
      const int ngroups = nblocks < (unsigned)kGroups ? (int)nblocks : kGroups;
      const unsigned int b = __hip_atomic_fetch_add(&B.top->arrive, 1u, __ATOMIC_ACQ_REL,
                                                    __HIP_MEMORY_SCOPE_AGENT);
      if ((int)b == ngroups - 1) {
        // last overall: publish the totals, decide, clear, release every group
        const Totals all = take_totals(*B.top);
        st_agent(&B.top->arrive, 0u);
        if (publish >= 0) {
          publish_totals(ctl, publish, all);
          // groups without workgroups (nblocks < kGroups) publish empty segments
          for (int h = ngroups; h < kGroups; ++h) publish_segment(ctl, publish, bs, h);
        }
        const BarrierDecision dd = decide(ctl, all);
        fl = dd.flag & 1;
        const unsigned int next = (((gen0 >> 1) + 1u) << 1) | (unsigned)fl;
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        if (dd.resume >= 0) st_agent(&ctl->resume, (unsigned int)dd.resume);
        for (int h = 0; h < kGroups; ++h) st_agent(&B.gen[h].gen, next);
        released = true;
      }
    }
    if (!released) {
      // the error word is read in the same round trip as the flag: an
      // error recorded before the release stops this workgroup here, one
      // recorded later at its next wait (no load after the release)
      const uint64_t t0 = rt_clock();
      unsigned int v;
      for (;;) {
        v = ld_agent(&B.gen[g].gen);
        const int e = __hip_atomic_load(&ctl->err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (v != gen0) break;
        if (e != 0) {
          ok = 0;
          break;
        }
        __builtin_amdgcn_s_sleep(1);
        if (rt_clock() - t0 > B.limit) {
          __hip_atomic_store(&ctl->err, (int)GAP_ETIMEOUT, __ATOMIC_RELAXED,
                             __HIP_MEMORY_SCOPE_AGENT);
          ok = 0;
          break;
        }
      }
      fl = (int)(v & 1u);
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    s_ok = ok;
    s_flag = fl;
  }
  __syncthreads();
  flag = s_flag;
  return s_ok != 0;
}

__device__ inline bool grid_sync(Ctl *ctl, unsigned int nblocks, const Totals &part, int publish,
                                 int bs, uint64_t limit = kBarrierTimeoutTicks) {
  int flag;
  return grid_sync_x(ctl, main_barrier(ctl, limit), nblocks, part, publish, bs, NoDecision{}, flag);
}

// A parked workgroup waits until the small group sets ctl->resume above
// `level`, then takes over the handed-on state.  The wait is bounded by the
// time without progress, not by its total length: whenever `limit` ticks
// have passed, the small group's generation word is compared with its value
// at the previous check, and the clock restarts if the small group finished
// a level meanwhile.  So a search of millions of small levels in a row never
// trips it, a small group that stops making progress is caught within
// 2 * `limit` ticks, and the parked workgroups poll only `resume` and the
// error word in between, not the small barrier's release flag.
constexpr uint64_t kParkTimeoutTicks = 1000000000ull;  // ~10 s at 100 MHz

__device__ inline bool park_wait(Ctl *ctl, unsigned int level, ParkState &ps, uint64_t limit) {
  __syncthreads();
  __shared__ int s_ok;
  __shared__ ParkState s_ps;
  if (threadIdx.x == 0) {
    int ok = 1;
    uint64_t t0 = rt_clock();
    unsigned int seen = ld_agent(&ctl->sgen[0].gen);
    while (ld_agent(&ctl->resume) <= level) {
      __builtin_amdgcn_s_sleep(32);
      if (__hip_atomic_load(&ctl->err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) {
        ok = 0;
        break;
      }
      const uint64_t now = rt_clock();
      if (now - t0 > limit) {
        const unsigned int g = ld_agent(&ctl->sgen[0].gen);
        if (g != seen) {  // the small group finished a level within the last bound
          seen = g;
          t0 = now;
        } else {
          __hip_atomic_store(&ctl->err, (int)GAP_ETIMEOUT, __ATOMIC_RELAXED,
                             __HIP_MEMORY_SCOPE_AGENT);
          ok = 0;
          break;
        }
      }
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    if (__hip_atomic_load(&ctl->err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) ok = 0;
    s_ps = ctl->park;
    s_ok = ok;
  }
  __syncthreads();
  ps = s_ps;
  return s_ok != 0;
}

inline void set_wait_limits(Params &p, int32_t wait_limit_us) {
  p.wait = wait_limit_us > 0 ? (uint64_t)wait_limit_us * kTicksPerUs : kBarrierTimeoutTicks;
  p.wait_park = wait_limit_us > 0 ? (uint64_t)wait_limit_us * kTicksPerUs : kParkTimeoutTicks;
}

// End of a kernel that may have recorded an error in ctl->err: thread 0 of
// every workgroup copies it to the stream's sticky status word, which the
// next search does not clear (the host reads and clears it).  The workgroup
// that recorded the error always sees its own store, so a failure is never
// lost when the control block is cleared for a later search.
__device__ inline void note_error(int *sticky, const Ctl *ctl) {
  if (threadIdx.x != 0 || !sticky) return;
  const int e = __hip_atomic_load(&ctl->err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  if (e != 0) atomicCAS(sticky, 0, e);
}

}  // namespace gap
