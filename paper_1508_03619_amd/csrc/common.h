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

struct DevGraph {
  const int64_t *row_ptr;  // int64[n+1]
  const int32_t *col;      // int32[nnz], each row ascending
  int64_t n;
  int64_t nnz;
};

// Totals accumulated by one level (single-source search).
struct LevelCounters {
  unsigned long long nq;       // entries appended to the next vertex queue
  unsigned long long nc;       // chunk items appended to the next chunk queue
  unsigned long long nv;       // vertices claimed: |F_{d+1}|
  unsigned long long mf;       // sum of degrees over F_{d+1}
  unsigned long long scanned;  // adjacency entries read (statistics only)
  unsigned long long unvisited;// bottom-up vertices still searching (stats)
  unsigned long long pad[2];
};

// Device-resident control block of one workspace.
struct Ctl {
  LevelCounters cnt[3];     // ring: level d accumulates into cnt[d % 3]
  unsigned int bar_count;   // grid barrier arrivals
  unsigned int bar_gen;     // grid barrier generation
  int err;                  // GAP_ETIMEOUT when a bounded wait gave up
  int levels;               // levels run by the last search
  unsigned long long pad[4];
};

struct Params {
  int32_t alpha, beta, direction, hub, chunk;
};

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

// Real-time clock (100 MHz constant clock on CDNA).
__device__ inline uint64_t rt_clock() { return __builtin_amdgcn_s_memrealtime(); }

constexpr uint64_t kBarrierTimeoutTicks = 300000000ull;  // ~3 s at 100 MHz

// Grid-wide barrier for a cooperative launch.  Every workgroup of the grid
// must call it the same number of times.  Bounded: a workgroup that waits
// longer than the timeout records GAP_ETIMEOUT in ctl->err and returns.
// Returns false once an error has been recorded.
__device__ inline bool grid_barrier(Ctl *ctl, unsigned int nblocks) {
  __syncthreads();
  __shared__ int s_ok;
  if (threadIdx.x == 0) {
    int ok = 1;
    unsigned int gen = __hip_atomic_load(&ctl->bar_gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    unsigned int prev =
        __hip_atomic_fetch_add(&ctl->bar_count, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
    if (prev == nblocks - 1) {
      __hip_atomic_store(&ctl->bar_count, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __hip_atomic_store(&ctl->bar_gen, gen + 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    } else {
      const uint64_t t0 = rt_clock();
      while (__hip_atomic_load(&ctl->bar_gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == gen) {
        __builtin_amdgcn_s_sleep(1);
        if (rt_clock() - t0 > kBarrierTimeoutTicks) {
          __hip_atomic_store(&ctl->err, (int)GAP_ETIMEOUT, __ATOMIC_RELAXED,
                             __HIP_MEMORY_SCOPE_AGENT);
          ok = 0;
          break;
        }
      }
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    }
    if (__hip_atomic_load(&ctl->err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) ok = 0;
    s_ok = ok;
  }
  __syncthreads();
  return s_ok != 0;
}

}  // namespace gap
