// Betweenness centrality from a set of sources (Section 2.1, "Betweenness
// Centrality"; Brandes' method as the paper's reference code uses, Section 3).
//
// For each source s:
//   1. a direction-optimizing search (the library's single-source kernel)
//      gives depth[];
//   2. the reached vertices are grouped by (depth, length class of the
//      list) with a counting sort (LDS bins per tile, one global reservation
//      per bin and tile); a class-c list (at most 4 << c entries) is read by
//      1 << c lanes in one round, and every list longer than kLong entries
//      gets chunk items of kChunk entries instead (a directed graph has one
//      grouping by in-list and one by out-list length);
//   3. path counts, level by level away from s:
//        sigma[v] = sum of sigma[u] over in-neighbours u one level up;
//   4. dependencies, level by level towards s.  With
//        S[u] = sum over successors v (out-neighbours one level down) of
//               (1 + delta[v]) / sigma[v] = 1 / sigma[v] + S[v],
//      Brandes' dependency is delta[u] = sigma[u] * S[u], so a level reads
//      only (sigma, S) of the level below and no per-vertex finishing step is
//      needed between levels;
//   5. score[v] += sigma[v] * S[v] for every reached v != s.
// Each level of steps 3 and 4 either pulls (every vertex of the level sums
// over its own list: in-lists for sigma, out-lists for S) or pushes (every
// vertex of the neighbouring level adds its value atomically to the
// neighbours that lie in the level: out-lists for sigma, in-lists for S),
// whichever reads fewer adjacency entries -- the direction choice of the
// paper's BFS applied to the two passes of Brandes' method (pushed entries
// are charged four times for their atomics).
// Finally the scores are divided by the largest one (normalised to one),
// unless the caller asks for raw sums.
//
// Level membership is probed in bitmaps of n bits, which stay in L2 where
// the depth array would not.  Four bitmaps rotate (level d uses d mod 4):
// while a level kernel reads the bitmap of its own or the neighbouring
// level, it also marks the next level's vertices in a third (zeroing their
// path state) and clears the fourth for the level after.  Successors are found this way, not recorded: the paper
// keeps a successor bitmap to save memory over successor lists; this path
// keeps no per-edge state.  fp64 throughout.

#include <rocprim/device/device_scan.hpp>

#include "runtime.h"

namespace gap {
namespace {

constexpr int kBcBlock = 256;
constexpr int kTile = 8192;     // vertices per workgroup in the grouping kernels
constexpr int kLdsBins = 1024;  // keys counted in LDS; larger keys use global atomics
constexpr int kGroupClasses = 6;  // lists of <= 4 << c entries: 1 << c lanes per vertex
constexpr int kClasses = kGroupClasses + 1;  // the last class: chunk items
constexpr int kLong = 4 << (kGroupClasses - 1);  // 128: longer lists become chunk items
constexpr int kChunk = 512;     // entries per chunk item
constexpr int kPerLane = kChunk / kWave;
// A pushed entry costs about four probed ones: device-scope atomics are
// carried out at the memory side, not in the L2 (measured on the levels of
// R-MAT and uniform graphs of scale 22).
constexpr unsigned long long kPushWeight = 4;
constexpr int kWaves = kBcBlock / kWave;

// Per-vertex state read together by the level below: one 16-byte load.
struct __align__(16) PathState {
  double sigma;  // shortest paths from s
  double s;      // S = delta / sigma
};

__device__ inline uint32_t chunks_of(int64_t deg) {
  return deg > kLong ? (uint32_t)((deg + kChunk - 1) / kChunk) : 0u;
}

// Class c < kGroupClasses holds lists of at most 4 << c entries (one round
// of 4 loads per lane with 1 << c lanes per vertex).
__device__ inline int length_class(int64_t deg) {
  int c = 0;
  while (c < kGroupClasses && deg > (4 << c)) ++c;
  return c;
}

__device__ inline bool in_bitmap(const uint64_t *bm, int32_t u) {
  return (bm[u >> 6] >> (u & 63)) & 1ull;
}

__device__ inline void mark(uint64_t *bm, int32_t v) {
  atomicOr((unsigned long long *)&bm[v >> 6], 1ull << (v & 63));
}

// Workgroup maximum, then one atomic per workgroup.
template <class T>
__device__ inline void block_max_to(T m, T *out) {
  __shared__ T part[kBcBlock / kWave];
  for (int o = 32; o >= 1; o >>= 1) m = max(m, (T)__shfl_xor(m, o, kWave));
  if (lane_id() == 0) part[threadIdx.x / kWave] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < kBcBlock / kWave; ++w) m = max(m, part[w]);
    if (m > (T)0) atomicMax(out, m);
  }
}

// *dmax <- max depth; the four level bitmaps <- empty.
__global__ __launch_bounds__(kBcBlock) void k_bc_start(int64_t n, const int32_t *__restrict__ depth,
                                                       uint64_t *__restrict__ bms, int32_t *dmax) {
  int32_t m = 0;
  const int64_t stride = (int64_t)gridDim.x * kBcBlock;
  const int64_t tid = blockIdx.x * (int64_t)kBcBlock + threadIdx.x;
  for (int64_t v = tid; v < n; v += stride) m = max(m, depth[v]);
  const int64_t words = 4 * ((n + 63) / 64);
  for (int64_t w = tid; w < words; w += stride) bms[w] = 0ull;
  block_max_to(m, dmax);
}

// One grouping of the reached vertices for one set of lists.
struct GroupArgs {
  int64_t n;
  int32_t max_depth;  // bins exist for depths up to here; deeper vertices are left out
  const int32_t *depth;
  const int64_t *rp;  // the lists whose lengths set the class and the chunk items
  uint32_t *cnt;      // per key = depth * kClasses + class: vertices
  uint32_t *icnt;     // per depth: chunk items
  unsigned long long *esum;  // per depth: list entries (count pass only)
  int32_t *order;
  int2 *items;
};

__device__ inline void vertex_key(const GroupArgs &a, int64_t v, int32_t d, int64_t *key,
                                  uint32_t *nch, int64_t *deg) {
  *deg = a.rp[v + 1] - a.rp[v];
  *key = (int64_t)d * kClasses + length_class(*deg);
  *nch = chunks_of(*deg);
}

// Counts per key, and chunk items and list entries per depth.
__global__ __launch_bounds__(kBcBlock) void k_bc_count(GroupArgs a) {
  __shared__ uint32_t c[kLdsBins], ci[kLdsBins];
  __shared__ unsigned long long ce[kLdsBins];
  for (int b = threadIdx.x; b < kLdsBins; b += kBcBlock) {
    c[b] = ci[b] = 0;
    ce[b] = 0;
  }
  __syncthreads();
  const int64_t base = (int64_t)blockIdx.x * kTile;
  const int64_t end = min(base + kTile, a.n);
  for (int64_t v = base + threadIdx.x; v < end; v += kBcBlock) {
    const int32_t d = a.depth[v];
    if (d < 0 || d > a.max_depth) continue;
    int64_t key, deg;
    uint32_t nch;
    vertex_key(a, v, d, &key, &nch, &deg);
    if (key < kLdsBins)
      atomicAdd(&c[key], 1u);
    else
      atomicAdd(&a.cnt[key], 1u);
    if (d < kLdsBins) {
      if (nch) atomicAdd(&ci[d], nch);
      if (deg) atomicAdd(&ce[d], (unsigned long long)deg);
    } else {
      if (nch) atomicAdd(&a.icnt[d], nch);
      if (deg) atomicAdd(&a.esum[d], (unsigned long long)deg);
    }
  }
  __syncthreads();
  for (int b = threadIdx.x; b < kLdsBins; b += kBcBlock) {
    if (c[b]) atomicAdd(&a.cnt[b], c[b]);
    if (ci[b]) atomicAdd(&a.icnt[b], ci[b]);
    if (ce[b]) atomicAdd(&a.esum[b], ce[b]);
  }
}

// Places vertices in order[] and chunk items in items[] at positions
// reserved from the cursors (cnt / icnt hold the bin starts on entry).
__global__ __launch_bounds__(kBcBlock) void k_bc_scatter(GroupArgs a) {
  __shared__ uint32_t c[kLdsBins], ci[kLdsBins], b0[kLdsBins], bi[kLdsBins];
  for (int b = threadIdx.x; b < kLdsBins; b += kBcBlock) c[b] = ci[b] = 0;
  __syncthreads();
  const int64_t base = (int64_t)blockIdx.x * kTile;
  const int64_t end = min(base + kTile, a.n);
  for (int64_t v = base + threadIdx.x; v < end; v += kBcBlock) {
    const int32_t d = a.depth[v];
    if (d < 0 || d > a.max_depth) continue;
    int64_t key, deg;
    uint32_t nch;
    vertex_key(a, v, d, &key, &nch, &deg);
    if (key < kLdsBins) atomicAdd(&c[key], 1u);
    if (nch && d < kLdsBins) atomicAdd(&ci[d], nch);
  }
  __syncthreads();
  for (int b = threadIdx.x; b < kLdsBins; b += kBcBlock) {
    b0[b] = c[b] ? atomicAdd(&a.cnt[b], c[b]) : 0u;
    bi[b] = ci[b] ? atomicAdd(&a.icnt[b], ci[b]) : 0u;
    c[b] = ci[b] = 0;  // reused as in-tile cursors
  }
  __syncthreads();
  for (int64_t v = base + threadIdx.x; v < end; v += kBcBlock) {
    const int32_t d = a.depth[v];
    if (d < 0 || d > a.max_depth) continue;
    int64_t key, deg;
    uint32_t nch;
    vertex_key(a, v, d, &key, &nch, &deg);
    const uint32_t pos = key < kLdsBins ? b0[key] + atomicAdd(&c[key], 1u) : atomicAdd(&a.cnt[key], 1u);
    a.order[pos] = (int32_t)v;
    if (nch) {
      const uint32_t ipos = d < kLdsBins ? bi[d] + atomicAdd(&ci[d], nch) : atomicAdd(&a.icnt[d], nch);
      for (uint32_t k = 0; k < nch; ++k) a.items[ipos + k] = make_int2((int)v, (int)k);
    }
  }
}

// A grouping as the level kernels read it.
struct GroupView {
  const int32_t *order;
  const uint32_t *off;   // key starts in order[], [(D + 1) * kClasses + 1]
  const int2 *items;
  const uint32_t *ioff;  // depth starts in items[], [D + 2]
  const unsigned long long *esum;  // list entries per depth
};

struct LevelArgs {
  GroupView gin, gout;  // grouped by in-list / out-list length (the same when undirected)
  const int64_t *rp_in, *rp_out;
  const int32_t *col_in, *col_out;
  uint64_t *bms;        // four bitmaps of nwords words
  int64_t nwords;
  int32_t dmax;
  PathState *ps;
};

// Level d of the forward (sigma) or backward (S) pass.  Wave tasks, in
// order: for each length class c, 64 >> c vertices with 1 << c lanes each
// (a list read in one round of 4 loads per lane); then one chunk item each.
// Pull: the tasks cover level d and sum over its lists.  Push: they cover
// the neighbouring level and add along its lists into level d.  Before that
// every thread helps mark the next level and clear the bitmap after it.
template <bool FORWARD>
__global__ __launch_bounds__(kBcBlock) void k_bc_level(LevelArgs a, int32_t d) {
  const int32_t other = FORWARD ? d - 1 : d + 1;
  // pull reads the lists of level d, push the other lists of the other level
  const unsigned long long pull_cost = FORWARD ? a.gin.esum[d] : a.gout.esum[d];
  const unsigned long long push_cost = FORWARD ? a.gout.esum[other] : a.gin.esum[other];
  const bool push = kPushWeight * push_cost < pull_cost;
  const bool use_in = FORWARD != push;  // pull forward / push backward read in-lists
  const GroupView &gv = use_in ? a.gin : a.gout;
  const int64_t *rp = use_in ? a.rp_in : a.rp_out;
  const int32_t *col = use_in ? a.col_in : a.col_out;
  const int32_t td = push ? other : d;  // the level whose lists are read
  uint64_t *bm_level = a.bms + (int64_t)(d & 3) * a.nwords;
  const uint64_t *bm_other = a.bms + (int64_t)(other & 3) * a.nwords;
  const uint64_t *probe = push ? bm_level : bm_other;

  // side work: mark the next level (zeroing its state on the way out),
  // clear the bitmap two levels on
  {
    const int32_t nxt = FORWARD ? d + 1 : d - 1;
    const int64_t stride = (int64_t)gridDim.x * kBcBlock;
    const int64_t tid = blockIdx.x * (int64_t)kBcBlock + threadIdx.x;
    // two levels on in either direction: (d + 2) mod 4 == (d - 2) mod 4
    uint64_t *bm_clear = a.bms + (int64_t)((d + 2) & 3) * a.nwords;
    for (int64_t w = tid; w < a.nwords; w += stride) bm_clear[w] = 0ull;
    if (nxt >= 1 && nxt <= a.dmax) {
      uint64_t *bm_next = a.bms + (int64_t)(nxt & 3) * a.nwords;
      const uint32_t lo = a.gin.off[nxt * kClasses], hi = a.gin.off[(nxt + 1) * kClasses];
      for (int64_t i = lo + tid; i < hi; i += stride) {
        const int32_t v = a.gin.order[i];
        mark(bm_next, v);
        if (FORWARD) a.ps[v] = PathState{0.0, 0.0};
      }
    }
  }

  uint32_t first[kClasses + 1];  // first task of each class; items last
  uint32_t t0 = 0;
#pragma unroll
  for (int c = 0; c < kGroupClasses; ++c) {
    first[c] = t0;
    const uint32_t cnt = gv.off[td * kClasses + c + 1] - gv.off[td * kClasses + c];
    t0 += (cnt + (kWave >> c) - 1) / (kWave >> c);
  }
  first[kGroupClasses] = t0;
  const uint32_t ilo = gv.ioff[td];
  const uint32_t total = t0 + (gv.ioff[td + 1] - ilo);
  const int lane = lane_id();
  const int wave = threadIdx.x / kWave;
  // partial sums of chunk items, combined per vertex inside the workgroup
  // (a vertex's items are adjacent tasks) before one atomic update
  __shared__ int32_t item_v[kWaves];
  __shared__ double item_acc[kWaves];
  // every wave of a workgroup runs the same number of rounds (barriers below)
  for (uint32_t bt = blockIdx.x; bt * kWaves < total; bt += gridDim.x) {
    const uint32_t t = bt * kWaves + wave;
    int32_t v = -1;
    int64_t beg = 0, end = 0, step = kWave;
    int gshift = 6;
    bool lead = false;
    if (t < first[kGroupClasses]) {
      int c = 0;
      while (c + 1 < kGroupClasses && t >= first[c + 1]) ++c;
      gshift = c;  // 1 << c lanes per vertex
      const uint32_t lo = gv.off[td * kClasses + c];
      const uint32_t cnt = gv.off[td * kClasses + c + 1] - lo;
      const uint32_t vi = (t - first[c]) * (uint32_t)(kWave >> gshift) + (uint32_t)(lane >> gshift);
      const int gi = lane & ((1 << gshift) - 1);
      if (vi < cnt) {
        v = gv.order[lo + vi];
        beg = rp[v] + gi;
        end = rp[v + 1];
        lead = gi == 0;
      }
      step = (int64_t)1 << gshift;
    } else if (t < total) {
      const int2 it = gv.items[ilo + (t - first[kGroupClasses])];
      v = it.x;
      const int64_t rb = rp[v] + (int64_t)it.y * kChunk;
      beg = rb + lane;
      end = min(rb + (int64_t)kChunk, rp[v + 1]);
      lead = lane == 0;
    }
    constexpr int R = kPerLane;  // items: kPerLane rounds; groups use the first 4
    const int rounds = gshift < 6 ? 4 : R;
    int32_t u[R];
#pragma unroll
    for (int j = 0; j < R; ++j) {
      const int64_t e = beg + j * step;
      u[j] = (j < rounds && e < end) ? col[e] : -1;
    }
    bool hit[R];
#pragma unroll
    for (int j = 0; j < R; ++j) hit[j] = u[j] >= 0 && in_bitmap(probe, u[j]);
    if (push) {
      // every lane of the group holds the pushed value of its vertex
      double val = 0.0;
      if (v >= 0) {
        if (FORWARD) {
          val = a.ps[v].sigma;
        } else {
          const PathState q = a.ps[v];
          val = 1.0 / q.sigma + q.s;
        }
      }
#pragma unroll
      for (int j = 0; j < R; ++j)
        if (hit[j]) unsafeAtomicAdd(FORWARD ? &a.ps[u[j]].sigma : &a.ps[u[j]].s, val);
    } else {
      double acc = 0.0;
#pragma unroll
      for (int j = 0; j < R; ++j) {
        if (!hit[j]) continue;
        if (FORWARD) {
          acc += a.ps[u[j]].sigma;
        } else {
          const PathState q = a.ps[u[j]];
          acc += 1.0 / q.sigma + q.s;
        }
      }
      for (int o = (1 << gshift) >> 1; o >= 1; o >>= 1) acc += __shfl_xor(acc, o, kWave);
      if (lead && gshift < 6) {  // a whole list: store
        if (FORWARD)
          a.ps[v].sigma = acc;
        else
          a.ps[v].s = acc;
      }
      if (lane == 0) {
        item_v[wave] = (gshift == 6) ? v : -1;
        item_acc[wave] = acc;
      }
      __syncthreads();
      if (threadIdx.x < kWaves) {
        const int w = threadIdx.x;
        const int32_t x = item_v[w];
        bool first_of_v = x >= 0;
        for (int k = 0; k < w; ++k)
          if (item_v[k] == x) first_of_v = false;
        if (first_of_v) {
          double sum = 0.0;
          for (int k = w; k < kWaves; ++k)
            if (item_v[k] == x) sum += item_acc[k];
          if (sum != 0.0) unsafeAtomicAdd(FORWARD ? &a.ps[x].sigma : &a.ps[x].s, sum);
        }
      }
      __syncthreads();
    }
  }
}

// Level 0 and level 1 set up for the forward pass: sigma[s] = 1, s marked
// in bitmap 0; level 1 marked in bitmap 1 with zero state.
__global__ __launch_bounds__(kBcBlock) void k_bc_first(LevelArgs a, int32_t src) {
  const int64_t tid = blockIdx.x * (int64_t)kBcBlock + threadIdx.x;
  if (tid == 0) {
    a.ps[src] = PathState{1.0, 0.0};
    mark(a.bms, src);
  }
  if (a.dmax < 1) return;
  uint64_t *bm1 = a.bms + a.nwords;
  const uint32_t lo = a.gin.off[kClasses], hi = a.gin.off[2 * kClasses];
  for (int64_t i = lo + tid; i < hi; i += (int64_t)gridDim.x * kBcBlock) {
    const int32_t v = a.gin.order[i];
    mark(bm1, v);
    a.ps[v] = PathState{0.0, 0.0};
  }
}

// score[v] += sigma[v] * S[v] for the reached vertices other than the source
// (depth >= 1), in vertex order.
__global__ __launch_bounds__(kBcBlock) void k_bc_accumulate(int64_t n, const int32_t *__restrict__ depth,
                                                            const PathState *__restrict__ ps,
                                                            double *__restrict__ score) {
  for (int64_t v = blockIdx.x * (int64_t)kBcBlock + threadIdx.x; v < n;
       v += (int64_t)gridDim.x * kBcBlock) {
    if (depth[v] >= 1) {
      const PathState q = ps[v];
      score[v] += q.sigma * q.s;
    }
  }
}

// Scores are non-negative, so their IEEE bit patterns order like the values.
__global__ __launch_bounds__(kBcBlock) void k_bc_max(int64_t n, const double *__restrict__ score,
                                                     unsigned long long *top) {
  unsigned long long m = 0;
  for (int64_t v = blockIdx.x * (int64_t)kBcBlock + threadIdx.x; v < n;
       v += (int64_t)gridDim.x * kBcBlock)
    m = max(m, (unsigned long long)__double_as_longlong(score[v]));
  block_max_to(m, top);
}

__global__ __launch_bounds__(kBcBlock) void k_bc_scale(int64_t n, double *__restrict__ score,
                                                       const unsigned long long *top) {
  const double t = __longlong_as_double((long long)*top);
  if (!(t > 0.0)) return;
  for (int64_t v = blockIdx.x * (int64_t)kBcBlock + threadIdx.x; v < n;
       v += (int64_t)gridDim.x * kBcBlock)
    score[v] /= t;
}

int blocks_for(int64_t work, int cap) {
  const int64_t b = (work + kBcBlock - 1) / kBcBlock;
  return (int)std::max<int64_t>(1, std::min<int64_t>(b, cap));
}

template <class T>
T *carve(char *&p, size_t count) {
  T *r = reinterpret_cast<T *>(p);
  p += (sizeof(T) * count + 255) & ~(size_t)255;
  return r;
}

}  // namespace

// Vertices of one search grouped by (depth, class of the given lists) and
// the chunk items of the long lists, per depth.
struct Grouping {
  int32_t *order;
  int2 *items;
  uint32_t *cnt, *icnt;  // counts, then cursors
  uint32_t *off, *ioff;  // their exclusive scans
  unsigned long long *esum;
};

static gap_status build_grouping(const Grouping &gr, int64_t n, int32_t max_depth,
                                 const int32_t *depth, const int64_t *rp, size_t nk, size_t nl,
                                 void *scan_tmp, size_t scan_bytes, int grid_tiles,
                                 hipStream_t stream) {
  GAP_HIP(hipMemsetAsync(gr.cnt, 0, nk * sizeof(uint32_t), stream));
  GAP_HIP(hipMemsetAsync(gr.icnt, 0, nl * sizeof(uint32_t), stream));
  GAP_HIP(hipMemsetAsync(gr.esum, 0, nl * sizeof(unsigned long long), stream));
  GroupArgs ga{n, max_depth, depth, rp, gr.cnt, gr.icnt, gr.esum, gr.order, gr.items};
  k_bc_count<<<grid_tiles, kBcBlock, 0, stream>>>(ga);
  GAP_HIP(hipGetLastError());
  GAP_HIP(rocprim::exclusive_scan(scan_tmp, scan_bytes, gr.cnt, gr.off, 0u, nk,
                                  rocprim::plus<uint32_t>(), stream));
  GAP_HIP(rocprim::exclusive_scan(scan_tmp, scan_bytes, gr.icnt, gr.ioff, 0u, nl,
                                  rocprim::plus<uint32_t>(), stream));
  // the counts become cursors starting at each bin's first slot
  GAP_HIP(hipMemcpyAsync(gr.cnt, gr.off, nk * sizeof(uint32_t), hipMemcpyDeviceToDevice, stream));
  GAP_HIP(hipMemcpyAsync(gr.icnt, gr.ioff, nl * sizeof(uint32_t), hipMemcpyDeviceToDevice, stream));
  k_bc_scatter<<<grid_tiles, kBcBlock, 0, stream>>>(ga);
  GAP_HIP(hipGetLastError());
  return GAP_OK;
}

// Per-depth arrays of the groupings for searches of at most max_depth
// levels, carved from the workspace.
static gap_status groupings_for(Workspace *ws, int32_t max_depth, int ngroup, Grouping *gr,
                                size_t vbytes, size_t *nk, size_t *nl, void **scan_tmp,
                                size_t *scan_bytes, hipStream_t stream) {
  *nk = (size_t)(max_depth + 1) * kClasses + 1;
  *nl = (size_t)max_depth + 2;
  auto al = [](size_t bytes) { return (bytes + 255) & ~(size_t)255; };
  *scan_bytes = 0;
  GAP_HIP(rocprim::exclusive_scan(nullptr, *scan_bytes, (uint32_t *)nullptr, (uint32_t *)nullptr,
                                  0u, *nk, rocprim::plus<uint32_t>(), stream));
  gap_status st = workspace_reserve_bc(
      ws, vbytes, ngroup * (2 * al(4 * *nk) + 2 * al(4 * *nl) + al(8 * *nl)) + *scan_bytes + 256);
  if (st != GAP_OK) return st;
  char *q = reinterpret_cast<char *>(ws->bc_lv);
  for (int i = 0; i < ngroup; ++i) {
    gr[i].cnt = carve<uint32_t>(q, *nk);
    gr[i].off = carve<uint32_t>(q, *nk);
    gr[i].icnt = carve<uint32_t>(q, *nl);
    gr[i].ioff = carve<uint32_t>(q, *nl);
    gr[i].esum = carve<unsigned long long>(q, *nl);
  }
  *scan_tmp = q;
  return GAP_OK;
}

// Searches up to this depth are grouped before the host knows the depth
// (the read-back overlaps the grouping); deeper ones are grouped again.
constexpr int32_t kPresizedDepth = 254;

gap_status run_bc(const gap_graph *g, const int32_t *sources, int32_t num_sources, double *score,
                  bool normalise, hipStream_t stream) {
  const DeviceInfo *di = nullptr;
  gap_status st = device_info(g->device, &di);
  if (st != GAP_OK) return st;
  Workspace *ws = workspace_for(g->device, stream);
  if (!ws) {
    set_error("gap_bc: no workspace for the stream");
    return GAP_ENOMEM;
  }
  const int64_t n = g->n;
  const int64_t nwords = (n + 63) / 64;
  const bool directed = g->directed != 0;
  const int ngroup = directed ? 2 : 1;  // in-lists, and out-lists when they differ
  // chunk items: sum over long lists of ceil(deg / kChunk)
  const int64_t cap_items = g->nnz / kChunk + g->nnz / (kLong + 1) + 1;
  const size_t vbytes = 16 * 256 + sizeof(int32_t) * (2 + ngroup) * (size_t)n +
                        sizeof(PathState) * (size_t)n + sizeof(uint64_t) * 4 * (size_t)nwords +
                        sizeof(int2) * (size_t)cap_items * ngroup;
  st = workspace_reserve_bc(ws, vbytes, 0);
  if (st != GAP_OK) return st;
  char *p = reinterpret_cast<char *>(ws->bc_buf);
  int32_t *depth = carve<int32_t>(p, n);
  int32_t *parent = carve<int32_t>(p, n);
  PathState *ps = carve<PathState>(p, n);
  uint64_t *bms = carve<uint64_t>(p, 4 * nwords);
  Grouping gr[2];
  for (int i = 0; i < ngroup; ++i) {
    gr[i].order = carve<int32_t>(p, n);
    gr[i].items = carve<int2>(p, cap_items);
  }
  int32_t *dmax_d = carve<int32_t>(p, 1);
  unsigned long long *top_d = carve<unsigned long long>(p, 1);

  GAP_HIP(hipMemsetAsync(score, 0, sizeof(double) * (size_t)n, stream));
  const gap_params bp = params_current();
  const int grid_v = blocks_for(n, di->cus * 4);
  const int grid_lv = di->cus * 8;
  const int grid_tiles = (int)((n + kTile - 1) / kTile);
  for (int32_t k = 0; k < num_sources; ++k) {
    const int32_t s = sources[k];
    st = run_bfs(g, s, parent, depth, stream, bp, nullptr, 0, nullptr);
    if (st != GAP_OK) return st;
    GAP_HIP(hipMemsetAsync(dmax_d, 0, sizeof(int32_t), stream));
    k_bc_start<<<grid_v, kBcBlock, 0, stream>>>(n, depth, bms, dmax_d);
    GAP_HIP(hipGetLastError());
    // the depth travels to the host while the grouping (sized for
    // kPresizedDepth levels) runs
    int32_t *h = reinterpret_cast<int32_t *>(ws->bc_host);
    GAP_HIP(hipMemcpyAsync(h, dmax_d, sizeof(int32_t), hipMemcpyDeviceToHost, stream));
    GAP_HIP(hipEventRecord(ws->bc_event, stream));
    const int32_t cap = (int32_t)std::min<int64_t>(kPresizedDepth, n - 1);
    size_t nk = 0, nl = 0, scan_bytes = 0;
    void *scan_tmp = nullptr;
    st = groupings_for(ws, cap, ngroup, gr, vbytes, &nk, &nl, &scan_tmp, &scan_bytes, stream);
    if (st != GAP_OK) return st;
    for (int i = 0; i < ngroup; ++i) {
      st = build_grouping(gr[i], n, cap, depth, i == 0 ? g->row_ptr_in : g->row_ptr, nk, nl,
                          scan_tmp, scan_bytes, grid_tiles, stream);
      if (st != GAP_OK) return st;
    }
    GAP_HIP(hipEventSynchronize(ws->bc_event));
    const int32_t D = h[0];
    if (D < 0 || D >= n) {
      set_error("gap_bc: inconsistent depth %d after the search", D);
      return GAP_EINTERNAL;
    }
    if (D > cap) {  // a deep search: group again with room for every level
      st = groupings_for(ws, D, ngroup, gr, vbytes, &nk, &nl, &scan_tmp, &scan_bytes, stream);
      if (st != GAP_OK) return st;
      for (int i = 0; i < ngroup; ++i) {
        st = build_grouping(gr[i], n, D, depth, i == 0 ? g->row_ptr_in : g->row_ptr, nk, nl,
                            scan_tmp, scan_bytes, grid_tiles, stream);
        if (st != GAP_OK) return st;
      }
    }
    const Grouping &gi = gr[0], &go = gr[ngroup - 1];
    LevelArgs la{GroupView{gi.order, gi.off, gi.items, gi.ioff, gi.esum},
                 GroupView{go.order, go.off, go.items, go.ioff, go.esum},
                 g->row_ptr_in, g->row_ptr, g->col_in, g->col, bms, nwords, D, ps};
    k_bc_first<<<grid_v, kBcBlock, 0, stream>>>(la, s);
    for (int32_t d = 1; d <= D; ++d) k_bc_level<true><<<grid_lv, kBcBlock, 0, stream>>>(la, d);
    // the source's own S is never used
    for (int32_t d = D - 1; d >= 1; --d) k_bc_level<false><<<grid_lv, kBcBlock, 0, stream>>>(la, d);
    k_bc_accumulate<<<grid_v, kBcBlock, 0, stream>>>(n, depth, ps, score);
    GAP_HIP(hipGetLastError());
  }
  if (normalise) {
    GAP_HIP(hipMemsetAsync(top_d, 0, sizeof(unsigned long long), stream));
    k_bc_max<<<grid_v, kBcBlock, 0, stream>>>(n, score, top_d);
    k_bc_scale<<<grid_v, kBcBlock, 0, stream>>>(n, score, top_d);
    GAP_HIP(hipGetLastError());
  }
  return GAP_OK;
}

}  // namespace gap
