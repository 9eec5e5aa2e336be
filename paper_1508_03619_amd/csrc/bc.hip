// Betweenness centrality from a set of sources (Section 2.1, "Betweenness
// Centrality"; Brandes' method as the paper's reference code uses, Section 3).
//
// For each source s:
//   1. a direction-optimizing search (the library's single-source kernel)
//      gives depth[];
//   2. the reached vertices are grouped by depth (counting sort: LDS bins per
//      tile, one global reservation per bin and tile), and every vertex whose
//      list is longer than kLight entries gets chunk items of kChunk entries;
//   3. path counts, level by level away from s, pulled over in-lists:
//        sigma[v] = sum of sigma[u] over in-neighbours u one level up;
//   4. dependencies, level by level towards s, pulled over out-lists.  With
//        S[u] = sum over successors v (out-neighbours one level down) of
//               (1 + delta[v]) / sigma[v] = 1 / sigma[v] + S[v],
//      Brandes' dependency is delta[u] = sigma[u] * S[u], so a level reads
//      only (sigma, S) of the level below and no per-vertex finishing step is
//      needed between levels; chunk items add partial sums atomically;
//   5. score[v] += sigma[v] * S[v] for every reached v != s.
// Finally the scores are divided by the largest one (normalised to one),
// unless the caller asks for raw sums.
//
// Successors are found by their depth, not recorded: the paper keeps a
// successor bitmap to save memory over successor lists; this path keeps no
// per-edge state at all.  fp64 throughout.

#include <rocprim/device/device_scan.hpp>

#include "runtime.h"

namespace gap {
namespace {

constexpr int kBcBlock = 256;
constexpr int kTile = 8192;     // vertices per workgroup in the grouping kernels
constexpr int kLdsBins = 1024;  // depths counted in LDS; deeper ones use global atomics
constexpr int kLight = 32;      // lists up to this long: one lane per vertex
constexpr int kChunk = 512;     // entries per chunk item of a longer list
constexpr int kPerLane = kChunk / kWave;

// Per-vertex state read together by the level below: one 16-byte load.
struct __align__(16) PathState {
  double sigma;  // shortest paths from s
  double s;      // S = delta / sigma
};

__device__ inline double wave_sum_f64(double x) {
  for (int o = 32; o >= 1; o >>= 1) x += __shfl_xor(x, o, kWave);
  return x;
}

__device__ inline uint32_t chunks_of(int64_t deg) {
  return deg > kLight ? (uint32_t)((deg + kChunk - 1) / kChunk) : 0u;
}

// ps <- (s ? 1 : 0, 0); *dmax <- max depth.
__global__ __launch_bounds__(kBcBlock) void k_bc_init(int64_t n, const int32_t *__restrict__ depth,
                                                      int32_t src, PathState *__restrict__ ps,
                                                      int32_t *dmax) {
  int32_t m = 0;
  for (int64_t v = blockIdx.x * (int64_t)kBcBlock + threadIdx.x; v < n;
       v += (int64_t)gridDim.x * kBcBlock) {
    ps[v] = PathState{v == src ? 1.0 : 0.0, 0.0};
    m = max(m, depth[v]);
  }
  for (int o = 32; o >= 1; o >>= 1) m = max(m, __shfl_xor(m, o, kWave));
  if (lane_id() == 0 && m > 0) atomicMax(dmax, m);
}

struct GroupArgs {
  int64_t n;
  const int32_t *depth;
  const int64_t *rp_in, *rp_out;  // rp_out == nullptr: undirected, one item set
  uint32_t *cnt, *icnt_in, *icnt_out;  // per depth: vertices, chunk items
  int32_t *order;
  int2 *items_in, *items_out;
};

// Per depth: number of reached vertices and of chunk items.
__global__ __launch_bounds__(kBcBlock) void k_bc_count(GroupArgs a) {
  __shared__ uint32_t c[kLdsBins], ci[kLdsBins], co[kLdsBins];
  for (int b = threadIdx.x; b < kLdsBins; b += kBcBlock) c[b] = ci[b] = co[b] = 0;
  __syncthreads();
  const int64_t base = (int64_t)blockIdx.x * kTile;
  const int64_t end = min(base + kTile, a.n);
  for (int64_t v = base + threadIdx.x; v < end; v += kBcBlock) {
    const int32_t d = a.depth[v];
    if (d < 0) continue;
    const uint32_t ni = chunks_of(a.rp_in[v + 1] - a.rp_in[v]);
    const uint32_t no = a.rp_out ? chunks_of(a.rp_out[v + 1] - a.rp_out[v]) : 0u;
    if (d < kLdsBins) {
      atomicAdd(&c[d], 1u);
      if (ni) atomicAdd(&ci[d], ni);
      if (no) atomicAdd(&co[d], no);
    } else {
      atomicAdd(&a.cnt[d], 1u);
      if (ni) atomicAdd(&a.icnt_in[d], ni);
      if (no) atomicAdd(&a.icnt_out[d], no);
    }
  }
  __syncthreads();
  for (int b = threadIdx.x; b < kLdsBins; b += kBcBlock) {
    if (c[b]) atomicAdd(&a.cnt[b], c[b]);
    if (ci[b]) atomicAdd(&a.icnt_in[b], ci[b]);
    if (co[b]) atomicAdd(&a.icnt_out[b], co[b]);
  }
}

// Places vertices in order[] and chunk items in items_*[] at the positions
// reserved from the cursors (cnt / icnt_* hold the level starts on entry).
__global__ __launch_bounds__(kBcBlock) void k_bc_scatter(GroupArgs a) {
  __shared__ uint32_t c[kLdsBins], ci[kLdsBins], co[kLdsBins];
  __shared__ uint32_t b0[kLdsBins], bi[kLdsBins], bo[kLdsBins];
  for (int b = threadIdx.x; b < kLdsBins; b += kBcBlock) c[b] = ci[b] = co[b] = 0;
  __syncthreads();
  const int64_t base = (int64_t)blockIdx.x * kTile;
  const int64_t end = min(base + kTile, a.n);
  for (int64_t v = base + threadIdx.x; v < end; v += kBcBlock) {
    const int32_t d = a.depth[v];
    if (d < 0 || d >= kLdsBins) continue;
    const uint32_t ni = chunks_of(a.rp_in[v + 1] - a.rp_in[v]);
    const uint32_t no = a.rp_out ? chunks_of(a.rp_out[v + 1] - a.rp_out[v]) : 0u;
    atomicAdd(&c[d], 1u);
    if (ni) atomicAdd(&ci[d], ni);
    if (no) atomicAdd(&co[d], no);
  }
  __syncthreads();
  for (int b = threadIdx.x; b < kLdsBins; b += kBcBlock) {
    b0[b] = c[b] ? atomicAdd(&a.cnt[b], c[b]) : 0u;
    bi[b] = ci[b] ? atomicAdd(&a.icnt_in[b], ci[b]) : 0u;
    bo[b] = co[b] ? atomicAdd(&a.icnt_out[b], co[b]) : 0u;
    c[b] = ci[b] = co[b] = 0;  // reused as in-tile cursors
  }
  __syncthreads();
  for (int64_t v = base + threadIdx.x; v < end; v += kBcBlock) {
    const int32_t d = a.depth[v];
    if (d < 0) continue;
    const uint32_t ni = chunks_of(a.rp_in[v + 1] - a.rp_in[v]);
    const uint32_t no = a.rp_out ? chunks_of(a.rp_out[v + 1] - a.rp_out[v]) : 0u;
    uint32_t pos, ipos = 0, opos = 0;
    if (d < kLdsBins) {
      pos = b0[d] + atomicAdd(&c[d], 1u);
      if (ni) ipos = bi[d] + atomicAdd(&ci[d], ni);
      if (no) opos = bo[d] + atomicAdd(&co[d], no);
    } else {
      pos = atomicAdd(&a.cnt[d], 1u);
      if (ni) ipos = atomicAdd(&a.icnt_in[d], ni);
      if (no) opos = atomicAdd(&a.icnt_out[d], no);
    }
    a.order[pos] = (int32_t)v;
    for (uint32_t k = 0; k < ni; ++k) a.items_in[ipos + k] = make_int2((int)v, (int)k);
    for (uint32_t k = 0; k < no; ++k) a.items_out[opos + k] = make_int2((int)v, (int)k);
  }
}

struct LevelArgs {
  const int32_t *order;
  const uint32_t *off;   // level starts in order[], [D + 2]
  const int2 *items;
  const uint32_t *ioff;  // level starts in items[], [D + 2]
  const int64_t *rp;     // in-lists (forward) or out-lists (backward)
  const int32_t *col;
  const int32_t *depth;
  PathState *ps;
};

// One level.  FORWARD: sigma of level d from level d - 1 over in-lists.
// Backward: S of level d from level d + 1 over out-lists.  Wave tasks: first
// the level's vertices 64 at a time (one lane each, lists up to kLight), then
// one chunk item each.
template <bool FORWARD>
__global__ __launch_bounds__(kBcBlock) void k_bc_level(LevelArgs a, int32_t d) {
  const uint32_t lo = a.off[d], nv = a.off[d + 1] - lo;
  const uint32_t ilo = a.ioff[d], ni = a.ioff[d + 1] - ilo;
  const uint32_t ntl = (nv + kWave - 1) / kWave;
  const uint32_t total = ntl + ni;
  const int lane = lane_id();
  const uint32_t nw = gridDim.x * (kBcBlock / kWave);
  const int32_t want = FORWARD ? d - 1 : d + 1;
  for (uint32_t t = blockIdx.x * (kBcBlock / kWave) + threadIdx.x / kWave; t < total; t += nw) {
    if (t < ntl) {
      const uint32_t i = t * kWave + lane;
      int32_t v = -1;
      int64_t beg = 0;
      int32_t deg = 0;
      if (i < nv) {
        v = a.order[lo + i];
        beg = a.rp[v];
        deg = (int32_t)(a.rp[v + 1] - beg);
        if (deg > kLight) v = -1;  // covered by its chunk items
      }
      if (v < 0) continue;
      double acc = 0.0;
      for (int k = 0; k < deg; k += 4) {
        int32_t u[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) u[j] = k + j < deg ? a.col[beg + k + j] : -1;
        bool hit[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) hit[j] = u[j] >= 0 && a.depth[u[j]] == want;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          if (!hit[j]) continue;
          if (FORWARD) {
            acc += a.ps[u[j]].sigma;
          } else {
            const PathState q = a.ps[u[j]];
            acc += 1.0 / q.sigma + q.s;
          }
        }
      }
      if (FORWARD)
        a.ps[v].sigma = acc;
      else
        a.ps[v].s = acc;
    } else {
      const int2 it = a.items[ilo + (t - ntl)];
      const int32_t v = it.x;
      const int64_t beg = a.rp[v] + (int64_t)it.y * kChunk;
      const int64_t end = min(beg + (int64_t)kChunk, a.rp[v + 1]);
      int32_t u[kPerLane];
#pragma unroll
      for (int j = 0; j < kPerLane; ++j) {
        const int64_t e = beg + j * kWave + lane;
        u[j] = e < end ? a.col[e] : -1;
      }
      bool hit[kPerLane];
#pragma unroll
      for (int j = 0; j < kPerLane; ++j) hit[j] = u[j] >= 0 && a.depth[u[j]] == want;
      double acc = 0.0;
#pragma unroll
      for (int j = 0; j < kPerLane; ++j) {
        if (!hit[j]) continue;
        if (FORWARD) {
          acc += a.ps[u[j]].sigma;
        } else {
          const PathState q = a.ps[u[j]];
          acc += 1.0 / q.sigma + q.s;
        }
      }
      acc = wave_sum_f64(acc);
      if (lane == 0 && acc != 0.0) unsafeAtomicAdd(FORWARD ? &a.ps[v].sigma : &a.ps[v].s, acc);
    }
  }
}

// score[v] += sigma[v] * S[v] for the reached vertices after the source.
__global__ __launch_bounds__(kBcBlock) void k_bc_accumulate(const int32_t *__restrict__ order,
                                                            const uint32_t *__restrict__ off,
                                                            int32_t dmax, const PathState *__restrict__ ps,
                                                            double *__restrict__ score) {
  const uint32_t lo = off[1], hi = off[dmax + 1];
  for (uint32_t i = lo + blockIdx.x * kBcBlock + threadIdx.x; i < hi; i += gridDim.x * kBcBlock) {
    const int32_t v = order[i];
    const PathState q = ps[v];
    score[v] += q.sigma * q.s;
  }
}

// Scores are non-negative, so their IEEE bit patterns order like the values.
__global__ __launch_bounds__(kBcBlock) void k_bc_max(int64_t n, const double *__restrict__ score,
                                                     unsigned long long *top) {
  unsigned long long m = 0;
  for (int64_t v = blockIdx.x * (int64_t)kBcBlock + threadIdx.x; v < n;
       v += (int64_t)gridDim.x * kBcBlock)
    m = max(m, (unsigned long long)__double_as_longlong(score[v]));
  for (int o = 32; o >= 1; o >>= 1) m = max(m, (unsigned long long)__shfl_xor(m, o, kWave));
  if (lane_id() == 0 && m) atomicMax(top, m);
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
  const bool directed = g->directed != 0;
  // chunk items: sum over long lists of ceil(deg / kChunk)
  const int64_t cap_items = g->nnz / kChunk + g->nnz / (kLight + 1) + 1;
  const size_t vbytes = 4 * 256 + sizeof(int32_t) * 3 * (size_t)n + sizeof(PathState) * (size_t)n +
                        sizeof(int2) * (size_t)cap_items * (directed ? 2 : 1) + 6 * 256;
  st = workspace_reserve_bc(ws, vbytes, 0);
  if (st != GAP_OK) return st;
  char *p = reinterpret_cast<char *>(ws->bc_buf);
  int32_t *depth = carve<int32_t>(p, n);
  int32_t *parent = carve<int32_t>(p, n);
  int32_t *order = carve<int32_t>(p, n);
  PathState *ps = carve<PathState>(p, n);
  int2 *items_in = carve<int2>(p, cap_items);
  int2 *items_out = directed ? carve<int2>(p, cap_items) : items_in;
  int32_t *dmax_d = carve<int32_t>(p, 1);
  unsigned long long *top_d = carve<unsigned long long>(p, 1);

  GAP_HIP(hipMemsetAsync(score, 0, sizeof(double) * (size_t)n, stream));
  const gap_params bp = params_current();
  const int grid_v = blocks_for(n, di->cus * 16);
  const int grid_lv = di->cus * 8;
  const int grid_tiles = (int)((n + kTile - 1) / kTile);
  for (int32_t k = 0; k < num_sources; ++k) {
    const int32_t s = sources[k];
    st = run_bfs(g, s, parent, depth, stream, bp, nullptr, 0, nullptr);
    if (st != GAP_OK) return st;
    GAP_HIP(hipMemsetAsync(dmax_d, 0, sizeof(int32_t), stream));
    k_bc_init<<<grid_v, kBcBlock, 0, stream>>>(n, depth, s, ps, dmax_d);
    GAP_HIP(hipGetLastError());
    int32_t *h = reinterpret_cast<int32_t *>(ws->bc_host);
    GAP_HIP(hipMemcpyAsync(h, dmax_d, sizeof(int32_t), hipMemcpyDeviceToHost, stream));
    GAP_HIP(hipStreamSynchronize(stream));
    const int32_t D = h[0];
    if (D < 0 || D >= n) {
      set_error("gap_bc: inconsistent depth %d after the search", D);
      return GAP_EINTERNAL;
    }
    // per-depth arrays: counts (then cursors) and their scans, D + 2 entries
    const size_t nl = (size_t)D + 2;
    size_t scan_bytes = 0;
    GAP_HIP(rocprim::exclusive_scan(nullptr, scan_bytes, (uint32_t *)nullptr, (uint32_t *)nullptr,
                                    0u, nl, rocprim::plus<uint32_t>(), stream));
    st = workspace_reserve_bc(ws, vbytes,
                              6 * ((nl * sizeof(uint32_t) + 255) & ~(size_t)255) + scan_bytes + 256);
    if (st != GAP_OK) return st;
    char *q = reinterpret_cast<char *>(ws->bc_lv);
    uint32_t *cnt = carve<uint32_t>(q, nl);
    uint32_t *icnt_in = carve<uint32_t>(q, nl);
    uint32_t *icnt_out = carve<uint32_t>(q, nl);
    uint32_t *off = carve<uint32_t>(q, nl);
    uint32_t *ioff_in = carve<uint32_t>(q, nl);
    uint32_t *ioff_out = directed ? carve<uint32_t>(q, nl) : ioff_in;
    void *scan_tmp = q;
    GAP_HIP(hipMemsetAsync(cnt, 0, 3 * ((nl * sizeof(uint32_t) + 255) & ~(size_t)255), stream));
    GroupArgs ga{n, depth, g->row_ptr_in, directed ? g->row_ptr : nullptr, cnt, icnt_in, icnt_out,
                 order, items_in, items_out};
    k_bc_count<<<grid_tiles, kBcBlock, 0, stream>>>(ga);
    GAP_HIP(hipGetLastError());
    GAP_HIP(rocprim::exclusive_scan(scan_tmp, scan_bytes, cnt, off, 0u, nl,
                                    rocprim::plus<uint32_t>(), stream));
    GAP_HIP(rocprim::exclusive_scan(scan_tmp, scan_bytes, icnt_in, ioff_in, 0u, nl,
                                    rocprim::plus<uint32_t>(), stream));
    if (directed)
      GAP_HIP(rocprim::exclusive_scan(scan_tmp, scan_bytes, icnt_out, ioff_out, 0u, nl,
                                      rocprim::plus<uint32_t>(), stream));
    // the counts become cursors starting at each level's first slot
    GAP_HIP(hipMemcpyAsync(cnt, off, nl * sizeof(uint32_t), hipMemcpyDeviceToDevice, stream));
    GAP_HIP(hipMemcpyAsync(icnt_in, ioff_in, nl * sizeof(uint32_t), hipMemcpyDeviceToDevice, stream));
    if (directed)
      GAP_HIP(hipMemcpyAsync(icnt_out, ioff_out, nl * sizeof(uint32_t), hipMemcpyDeviceToDevice,
                             stream));
    k_bc_scatter<<<grid_tiles, kBcBlock, 0, stream>>>(ga);
    GAP_HIP(hipGetLastError());
    LevelArgs fa{order, off, items_in, ioff_in, g->row_ptr_in, g->col_in, depth, ps};
    for (int32_t d = 1; d <= D; ++d) k_bc_level<true><<<grid_lv, kBcBlock, 0, stream>>>(fa, d);
    LevelArgs ba{order, off, items_out, ioff_out, g->row_ptr, g->col, depth, ps};
    for (int32_t d = D - 1; d >= 0; --d) k_bc_level<false><<<grid_lv, kBcBlock, 0, stream>>>(ba, d);
    k_bc_accumulate<<<grid_v, kBcBlock, 0, stream>>>(order, off, D, ps, score);
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
