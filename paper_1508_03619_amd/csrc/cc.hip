// Connected components (Section 2.1, "CC": weak components of a directed
// graph; each vertex labelled with its component) by lock-free union-find,
// one pass over the edges.
//
// The label array is the union-find forest.  Every edge {u, v} hooks the
// larger of the two roots under the smaller with a compare-and-swap, so a
// tree's root is always its smallest vertex and no cycle can form; finds
// halve the paths they walk.  A final pass points every vertex at its root,
// so the label of a vertex is the smallest vertex of its component (the
// paper's reference code uses Shiloach-Vishkin hooking and shortcutting
// rounds; one pass of hooking on roots reaches the same partition without
// the rounds).  The final pass walks without writing, so each vertex's root
// pointer is stored by its own thread only.  Stale reads of a parent are
// harmless: a vertex that is not a root never becomes one again, so a stale
// value still names an ancestor, and a hook on a vertex that stopped being
// a root fails its compare-and-swap and retries from the fresh value.
//
// Most edges need no hook: they join vertices already in one tree.  So the
// edges are taken in two steps (the sampling scheme of GPU union-find
// codes): first every vertex is hooked to its first kSampleRounds list
// entries (where they are smaller than it) and the forest is flattened
// after each round.  These sampling links are plain stores, not
// compare-and-swaps: concurrent links of one root overwrite each other, so
// some are lost, but every stored pointer goes to a smaller vertex of the
// same component, so the forest stays acyclic and sound, and the pass
// that follows is complete on its own.  (A compare-and-swap round here
// took over a millisecond at scale 22: the dies' L2 copies of a root
// stayed stale after a memory-side swap, so most swaps failed and retried
// on a few hot roots.)  The most frequent root among
// kSample spread-out vertices names the giant tree (found on the device,
// so the call never waits for the host); then only vertices
// outside it walk their lists (all entries, and for a directed graph its
// in-list too, so an edge from the giant tree into a small one is seen
// from the small end).  Skipping the giant tree's vertices is safe for any
// choice of it: an edge to a vertex outside it is hooked from that end.
// Lists of up to kLight entries are walked by one lane each; longer lists
// become chunk items of kChunk entries walked by a whole wave.

#include "runtime.h"

namespace gap {
namespace {

constexpr int kCcBlock = 256;
constexpr int kLight = 32;
constexpr int kChunk = 256;
#ifndef GAP_CC_SAMPLE_ROUNDS
#define GAP_CC_SAMPLE_ROUNDS 2
#endif
constexpr int kSampleRounds = GAP_CC_SAMPLE_ROUNDS;
constexpr int kSample = 1024;

// First sampling round fused with the initialisation: each vertex starts
// as its own root and is hooked under its first list entry (the smallest
// neighbour, lists being ascending) when that is smaller.  No other thread
// writes parent[v] here, and parents only decrease, so no cycle forms.
// The first entries come from the graph's 16-byte head records (read in
// vertex order), not from one line of the column array per vertex.
__global__ __launch_bounds__(kCcBlock) void k_cc_init(int64_t n, const int4 *__restrict__ head,
                                                      int32_t *__restrict__ parent) {
  for (int64_t v = blockIdx.x * (int64_t)kCcBlock + threadIdx.x; v < n;
       v += (int64_t)gridDim.x * kCcBlock) {
    const int32_t h = head[v].x;
    const int32_t first = h >= 0 ? h : (int32_t)v;
    parent[v] = first < (int32_t)v ? first : (int32_t)v;
  }
}

__device__ inline int32_t find_root(int32_t *parent, int32_t x) {
  for (;;) {
    const int32_t p = parent[x];
    if (p == x) return x;
    const int32_t gp = parent[p];
    if (gp == p) return p;
    parent[x] = gp;  // path halving
    x = gp;
  }
}

__device__ inline void hook(int32_t *parent, int32_t u, int32_t v) {
  int32_t ru = find_root(parent, u), rv = find_root(parent, v);
  while (ru != rv) {
    if (ru < rv) {
      const int32_t t = ru;
      ru = rv;
      rv = t;
    }
    // ru > rv: the larger root goes under the smaller
    const int32_t old = atomicCAS(&parent[ru], ru, rv);
    if (old == ru) return;
    ru = find_root(parent, old);
    rv = find_root(parent, rv);
  }
}

// A sampling link: the larger of the two roots is pointed at the smaller
// with a plain store (one attempt; a lost race loses the link).
__device__ inline void link_sample(int32_t *parent, int32_t u, int32_t v) {
  const int32_t ru = find_root(parent, u), rv = find_root(parent, v);
  if (ru > rv)
    parent[ru] = rv;
  else if (rv > ru)
    parent[rv] = ru;
}

struct CcArgs {
  int64_t n;
  const int64_t *rp;
  const int32_t *col;
  int32_t *parent;
  int2 *items;
  unsigned int *nitems;
  const int32_t *skip;  // vertices whose root is *skip do not walk their lists
};

// Sampling round r >= 1: vertex u linked to list entry r when it is
// smaller than u (lists are ascending, so a vertex whose entries are larger
// is a local minimum and is left for its neighbours to find).
__global__ __launch_bounds__(kCcBlock) void k_cc_sample(int64_t n, const int64_t *__restrict__ rp,
                                                        const int32_t *__restrict__ col,
                                                        const int4 *__restrict__ head,
                                                        int32_t *parent, int r) {
  for (int64_t u = blockIdx.x * (int64_t)kCcBlock + threadIdx.x; u < n;
       u += (int64_t)gridDim.x * kCcBlock) {
    int32_t v = -1;
    if (r < 4) {  // in the head record (-1 past the list's end)
      const int4 h = head[u];
      v = r == 1 ? h.y : (r == 2 ? h.z : h.w);
    } else {
      const int64_t beg = rp[u], deg = rp[u + 1] - beg;
      if (r < deg) v = col[beg + r];
    }
    if (v >= 0 && v < u) link_sample(parent, (int32_t)u, v);
  }
}

// Short lists of vertices outside the giant tree, one lane each; long
// lists become chunk items.
__global__ __launch_bounds__(kCcBlock) void k_cc_light(CcArgs a) {
  const int32_t giant = *a.skip;
  const int64_t stride = (int64_t)gridDim.x * kCcBlock;
  const int64_t n_round = (a.n + stride - 1) / stride * stride;  // whole waves iterate together
  for (int64_t u = blockIdx.x * (int64_t)kCcBlock + threadIdx.x; u < n_round; u += stride) {
    int64_t beg = 0, deg = 0;
    if (u < a.n && find_root(a.parent, (int32_t)u) != giant) {
      beg = a.rp[u];
      deg = a.rp[u + 1] - beg;
    }
    const uint32_t nch = deg > kLight ? (uint32_t)((deg + kChunk - 1) / kChunk) : 0u;
    uint32_t total = 0;
    const uint32_t off = wave_excl_scan_u32(nch, total);
    if (total) {
      uint32_t base = 0;
      if (lane_id() == 0) base = atomicAdd(a.nitems, total);
      base = __shfl(base, 0, kWave);
      for (uint32_t k = 0; k < nch; ++k) a.items[base + off + k] = make_int2((int)u, (int)k);
    }
    if (nch == 0)
      for (int64_t e = beg; e < beg + deg; ++e) hook(a.parent, (int32_t)u, a.col[e]);
  }
}

// One chunk item per wave.
__global__ __launch_bounds__(kCcBlock) void k_cc_heavy(CcArgs a) {
  const uint32_t ni = *a.nitems;
  const int lane = lane_id();
  const uint32_t nw = gridDim.x * (kCcBlock / kWave);
  for (uint32_t t = blockIdx.x * (kCcBlock / kWave) + threadIdx.x / kWave; t < ni; t += nw) {
    const int2 it = a.items[t];
    const int32_t u = it.x;
    const int64_t beg = a.rp[u] + (int64_t)it.y * kChunk;
    const int64_t end = min(beg + (int64_t)kChunk, a.rp[u + 1]);
    for (int64_t e = beg + lane; e < end; e += kWave) hook(a.parent, u, a.col[e]);
  }
}

// The giant tree: the most frequent root among kSample vertices spread over
// the vertex range (the smallest such root on a tie), by one workgroup:
// the roots are sorted in LDS (bitonic network), the thread at the start
// of each run finds the run's end by bisection, and a block maximum over
// (run length, -root) keeps the winner.
// Thread 0 also clears the two chunk-item counters of the passes that
// follow (a kernel, not a memset, so the call can be captured in a graph).
__global__ __launch_bounds__(kSample) void k_cc_pick(int64_t n, const int32_t *__restrict__ parent,
                                                     int32_t *giant, unsigned int *nitems) {
  __shared__ int32_t key[kSample];
  __shared__ unsigned long long wbest[kSample / kWave];
  const int t = threadIdx.x;
  key[t] = parent[(int64_t)(((uint64_t)t * 2654435761ull + 12345ull) % (uint64_t)n)];
  __syncthreads();
  for (int k = 2; k <= kSample; k <<= 1)
    for (int j = k >> 1; j > 0; j >>= 1) {
      const int p = t ^ j;
      if (p > t) {
        const int32_t x = key[t], y = key[p];
        if ((x > y) == ((t & k) == 0)) {
          key[t] = y;
          key[p] = x;
        }
      }
      __syncthreads();
    }
  unsigned long long best = 0;
  if (t == 0 || key[t - 1] != key[t]) {
    int lo = t, hi = kSample;  // key[lo] == key[t]; hi == kSample or key[hi] != key[t]
    while (hi - lo > 1) {
      const int mid = (lo + hi) >> 1;
      if (key[mid] == key[t])
        lo = mid;
      else
        hi = mid;
    }
    best = ((unsigned long long)(hi - t) << 32) | (uint32_t)(INT32_MAX - key[t]);
  }
  for (int o = kWave / 2; o >= 1; o >>= 1) {
    const unsigned long long other = __shfl_xor(best, o, kWave);
    best = other > best ? other : best;
  }
  if (lane_id() == 0) wbest[t / kWave] = best;
  __syncthreads();
  if (t == 0) {
    for (int w = 1; w < kSample / kWave; ++w) best = wbest[w] > best ? wbest[w] : best;
    *giant = INT32_MAX - (int32_t)(uint32_t)best;
    nitems[0] = 0;
    nitems[1] = 0;
  }
}

// Every vertex points at its root: the smallest vertex of its component.
// The walk only reads: a halving store by a walker passing through v could
// otherwise land after v's own thread stored the root and leave v pointing
// at an ancestor that is not the root.
__global__ __launch_bounds__(kCcBlock) void k_cc_compress(int64_t n, int32_t *__restrict__ parent) {
  for (int64_t v = blockIdx.x * (int64_t)kCcBlock + threadIdx.x; v < n;
       v += (int64_t)gridDim.x * kCcBlock) {
    int32_t x = (int32_t)v, p = parent[x];
    while (p != x) {
      x = p;
      p = parent[x];
    }
    parent[v] = x;
  }
}

template <class T>
T *carve(char *&p, size_t count) {
  T *r = reinterpret_cast<T *>(p);
  p += (sizeof(T) * count + 255) & ~(size_t)255;
  return r;
}

}  // namespace

gap_status run_cc(const gap_graph *g, int32_t *labels, hipStream_t stream) {
  const DeviceInfo *di = nullptr;
  gap_status st = device_info(g->device, &di);
  if (st != GAP_OK) return st;
  Workspace *ws = workspace_for(g->device, stream);
  if (!ws) {
    set_error("gap_cc: no workspace for the stream");
    return GAP_ENOMEM;
  }
  // chunk items: sum over long lists of ceil(deg / kChunk), per list set
  const int64_t cap_items = g->nnz / kChunk + g->nnz / (kLight + 1) + 1;
  st = workspace_reserve_cc(ws, sizeof(int2) * (size_t)cap_items + 1024);
  if (st != GAP_OK) return st;
  char *p = reinterpret_cast<char *>(ws->cc_buf);
  unsigned int *nitems = carve<unsigned int>(p, 2);  // one per pass
  int32_t *giant = carve<int32_t>(p, 1);
  int2 *items = carve<int2>(p, cap_items);
  const int grid = di->cus * 8;
  const int64_t n = g->n;
  k_cc_init<<<grid, kCcBlock, 0, stream>>>(n, g->head, labels);
  k_cc_compress<<<grid, kCcBlock, 0, stream>>>(n, labels);
  for (int r = 1; r < kSampleRounds; ++r) {
    k_cc_sample<<<grid, kCcBlock, 0, stream>>>(n, g->row_ptr, g->col, g->head, labels, r);
    k_cc_compress<<<grid, kCcBlock, 0, stream>>>(n, labels);
  }
  k_cc_pick<<<1, kSample, 0, stream>>>(n, labels, giant, nitems);
  // the lists of the vertices outside the giant tree: out-lists, and the
  // in-lists of a directed graph
  const int passes = g->directed ? 2 : 1;
  for (int pass = 0; pass < passes; ++pass) {
    CcArgs a{};
    a.n = n;
    a.rp = pass == 0 ? g->row_ptr : g->row_ptr_in;
    a.col = pass == 0 ? g->col : g->col_in;
    a.parent = labels;
    a.items = items;
    a.nitems = nitems + pass;
    a.skip = giant;
    k_cc_light<<<grid, kCcBlock, 0, stream>>>(a);
    k_cc_heavy<<<grid, kCcBlock, 0, stream>>>(a);
  }
  k_cc_compress<<<grid, kCcBlock, 0, stream>>>(n, labels);
  GAP_HIP(hipGetLastError());
  return GAP_OK;
}

}  // namespace gap
