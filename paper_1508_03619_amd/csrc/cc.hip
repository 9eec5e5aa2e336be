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
// Lists of up to kLight entries are walked by one lane each; longer lists
// become chunk items of kChunk entries walked by a whole wave.  An
// undirected graph hooks each edge once (from its larger end); a directed
// graph hooks every out-list entry.

#include "runtime.h"

namespace gap {
namespace {

constexpr int kCcBlock = 256;
constexpr int kLight = 32;
constexpr int kChunk = 256;

__global__ __launch_bounds__(kCcBlock) void k_cc_init(int64_t n, int32_t *__restrict__ parent) {
  for (int64_t v = blockIdx.x * (int64_t)kCcBlock + threadIdx.x; v < n;
       v += (int64_t)gridDim.x * kCcBlock)
    parent[v] = (int32_t)v;
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

struct CcArgs {
  int64_t n;
  const int64_t *rp;
  const int32_t *col;
  int32_t *parent;
  int2 *items;
  unsigned int *nitems;
  int directed;
};

// Short lists, one lane each; long lists become chunk items.
__global__ __launch_bounds__(kCcBlock) void k_cc_light(CcArgs a) {
  const int64_t stride = (int64_t)gridDim.x * kCcBlock;
  const int64_t n_round = (a.n + stride - 1) / stride * stride;  // whole waves iterate together
  for (int64_t u = blockIdx.x * (int64_t)kCcBlock + threadIdx.x; u < n_round; u += stride) {
    int64_t beg = 0, deg = 0;
    if (u < a.n) {
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
    if (nch == 0) {
      for (int64_t e = beg; e < beg + deg; ++e) {
        const int32_t v = a.col[e];
        if (v < u || (a.directed && v != u)) hook(a.parent, (int32_t)u, v);
      }
    }
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
    for (int64_t e = beg + lane; e < end; e += kWave) {
      const int32_t v = a.col[e];
      if (v < u || (a.directed && v != u)) hook(a.parent, u, v);
    }
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
  // chunk items: sum over long lists of ceil(deg / kChunk)
  const int64_t cap_items = g->nnz / kChunk + g->nnz / (kLight + 1) + 1;
  st = workspace_reserve_cc(ws, sizeof(int2) * (size_t)cap_items + 512);
  if (st != GAP_OK) return st;
  char *p = reinterpret_cast<char *>(ws->cc_buf);
  CcArgs a{};
  a.n = g->n;
  a.rp = g->row_ptr;
  a.col = g->col;
  a.parent = labels;
  a.nitems = carve<unsigned int>(p, 1);
  a.items = carve<int2>(p, cap_items);
  a.directed = g->directed;
  const int grid = di->cus * 8;
  GAP_HIP(hipMemsetAsync(a.nitems, 0, sizeof(unsigned int), stream));
  k_cc_init<<<grid, kCcBlock, 0, stream>>>(g->n, labels);
  k_cc_light<<<grid, kCcBlock, 0, stream>>>(a);
  k_cc_heavy<<<grid, kCcBlock, 0, stream>>>(a);
  k_cc_compress<<<grid, kCcBlock, 0, stream>>>(g->n, labels);
  GAP_HIP(hipGetLastError());
  return GAP_OK;
}

}  // namespace gap
