// Host runtime of libgapbfs: graph handle, device facts, per-stream
// workspaces and the parameter set.  Internal to the library.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdarg>
#include <cstddef>
#include <cstdint>
#include <mutex>
#include <vector>

#include "common.h"

struct gap_graph {
  int device;
  int directed;         // 1: out-lists and in-lists differ
  int64_t n;
  int64_t nnz;          // out-list entries
  int64_t *row_ptr;     // device int64[n+1], out-lists
  int32_t *col;         // device int32[nnz]
  int64_t nnz_in;       // in-list entries (== nnz)
  int64_t *row_ptr_in;  // device in-lists; the same arrays as row_ptr/col when undirected
  int32_t *col_in;
  int64_t max_degree;
  int64_t n_sinks;      // vertices with no out-list entry
  int32_t *wt;          // device int32[nnz] out-list weights, or NULL (every weight 1)
  int32_t max_weight;   // 1 when unweighted
  // First four entries of every list, one 16-byte record per vertex (-1 past
  // the list's end): a search's first read of a list, and the components'
  // sampling, read these records in vertex order instead of one line of
  // `col` per vertex.  head_in == head when undirected.
  int4 *head;           // device int4[n], out-lists
  int4 *head_in;        // device int4[n], in-lists
};

namespace gap {

void set_error(const char *fmt, ...);
void clear_error();

// Maps a HIP error to a status and records a message.
gap_status hip_fail(hipError_t e, const char *what);
#define GAP_HIP(call)                                   \
  do {                                                  \
    hipError_t _e = (call);                             \
    if (_e != hipSuccess) return ::gap::hip_fail(_e, #call); \
  } while (0)

struct DeviceInfo {
  int device = -1;
  int cus = 0;
  int lds_per_cu = 0;
  int lds_per_block = 0;
  int l2_bytes = 0;
  int clock_khz = 0;
  size_t total_mem = 0;
  char arch[64] = {0};
  int coop_supported = 0;
  int xccs = 1;  // accelerator complex dies; workgroups are dealt to them in turn
};

gap_status device_info(int dev, const DeviceInfo **out);

// Per-level record kept on the device when statistics are requested.
struct DevLevelRec {
  int32_t level, direction;
  unsigned long long frontier, frontier_edges, claimed, scanned, unvisited;
  unsigned long long t_start, t_end;  // device real-time clock (100 MHz ticks)
};

// Scratch for searches queued on one (device, stream).  Reused by calls in
// stream order; grown (after a stream synchronisation) when a larger graph
// or a smaller hub/chunk setting needs more room.
struct Workspace {
  int device = -1;
  hipStream_t stream = nullptr;
  // Sticky status of the searches queued on this stream: a kernel that
  // records an error (a timed-out wait, an inconsistent state) also stores
  // it here, where no later search clears it; gap_stream_status reads and
  // clears it.  Device int, allocated with the workspace.
  int *sticky = nullptr;
  // single source
  int64_t cap_n = 0;
  int64_t cap_chunks = 0;
  int32_t *q[2] = {nullptr, nullptr};
  int2 *cq[2] = {nullptr, nullptr};
  uint64_t *bm[3] = {nullptr, nullptr, nullptr};  // frontier A, frontier B, visited
  int32_t *depth_scratch = nullptr;
  // Two control blocks.  The per-level schedules use ctl[0] (reset by a
  // memset before each search).  Persistent searches alternate: search k
  // runs on ctl[k & 1] and its kernel clears the other block, which the
  // search before it has finished with, for search k + 1.
  Ctl *ctl = nullptr;
  uint64_t ctl_seq = 0;          // persistent searches queued
  bool ctl_next_clean = false;   // ctl[ctl_seq & 1] is being or has been cleared
  int *h_flags = nullptr;  // pinned readback of err, levels, done
  void *dd_args = nullptr; // device copy of the per-search arguments
  void *h_args = nullptr;  // pinned staging of the same
  void *graph_exec = nullptr;  // captured level graph (hipGraphExec_t)
  int graph_key = 0, graph_grid = 0;
  DevLevelRec *recs = nullptr;
  int32_t cap_recs = 0;
  // multi-source
  size_t ms_bytes = 0;
  void *ms_buf = nullptr;
  size_t ms_host_bytes = 0;
  void *ms_host = nullptr;  // pinned staging for per-lane metadata
  // betweenness centrality: per-vertex state, per-depth arrays, readback
  size_t bc_bytes = 0;
  void *bc_buf = nullptr;
  size_t bc_lv_bytes = 0;
  void *bc_lv = nullptr;
  void *bc_host = nullptr;  // pinned, 256 bytes
  hipEvent_t bc_event = nullptr;  // marks the depth read-back
  // shortest paths
  size_t sp_bytes = 0;
  void *sp_buf = nullptr;
  void *sp_host = nullptr;  // pinned, 256 bytes
  // connected components
  size_t cc_bytes = 0;
  void *cc_buf = nullptr;
};

// The workspace of (dev, stream), created on first use (NULL when its
// allocation fails).  The caller has made `dev` current.
Workspace *workspace_for(int dev, hipStream_t stream);
// Waits for `stream` and returns (and clears) the first error a kernel
// recorded in the sticky status word of any of its workspaces.
gap_status stream_status(hipStream_t stream);
// Waits for every device the library used and releases every workspace,
// event and captured graph it holds.
void release_all();
gap_status workspace_reserve_single(Workspace *ws, int64_t n, int64_t nnz, const gap_params &p);
gap_status workspace_reserve_recs(Workspace *ws, int32_t nrec);
gap_status workspace_reserve_ms(Workspace *ws, size_t bytes, size_t host_bytes);
gap_status workspace_reserve_bc(Workspace *ws, size_t vertex_bytes, size_t level_bytes);
gap_status workspace_reserve_sssp(Workspace *ws, size_t bytes);
gap_status workspace_reserve_cc(Workspace *ws, size_t bytes);

// Persistent kernels need every workgroup resident at once.  Two of them
// started on different streams could each get part of the machine and wait
// on each other.  With grid_split = k every persistent grid uses at most
// 1/k of the CUs and at most k persistent launches are in flight on the
// device: launch i waits (on the device) for an event recorded after launch
// i-k.  k = 1 orders all persistent launches.  Hold the order from begin to
// end.
struct CoopOrder {
  std::unique_lock<std::mutex> lock;
  int slot = 0;
};
gap_status coop_begin(int dev, hipStream_t s, int k, CoopOrder *o);
gap_status coop_end(int dev, hipStream_t s, CoopOrder *o);
// The same ordering for a launch that may not create events: it joins the
// device's ring as it is (of any size) and orders nothing when no ring
// exists yet.  coop_prepare creates the device's (empty) entry.
void coop_prepare(int dev);
gap_status coop_begin_existing(int dev, hipStream_t s, CoopOrder *o);
gap_status coop_end_existing(int dev, hipStream_t s, CoopOrder *o);

// Launches a kernel whose workgroups wait on each other (grid barriers).
// max_grid is the largest grid that is resident at once on the whole
// device; split = k > 1 takes max_grid / k workgroups rounded down to a
// multiple of the die count, so each die receives the same number.  coop =
// 0: an ordinary launch -- with at most k such grids in flight (the ring of
// coop_begin, which every grid-barrier kernel of the library goes through)
// their sum fits on every die at once, and any other kernel finishes on its
// own; a kernel whose waves need more than kOrdinaryScratchBytes of scratch
// in all is still launched cooperatively (its waves may be limited by
// scratch, not by occupancy).  coop = 1: a cooperative launch (the runtime
// checks residency; cooperative launches do not run concurrently, and each
// costs ~15 us more between consecutive searches).  Waits inside the
// kernels are bounded, so a broken residency assumption ends in
// GAP_ETIMEOUT rather than a hang.
gap_status launch_resident(const void *kern, int max_grid, int block, size_t shmem, void **kargs,
                           int split, int coop, const DeviceInfo *di, hipStream_t s, int *grid_out);

gap_params params_current();
gap_status params_check(const gap_params &p);

// Implemented in bfs.hip
gap_status run_bfs(const gap_graph *g, int32_t source, int32_t *parent, int32_t *depth,
                   hipStream_t stream, const gap_params &p, gap_level_stat *stats,
                   int32_t max_levels, int32_t *num_levels);
// The same search (persistent schedule) with every scratch buffer in a
// file-scope device array of GAP_NOALLOC_SCRATCH_BYTES: no allocation.
gap_status run_bfs_noalloc(const gap_graph *g, int32_t source, int32_t *parent, int32_t *depth,
                           hipStream_t stream);
// Waits for `stream`, then returns and clears the first failure recorded by
// no-allocation searches.
gap_status noalloc_status(hipStream_t stream);
// Implemented in msbfs.hip
gap_status run_bfs_batch(const gap_graph *const *graphs, int32_t num_graphs,
                         const int32_t *graph_of_source, const int32_t *sources,
                         int32_t num_sources, int32_t *const *parents, int32_t *const *depths,
                         hipStream_t stream, const gap_params &p, gap_level_stat *stats,
                         int32_t max_levels, int32_t *num_levels);
// Implemented in bc.hip
gap_status run_bc(const gap_graph *g, const int32_t *sources, int32_t num_sources, double *score,
                  bool normalise, hipStream_t stream);
// Implemented in cc.hip
gap_status run_cc(const gap_graph *g, int32_t *labels, hipStream_t stream);
// Implemented in sssp.hip
gap_status run_sssp(const gap_graph *g, int32_t source, uint32_t *dist, uint32_t delta,
                    hipStream_t stream, int32_t *phases);
// Implemented in build_csr.hip
gap_status build_csr(int64_t n, int64_t m, const int32_t *src, const int32_t *dst,
                     const int32_t *weights, bool directed, hipStream_t stream, gap_graph **out);
gap_status stream_copy(void *dst, const void *src, int64_t bytes, hipStream_t stream);

}  // namespace gap
