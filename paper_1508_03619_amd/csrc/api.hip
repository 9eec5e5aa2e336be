// C ABI of libgapbfs and its host runtime: errors, device facts, per-stream
// workspaces, the parameter set.
#include <cstdio>
#include <algorithm>
#include <cstring>
#include <map>
#include <memory>
#include <new>
#include <string>
#include <vector>

#include "runtime.h"

namespace gap {

static thread_local std::string t_error;

void set_error(const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  t_error = buf;
}

void clear_error() { t_error.clear(); }

gap_status hip_fail(hipError_t e, const char *what) {
  set_error("%s: %s", what, hipGetErrorString(e));
  if (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation) return GAP_ENOMEM;
  return GAP_EDEVICE;
}

// ---- device facts ---------------------------------------------------------------

static std::mutex g_mu;
static std::map<int, DeviceInfo> g_dev;

gap_status device_info(int dev, const DeviceInfo **out) {
  std::lock_guard<std::mutex> lk(g_mu);
  auto it = g_dev.find(dev);
  if (it == g_dev.end()) {
    hipDeviceProp_t prop;
    GAP_HIP(hipGetDeviceProperties(&prop, dev));
    DeviceInfo di;
    di.device = dev;
    di.cus = prop.multiProcessorCount;
    di.lds_per_cu = (int)prop.maxSharedMemoryPerMultiProcessor;
    di.lds_per_block = (int)prop.sharedMemPerBlock;
    di.l2_bytes = prop.l2CacheSize;
    di.clock_khz = prop.clockRate;
    di.total_mem = prop.totalGlobalMem;
    di.coop_supported = prop.cooperativeLaunch;
    int xccs = 1;
    if (hipDeviceGetAttribute(&xccs, hipDeviceAttributeNumberOfXccs, dev) != hipSuccess || xccs < 1)
      xccs = 1;
    (void)hipGetLastError();
    di.xccs = xccs;
    snprintf(di.arch, sizeof(di.arch), "%s", prop.gcnArchName);
    it = g_dev.emplace(dev, di).first;
  }
  *out = &it->second;
  return GAP_OK;
}

// ---- ordering of persistent launches across streams ------------------------------

struct CoopState {
  std::mutex mu;
  std::vector<hipEvent_t> ev;      // ring of k events
  std::vector<bool> recorded;
  std::vector<hipStream_t> on;     // stream of the launch each event follows
  int k = 0;
  unsigned long long next = 0;     // launches ordered so far
};
static std::map<int, std::unique_ptr<CoopState>> g_coop;

static CoopState *coop_state(int dev) {
  std::lock_guard<std::mutex> lk(g_mu);
  auto &p = g_coop[dev];
  if (!p) p.reset(new CoopState());
  return p.get();
}

gap_status coop_begin(int dev, hipStream_t s, int k, CoopOrder *o) {
  CoopState *cs = coop_state(dev);
  o->lock = std::unique_lock<std::mutex>(cs->mu);
  if (k < 1) k = 1;
  // a launch queued earlier on the same stream is ordered by the stream
  // itself: no wait is queued for it
  if (cs->k != k) {
    // a new ring size: the first launch waits for every launch of the old ring
    for (size_t i = 0; i < cs->ev.size(); ++i)
      if (cs->recorded[i] && cs->on[i] != s) GAP_HIP(hipStreamWaitEvent(s, cs->ev[i], 0));
    for (hipEvent_t e : cs->ev) (void)hipEventDestroy(e);
    cs->ev.assign((size_t)k, nullptr);
    cs->recorded.assign((size_t)k, false);
    cs->on.assign((size_t)k, nullptr);
    for (auto &e : cs->ev) GAP_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    cs->k = k;
    cs->next = 0;
  }
  o->slot = (int)(cs->next % (unsigned long long)k);
  const size_t i = (size_t)o->slot;
  if (cs->recorded[i] && cs->on[i] != s) GAP_HIP(hipStreamWaitEvent(s, cs->ev[i], 0));
  return GAP_OK;
}

void coop_prepare(int dev) { (void)coop_state(dev); }

gap_status coop_begin_existing(int dev, hipStream_t s, CoopOrder *o) {
  CoopState *cs = coop_state(dev);
  o->lock = std::unique_lock<std::mutex>(cs->mu);
  if (cs->k < 1) {
    o->slot = -1;
    return GAP_OK;
  }
  o->slot = (int)(cs->next % (unsigned long long)cs->k);
  const size_t i = (size_t)o->slot;
  if (cs->recorded[i] && cs->on[i] != s) GAP_HIP(hipStreamWaitEvent(s, cs->ev[i], 0));
  return GAP_OK;
}

gap_status coop_end_existing(int dev, hipStream_t s, CoopOrder *o) {
  if (o->slot < 0) {
    o->lock.unlock();
    return GAP_OK;
  }
  return coop_end(dev, s, o);
}

gap_status coop_end(int dev, hipStream_t s, CoopOrder *o) {
  CoopState *cs = coop_state(dev);
  hipError_t e = hipEventRecord(cs->ev[(size_t)o->slot], s);
  cs->recorded[(size_t)o->slot] = (e == hipSuccess);
  cs->on[(size_t)o->slot] = s;
  cs->next += 1;
  o->lock.unlock();
  if (e != hipSuccess) return hip_fail(e, "hipEventRecord");
  return GAP_OK;
}

// Private (scratch) bytes per lane of a kernel, cached.  Scratch is granted
// per wave: a grid whose waves need a large total may have fewer waves
// resident than its occupancy says, so an ordinary launch relies on
// residency only below kOrdinaryScratchBytes for the whole grid.
static size_t kernel_scratch(const void *kern) {
  static std::mutex mu;
  static std::map<const void *, size_t> cache;
  std::lock_guard<std::mutex> lk(mu);
  auto it = cache.find(kern);
  if (it != cache.end()) return it->second;
  hipFuncAttributes attr{};
  size_t bytes = 1;  // unknown: treat as spilling
  if (hipFuncGetAttributes(&attr, kern) == hipSuccess) bytes = attr.localSizeBytes;
  (void)hipGetLastError();
  cache.emplace(kern, bytes);
  return bytes;
}

constexpr size_t kOrdinaryScratchBytes = 256ull << 20;

gap_status launch_resident(const void *kern, int max_grid, int block, size_t shmem, void **kargs,
                           int split, int coop, const DeviceInfo *di, hipStream_t s, int *grid_out) {
  int grid = max_grid;
  if (split > 1) {
    const int x = di->xccs;
    grid = max_grid / split / x * x;
    if (grid < x) grid = max_grid / split;
    if (grid < 1) grid = 1;
  }
  const size_t scratch = kernel_scratch(kern) * (size_t)block * (size_t)grid;
  if (!coop && scratch <= kOrdinaryScratchBytes) {
    // an ordinary launch: the grid is sized to be resident, and the
    // device's launch ring (coop_begin) keeps the library's grid-barrier
    // kernels from running more than `split` at once; the barriers' bounded
    // waits turn a broken assumption into GAP_ETIMEOUT
    GAP_HIP(hipLaunchKernel(kern, dim3(grid), dim3(block), kargs, shmem, s));
  } else {
    // the runtime checks residency (and such launches do not overlap)
    GAP_HIP(hipLaunchCooperativeKernel(kern, dim3(grid), dim3(block), kargs, (unsigned int)shmem, s));
  }
  if (grid_out) *grid_out = grid;
  return GAP_OK;
}

// ---- parameters --------------------------------------------------------------------

static gap_params default_params() {
  gap_params p;
  memset(&p, 0, sizeof(p));
  p.mode = GAP_MODE_PERSISTENT;
  p.direction = GAP_DIR_AUTO;
  p.alpha = 15;
  p.beta = 128;
  p.block = 1024;
  p.blocks_per_cu = 1;
  p.hub_degree = 256;
  p.chunk_edges = 256;
  p.graph_chunk = 16;
  p.batch_mode = 0;
  p.batch_alpha = 8;
  p.batch_beta = 18;
  p.grid_split = 1;
  p.small_frontier = 32768;
  p.lds_bitmap = 1;
  p.bu_mapping = 0;
  p.batch_words = 4;
  p.serve_window_us = 5000;
  p.td_plain = 8;
  p.coop_launch = 0;
  return p;
}

static gap_params g_params = default_params();

gap_params params_current() {
  std::lock_guard<std::mutex> lk(g_mu);
  return g_params;
}

gap_status params_check(const gap_params &p) {
  if (p.mode < GAP_MODE_PERSISTENT || p.mode > GAP_MODE_GRAPH) {
    set_error("params: mode %d out of range", p.mode);
    return GAP_EINVAL;
  }
  if (p.direction < GAP_DIR_AUTO || p.direction > GAP_DIR_BOTTOMUP) {
    set_error("params: direction %d out of range", p.direction);
    return GAP_EINVAL;
  }
  if (p.alpha < 1 || p.beta < 1) {
    set_error("params: alpha and beta must be >= 1");
    return GAP_EINVAL;
  }
  if (p.block != 256 && p.block != 512 && p.block != 1024) {
    set_error("params: block must be 256, 512 or 1024");
    return GAP_EINVAL;
  }
  if (p.blocks_per_cu < 0 || p.blocks_per_cu > 32) {
    set_error("params: blocks_per_cu must be in [0, 32]");
    return GAP_EINVAL;
  }
  if (p.hub_degree < 1 || p.hub_degree > (1 << 20)) {
    set_error("params: hub_degree must be in [1, 2^20]");
    return GAP_EINVAL;
  }
  if (p.chunk_edges < 64 || p.chunk_edges > (1 << 20) || p.chunk_edges % 64 != 0) {
    set_error("params: chunk_edges must be a multiple of 64 in [64, 2^20]");
    return GAP_EINVAL;
  }
  if (p.graph_chunk < 1 || p.graph_chunk > 4096) {
    set_error("params: graph_chunk must be in [1, 4096]");
    return GAP_EINVAL;
  }
  if (p.batch_mode != 0) {
    set_error("params: batch_mode must be 0 (persistent kernel)");
    return GAP_EINVAL;
  }
  if (p.grid_split < 1 || p.grid_split > 64) {
    set_error("params: grid_split must be in [1, 64]");
    return GAP_EINVAL;
  }
  if (p.lds_bitmap != 0 && p.lds_bitmap != 1) {
    set_error("params: lds_bitmap must be 0 or 1");
    return GAP_EINVAL;
  }
  if (p.batch_words != 1 && p.batch_words != 2 && p.batch_words != 4) {
    set_error("params: batch_words must be 1, 2 or 4");
    return GAP_EINVAL;
  }
  if (p.serve_window_us < 0) {
    set_error("params: serve_window_us must be >= 0");
    return GAP_EINVAL;
  }
  if (p.coop_launch != 0 && p.coop_launch != 1) {
    set_error("params: coop_launch must be 0 or 1");
    return GAP_EINVAL;
  }
  if (p.td_plain < 0) {
    set_error("params: td_plain must be >= 0");
    return GAP_EINVAL;
  }
  if (p.bu_mapping != 0 && p.bu_mapping != 1) {
    set_error("params: bu_mapping must be 0 or 1");
    return GAP_EINVAL;
  }
  if (p.small_frontier < 0) {
    set_error("params: small_frontier must be >= 0");
    return GAP_EINVAL;
  }
  if (p.wait_limit_us < 0) {
    set_error("params: wait_limit_us must be >= 0");
    return GAP_EINVAL;
  }
  if (p.batch_alpha < 1 || p.batch_beta < 1) {
    set_error("params: batch_alpha and batch_beta must be >= 1");
    return GAP_EINVAL;
  }
  return GAP_OK;
}

// ---- workspaces ---------------------------------------------------------------------

static std::map<std::pair<int, hipStream_t>, std::unique_ptr<Workspace>> g_ws;

Workspace *workspace_for(int dev, hipStream_t stream) {
  std::lock_guard<std::mutex> lk(g_mu);
  auto key = std::make_pair(dev, stream);
  auto it = g_ws.find(key);
  if (it != g_ws.end()) return it->second.get();
  std::unique_ptr<Workspace> ws(new (std::nothrow) Workspace());
  if (!ws) return nullptr;
  ws->device = dev;
  ws->stream = stream;
  if (hipMalloc(&ws->sticky, 256) != hipSuccess) {
    (void)hipGetLastError();
    return nullptr;
  }
  if (hipMemsetAsync(ws->sticky, 0, 256, stream) != hipSuccess) {
    (void)hipGetLastError();
    (void)hipFree(ws->sticky);
    return nullptr;
  }
  Workspace *raw = ws.get();
  g_ws.emplace(key, std::move(ws));
  return raw;
}

template <class T>
static void free_dev(T *&p) {
  if (p) (void)hipFree(p);
  p = nullptr;
}

static void release_single(Workspace *ws) {
  for (auto &q : ws->q) free_dev(q);
  for (auto &c : ws->cq) free_dev(c);
  for (auto &b : ws->bm) free_dev(b);
  free_dev(ws->depth_scratch);
  free_dev(ws->ctl);
  free_dev(ws->dd_args);
  if (ws->h_flags) (void)hipHostFree(ws->h_flags);
  ws->h_flags = nullptr;
  if (ws->h_args) (void)hipHostFree(ws->h_args);
  ws->h_args = nullptr;
  if (ws->graph_exec) (void)hipGraphExecDestroy((hipGraphExec_t)ws->graph_exec);
  ws->graph_exec = nullptr;
  ws->graph_key = 0;
  ws->cap_n = 0;
  ws->cap_chunks = 0;
}

static constexpr size_t kArgsBytes = 1024;  // >= sizeof of the per-search argument block

gap_status workspace_reserve_single(Workspace *ws, int64_t n, int64_t nnz, const gap_params &p) {
  // Each vertex enters a level's queue at most once, so a segment of n slots
  // can take any group's share; hub chunk items per level are bounded by
  // nnz/chunk + nnz/hub (one partial chunk per vertex of degree > hub, and
  // there are at most nnz/hub of those).  Every group has its own segment.
  const int64_t chunks = nnz / p.chunk_edges + nnz / p.hub_degree + 2;
  if (ws->cap_n >= n && ws->cap_chunks >= chunks && ws->ctl) return GAP_OK;
  if (ws->ctl) GAP_HIP(hipStreamSynchronize(ws->stream));
  const int64_t cap_n = std::max<int64_t>(n, ws->cap_n);
  const int64_t cap_c = std::max<int64_t>(chunks, ws->cap_chunks);
  release_single(ws);
  const int64_t words = (cap_n + 63) / 64 + 1;
  hipError_t e = hipSuccess;
  for (auto &q : ws->q)
    if (e == hipSuccess) e = hipMalloc(&q, sizeof(int32_t) * (size_t)cap_n * kGroups);
  for (auto &c : ws->cq)
    if (e == hipSuccess) e = hipMalloc(&c, sizeof(int2) * (size_t)cap_c * kGroups);
  for (auto &b : ws->bm)
    if (e == hipSuccess) e = hipMalloc(&b, sizeof(uint64_t) * (size_t)words);
  if (e == hipSuccess) e = hipMalloc(&ws->depth_scratch, sizeof(int32_t) * (size_t)cap_n);
  if (e == hipSuccess) e = hipMalloc(&ws->ctl, 2 * sizeof(Ctl));
  if (e == hipSuccess) e = hipMalloc(&ws->dd_args, kArgsBytes);
  if (e == hipSuccess) e = hipHostMalloc(&ws->h_flags, 4 * sizeof(int));
  if (e == hipSuccess) e = hipHostMalloc(&ws->h_args, kArgsBytes);
  // on the workspace's stream: a null-stream memset is not ordered before
  // work on a non-blocking stream
  if (e == hipSuccess) e = hipMemsetAsync(ws->ctl, 0, 2 * sizeof(Ctl), ws->stream);

  if (e != hipSuccess) {
    release_single(ws);
    return hip_fail(e, "workspace allocation");
  }
  ws->cap_n = cap_n;
  ws->cap_chunks = cap_c;
  ws->ctl_seq = 0;
  ws->ctl_next_clean = true;
  return GAP_OK;
}

gap_status workspace_reserve_recs(Workspace *ws, int32_t nrec) {
  if (ws->cap_recs >= nrec) return GAP_OK;
  GAP_HIP(hipStreamSynchronize(ws->stream));
  free_dev(ws->recs);
  ws->cap_recs = 0;
  GAP_HIP(hipMalloc(&ws->recs, sizeof(DevLevelRec) * (size_t)nrec));
  ws->cap_recs = nrec;
  return GAP_OK;
}

gap_status workspace_reserve_ms(Workspace *ws, size_t bytes, size_t host_bytes) {
  if (ws->ms_bytes < bytes) {
    GAP_HIP(hipStreamSynchronize(ws->stream));
    if (ws->ms_buf) (void)hipFree(ws->ms_buf);
    ws->ms_buf = nullptr;
    ws->ms_bytes = 0;
    GAP_HIP(hipMalloc(&ws->ms_buf, bytes));
    ws->ms_bytes = bytes;
  }
  if (ws->ms_host_bytes < host_bytes) {
    GAP_HIP(hipStreamSynchronize(ws->stream));
    if (ws->ms_host) (void)hipHostFree(ws->ms_host);
    ws->ms_host = nullptr;
    ws->ms_host_bytes = 0;
    GAP_HIP(hipHostMalloc(&ws->ms_host, host_bytes));
    ws->ms_host_bytes = host_bytes;
  }
  return GAP_OK;
}

gap_status workspace_reserve_bc(Workspace *ws, size_t vertex_bytes, size_t level_bytes) {
  if (ws->bc_bytes < vertex_bytes) {
    GAP_HIP(hipStreamSynchronize(ws->stream));
    if (ws->bc_buf) (void)hipFree(ws->bc_buf);
    ws->bc_buf = nullptr;
    ws->bc_bytes = 0;
    GAP_HIP(hipMalloc(&ws->bc_buf, vertex_bytes));
    ws->bc_bytes = vertex_bytes;
  }
  if (ws->bc_lv_bytes < level_bytes) {
    GAP_HIP(hipStreamSynchronize(ws->stream));
    if (ws->bc_lv) (void)hipFree(ws->bc_lv);
    ws->bc_lv = nullptr;
    ws->bc_lv_bytes = 0;
    GAP_HIP(hipMalloc(&ws->bc_lv, level_bytes));
    ws->bc_lv_bytes = level_bytes;
  }
  if (!ws->bc_host) GAP_HIP(hipHostMalloc(&ws->bc_host, 256));
  if (!ws->bc_event) GAP_HIP(hipEventCreateWithFlags(&ws->bc_event, hipEventDisableTiming));
  return GAP_OK;
}

gap_status workspace_reserve_sssp(Workspace *ws, size_t bytes) {
  if (ws->sp_bytes < bytes) {
    GAP_HIP(hipStreamSynchronize(ws->stream));
    if (ws->sp_buf) (void)hipFree(ws->sp_buf);
    ws->sp_buf = nullptr;
    ws->sp_bytes = 0;
    GAP_HIP(hipMalloc(&ws->sp_buf, bytes));
    ws->sp_bytes = bytes;
  }
  if (!ws->sp_host) GAP_HIP(hipHostMalloc(&ws->sp_host, 256));
  return GAP_OK;
}

gap_status workspace_reserve_cc(Workspace *ws, size_t bytes) {
  if (ws->cc_bytes < bytes) {
    GAP_HIP(hipStreamSynchronize(ws->stream));
    if (ws->cc_buf) (void)hipFree(ws->cc_buf);
    ws->cc_buf = nullptr;
    ws->cc_bytes = 0;
    GAP_HIP(hipMalloc(&ws->cc_buf, bytes));
    ws->cc_bytes = bytes;
  }
  return GAP_OK;
}

gap_status stream_status(hipStream_t stream) {
  std::vector<Workspace *> wss;
  {
    std::lock_guard<std::mutex> lk(g_mu);
    for (auto &kv : g_ws)
      if (kv.first.second == stream) wss.push_back(kv.second.get());
  }
  gap_status first = GAP_OK;
  for (Workspace *ws : wss) {
    GAP_HIP(hipSetDevice(ws->device));
    GAP_HIP(hipStreamSynchronize(stream));
    int code = 0;
    GAP_HIP(hipMemcpy(&code, ws->sticky, sizeof(int), hipMemcpyDeviceToHost));
    if (code != 0) {
      GAP_HIP(hipMemsetAsync(ws->sticky, 0, sizeof(int), stream));
      GAP_HIP(hipStreamSynchronize(stream));
      if (first == GAP_OK) first = code;
    }
  }
  const gap_status na = noalloc_status(stream);
  if (first == GAP_OK) first = na;
  if (first != GAP_OK)
    set_error("a search queued on this stream failed on the device (%s); its outputs are undefined",
              first == GAP_ETIMEOUT ? "a bounded wait gave up" : "inconsistent state");
  return first;
}

static void release_workspace(Workspace *ws) {
  (void)hipSetDevice(ws->device);
  release_single(ws);
  free_dev(ws->recs);
  ws->cap_recs = 0;
  if (ws->ms_buf) (void)hipFree(ws->ms_buf);
  if (ws->ms_host) (void)hipHostFree(ws->ms_host);
  if (ws->bc_buf) (void)hipFree(ws->bc_buf);
  if (ws->bc_lv) (void)hipFree(ws->bc_lv);
  if (ws->bc_host) (void)hipHostFree(ws->bc_host);
  if (ws->bc_event) (void)hipEventDestroy(ws->bc_event);
  if (ws->sp_buf) (void)hipFree(ws->sp_buf);
  if (ws->sp_host) (void)hipHostFree(ws->sp_host);
  if (ws->cc_buf) (void)hipFree(ws->cc_buf);
  free_dev(ws->sticky);
}

void release_all() {
  std::lock_guard<std::mutex> lk(g_mu);
  std::vector<int> devs;
  for (auto &kv : g_ws) devs.push_back(kv.first.first);
  for (auto &kv : g_coop) devs.push_back(kv.first);
  std::sort(devs.begin(), devs.end());
  devs.erase(std::unique(devs.begin(), devs.end()), devs.end());
  for (int d : devs) {
    (void)hipSetDevice(d);
    (void)hipDeviceSynchronize();
  }
  for (auto &kv : g_ws) release_workspace(kv.second.get());
  g_ws.clear();
  for (auto &kv : g_coop) {
    (void)hipSetDevice(kv.first);
    for (hipEvent_t e : kv.second->ev) (void)hipEventDestroy(e);
  }
  g_coop.clear();
  (void)hipGetLastError();
}

}  // namespace gap

using namespace gap;

// ---- C ABI --------------------------------------------------------------------------

extern "C" {

const char *gap_last_error(void) { return t_error.c_str(); }

gap_status gap_device_query(gap_device_info *info) {
  if (!info) {
    set_error("gap_device_query: NULL info");
    return GAP_EINVAL;
  }
  int count = 0;
  hipError_t e = hipGetDeviceCount(&count);
  if (e != hipSuccess || count < 1) {
    set_error("no HIP device available");
    return GAP_EDEVICE;
  }
  int dev = 0;
  GAP_HIP(hipGetDevice(&dev));
  const DeviceInfo *di = nullptr;
  gap_status st = device_info(dev, &di);
  if (st != GAP_OK) return st;
  memset(info, 0, sizeof(*info));
  info->device = dev;
  info->compute_units = di->cus;
  info->lds_per_cu = di->lds_per_cu;
  info->l2_bytes = di->l2_bytes;
  info->wave_size = kWave;
  info->clock_khz = di->clock_khz;
  info->total_mem = (int64_t)di->total_mem;
  snprintf(info->arch, sizeof(info->arch), "%s", di->arch);
  return GAP_OK;
}

gap_status gap_set_params(const gap_params *p) {
  if (!p) {
    set_error("gap_set_params: NULL");
    return GAP_EINVAL;
  }
  gap_status st = params_check(*p);
  if (st != GAP_OK) return st;
  std::lock_guard<std::mutex> lk(g_mu);
  g_params = *p;
  return GAP_OK;
}

gap_status gap_get_params(gap_params *p) {
  if (!p) {
    set_error("gap_get_params: NULL");
    return GAP_EINVAL;
  }
  *p = params_current();
  return GAP_OK;
}

static gap_status require_device() {
  int count = 0;
  hipError_t e = hipGetDeviceCount(&count);
  if (e != hipSuccess || count < 1) {
    set_error("no HIP device available");
    return GAP_EDEVICE;
  }
  return GAP_OK;
}

static gap_status build_checked(int64_t num_vertices, int64_t num_edges, const int32_t *src,
                                const int32_t *dst, const int32_t *weights, uint32_t flags,
                                void *stream, gap_graph **out) {
  clear_error();
  if (!out) {
    set_error("gap_build_csr: NULL out");
    return GAP_EINVAL;
  }
  *out = nullptr;
  if (num_vertices < 1 || num_vertices > 2147483647ll) {
    set_error("gap_build_csr: n = %lld outside [1, 2^31-1]", (long long)num_vertices);
    return GAP_EINVAL;
  }
  if (num_edges < 0 || (num_edges > 0 && (!src || !dst))) {
    set_error("gap_build_csr: bad edge arrays");
    return GAP_EINVAL;
  }
  if ((flags & ~GAP_BUILD_DIRECTED) != 0) {
    set_error("gap_build_csr: unknown flag bits 0x%x", flags & ~GAP_BUILD_DIRECTED);
    return GAP_EINVAL;
  }
  gap_status st = require_device();
  if (st != GAP_OK) return st;
  return build_csr(num_vertices, num_edges, src, dst, weights, (flags & GAP_BUILD_DIRECTED) != 0,
                   (hipStream_t)stream, out);
}

gap_status gap_build_csr(int64_t num_vertices, int64_t num_edges, const int32_t *src,
                         const int32_t *dst, uint32_t flags, void *stream, gap_graph **out) {
  return build_checked(num_vertices, num_edges, src, dst, nullptr, flags, stream, out);
}

gap_status gap_build_csr_weighted(int64_t num_vertices, int64_t num_edges, const int32_t *src,
                                  const int32_t *dst, const int32_t *weights, uint32_t flags,
                                  void *stream, gap_graph **out) {
  if (num_edges > 0 && !weights) {
    clear_error();
    set_error("gap_build_csr_weighted: NULL weights");
    return GAP_EINVAL;
  }
  return build_checked(num_vertices, num_edges, src, dst, weights, flags, stream, out);
}

gap_status gap_graph_info(const gap_graph *g, int64_t *n, int64_t *nnz) {
  if (!g) {
    set_error("gap_graph_info: NULL graph");
    return GAP_EINVAL;
  }
  if (n) *n = g->n;
  if (nnz) *nnz = g->nnz;
  return GAP_OK;
}

static gap_status export_csr(const gap_graph *g, const int64_t *d_row_ptr, const int32_t *d_col,
                             int64_t nnz, int64_t *row_ptr, int32_t *col, const char *what) {
  if (!g) {
    set_error("%s: NULL graph", what);
    return GAP_EINVAL;
  }
  GAP_HIP(hipSetDevice(g->device));
  if (row_ptr)
    GAP_HIP(hipMemcpy(row_ptr, d_row_ptr, sizeof(int64_t) * (size_t)(g->n + 1),
                      hipMemcpyDeviceToHost));
  if (col && nnz > 0)
    GAP_HIP(hipMemcpy(col, d_col, sizeof(int32_t) * (size_t)nnz, hipMemcpyDeviceToHost));
  return GAP_OK;
}

gap_status gap_graph_export(const gap_graph *g, int64_t *row_ptr, int32_t *col) {
  clear_error();
  return export_csr(g, g ? g->row_ptr : nullptr, g ? g->col : nullptr, g ? g->nnz : 0, row_ptr,
                    col, "gap_graph_export");
}

gap_status gap_graph_export_in(const gap_graph *g, int64_t *row_ptr, int32_t *col) {
  clear_error();
  return export_csr(g, g ? g->row_ptr_in : nullptr, g ? g->col_in : nullptr, g ? g->nnz_in : 0,
                    row_ptr, col, "gap_graph_export_in");
}

gap_status gap_graph_export_weights(const gap_graph *g, int32_t *weights) {
  clear_error();
  if (!g || !weights) {
    set_error("gap_graph_export_weights: NULL %s", g ? "weights" : "graph");
    return GAP_EINVAL;
  }
  if (!g->wt) {
    set_error("gap_graph_export_weights: the graph has no weights");
    return GAP_EINVAL;
  }
  GAP_HIP(hipSetDevice(g->device));
  if (g->nnz > 0)
    GAP_HIP(hipMemcpy(weights, g->wt, sizeof(int32_t) * (size_t)g->nnz, hipMemcpyDeviceToHost));
  return GAP_OK;
}

gap_status gap_graph_directed(const gap_graph *g) {
  clear_error();
  if (!g) {
    set_error("gap_graph_directed: NULL graph");
    return GAP_EINVAL;
  }
  return g->directed ? 1 : 0;
}

gap_status gap_bfs_ex(const gap_graph *g, int32_t source, int32_t *parent, int32_t *depth,
                      void *stream, const gap_params *params, gap_level_stat *stats,
                      int32_t max_levels, int32_t *num_levels) {
  clear_error();
  if (!g || !parent) {
    set_error("gap_bfs: NULL %s", g ? "parent" : "graph");
    return GAP_EINVAL;
  }
  if (source < 0 || (int64_t)source >= g->n) {
    set_error("gap_bfs: source %d outside [0, %lld)", source, (long long)g->n);
    return GAP_EINVAL;
  }
  gap_params p = params ? *params : params_current();
  if (params) {
    gap_status st = params_check(p);
    if (st != GAP_OK) return st;
  }
  return run_bfs(g, source, parent, depth, (hipStream_t)stream, p, stats, max_levels, num_levels);
}

gap_status gap_bfs(const gap_graph *g, int32_t source, int32_t *parent, int32_t *depth,
                   void *stream) {
  return gap_bfs_ex(g, source, parent, depth, stream, nullptr, nullptr, 0, nullptr);
}

gap_status gap_bfs_noalloc(const gap_graph *g, int32_t source, int32_t *parent, int32_t *depth,
                           void *stream) {
  clear_error();
  if (!g || !parent) {
    set_error("gap_bfs_noalloc: NULL %s", g ? "parent" : "graph");
    return GAP_EINVAL;
  }
  if (source < 0 || (int64_t)source >= g->n) {
    set_error("gap_bfs_noalloc: source %d outside [0, %lld)", source, (long long)g->n);
    return GAP_EINVAL;
  }
  return run_bfs_noalloc(g, source, parent, depth, (hipStream_t)stream);
}

gap_status gap_bfs_batch(const gap_graph *const *graphs, int32_t num_graphs,
                         const int32_t *graph_of_source, const int32_t *sources,
                         int32_t num_sources, int32_t *const *parents, int32_t *const *depths,
                         void *stream) {
  return gap_bfs_batch_ex(graphs, num_graphs, graph_of_source, sources, num_sources, parents,
                          depths, stream, nullptr, 0, nullptr);
}

gap_status gap_bfs_batch_ex(const gap_graph *const *graphs, int32_t num_graphs,
                            const int32_t *graph_of_source, const int32_t *sources,
                            int32_t num_sources, int32_t *const *parents, int32_t *const *depths,
                            void *stream, gap_level_stat *stats, int32_t max_levels,
                            int32_t *num_levels) {
  clear_error();
  if (!graphs || !graph_of_source || !sources || !parents) {
    set_error("gap_bfs_batch: NULL array");
    return GAP_EINVAL;
  }
  if (num_graphs <= 0 || num_sources <= 0) {
    set_error("gap_bfs_batch: counts must be positive");
    return GAP_EINVAL;
  }
  for (int32_t i = 0; i < num_graphs; ++i) {
    if (!graphs[i]) {
      set_error("gap_bfs_batch: graph %d is NULL", i);
      return GAP_EINVAL;
    }
    if (graphs[i]->device != graphs[0]->device) {
      set_error("gap_bfs_batch: graphs on different devices");
      return GAP_EINVAL;
    }
    if (graphs[i]->directed) {
      set_error("gap_bfs_batch: graph %d is directed (batched searches take undirected graphs)", i);
      return GAP_EINVAL;
    }
  }
  for (int32_t i = 0; i < num_sources; ++i) {
    const int32_t gi = graph_of_source[i];
    if (gi < 0 || gi >= num_graphs) {
      set_error("gap_bfs_batch: graph_of_source[%d] = %d out of range", i, gi);
      return GAP_EINVAL;
    }
    if (sources[i] < 0 || (int64_t)sources[i] >= graphs[gi]->n) {
      set_error("gap_bfs_batch: sources[%d] = %d out of range", i, sources[i]);
      return GAP_EINVAL;
    }
    if (!parents[i]) {
      set_error("gap_bfs_batch: parents[%d] is NULL", i);
      return GAP_EINVAL;
    }
  }
  return run_bfs_batch(graphs, num_graphs, graph_of_source, sources, num_sources, parents, depths,
                       (hipStream_t)stream, params_current(), stats, max_levels, num_levels);
}

void gap_free(gap_graph *g) {
  if (!g) return;
  (void)hipSetDevice(g->device);
  (void)hipDeviceSynchronize();
  if (g->row_ptr_in && g->row_ptr_in != g->row_ptr) (void)hipFree(g->row_ptr_in);
  if (g->col_in && g->col_in != g->col) (void)hipFree(g->col_in);
  if (g->row_ptr) (void)hipFree(g->row_ptr);
  if (g->col) (void)hipFree(g->col);
  if (g->wt) (void)hipFree(g->wt);
  if (g->head_in && g->head_in != g->head) (void)hipFree(g->head_in);
  if (g->head) (void)hipFree(g->head);
  delete g;
}

gap_status gap_bc(const gap_graph *g, const int32_t *sources, int32_t num_sources, double *scores,
                  uint32_t flags, void *stream) {
  clear_error();
  if (!g || !sources || !scores) {
    set_error("gap_bc: NULL %s", !g ? "graph" : (!sources ? "sources" : "scores"));
    return GAP_EINVAL;
  }
  if (num_sources < 1) {
    set_error("gap_bc: num_sources = %d, need at least one", num_sources);
    return GAP_EINVAL;
  }
  if ((flags & ~GAP_BC_RAW) != 0) {
    set_error("gap_bc: unknown flag bits 0x%x", flags & ~GAP_BC_RAW);
    return GAP_EINVAL;
  }
  for (int32_t i = 0; i < num_sources; ++i) {
    if (sources[i] < 0 || (int64_t)sources[i] >= g->n) {
      set_error("gap_bc: sources[%d] = %d outside [0, %lld)", i, sources[i], (long long)g->n);
      return GAP_EINVAL;
    }
  }
  GAP_HIP(hipSetDevice(g->device));
  return run_bc(g, sources, num_sources, scores, (flags & GAP_BC_RAW) == 0, (hipStream_t)stream);
}

gap_status gap_sssp_ex(const gap_graph *g, int32_t source, uint32_t *dist, uint32_t delta,
                       void *stream, int32_t *phases) {
  clear_error();
  if (!g || !dist) {
    set_error("gap_sssp: NULL %s", g ? "dist" : "graph");
    return GAP_EINVAL;
  }
  if (source < 0 || (int64_t)source >= g->n) {
    set_error("gap_sssp: source %d outside [0, %lld)", source, (long long)g->n);
    return GAP_EINVAL;
  }
  // every distance and the sentinel must fit in 32 bits
  if ((uint64_t)(g->n - 1) * (uint64_t)g->max_weight >= 0xFFFFFFFFull) {
    set_error("gap_sssp: (n - 1) * max weight = %llu does not fit below 2^32 - 1",
              (unsigned long long)((uint64_t)(g->n - 1) * (uint64_t)g->max_weight));
    return GAP_EINVAL;
  }
  if (delta == 0) {
    // default bucket width: 16 times the weight range over the mean list
    // length, rounded down to a power of two (at least 1); measured best
    // on R-MAT and uniform graphs of scale 22 with weights 1..255
    const double mean_deg = g->n > 0 ? (double)g->nnz / (double)g->n : 1.0;
    double d = (double)g->max_weight * 16.0 / std::max(1.0, mean_deg);
    uint32_t p2 = 1;
    while (p2 < 0x40000000u && (double)(p2 * 2) <= d) p2 *= 2;
    delta = p2;
  }
  GAP_HIP(hipSetDevice(g->device));
  return run_sssp(g, source, dist, delta, (hipStream_t)stream, phases);
}

gap_status gap_sssp(const gap_graph *g, int32_t source, uint32_t *dist, uint32_t delta,
                    void *stream) {
  return gap_sssp_ex(g, source, dist, delta, stream, nullptr);
}

gap_status gap_cc(const gap_graph *g, int32_t *labels, void *stream) {
  clear_error();
  if (!g || !labels) {
    set_error("gap_cc: NULL %s", g ? "labels" : "graph");
    return GAP_EINVAL;
  }
  GAP_HIP(hipSetDevice(g->device));
  return run_cc(g, labels, (hipStream_t)stream);
}

gap_status gap_stream_status(void *stream) {
  clear_error();
  return stream_status((hipStream_t)stream);
}

void gap_shutdown(void) { release_all(); }

gap_status gap_stream_copy(void *dst, const void *src, int64_t bytes, void *stream) {
  clear_error();
  if (!dst || !src || bytes < 0 || bytes % 16 != 0) {
    set_error("gap_stream_copy: bad arguments");
    return GAP_EINVAL;
  }
  return stream_copy(dst, src, bytes, (hipStream_t)stream);
}

}  // extern "C"
