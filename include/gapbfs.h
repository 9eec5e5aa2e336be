/*
 * gapbfs.h -- C ABI of libgapbfs.so: direction-optimizing breadth-first
 * search on one AMD Instinct MI355X (gfx950), and the kernels of the same
 * suite built on the traversal: betweenness centrality (gap_bc), shortest
 * paths (gap_sssp) and connected components (gap_cc).
 *
 * The operation is the BFS kernel of the GAP Benchmark Suite (Beamer,
 * Asanovic, Patterson, arXiv 1508.03619):
 *   - Section 2.1, "Breadth-First Search": from a source vertex, produce a
 *     parent array with parent[source] = source, parent[v] = -1 when v is
 *     unreachable, and, for every reachable v with parent u, an edge u-v and
 *     depth[v] = depth[u] + 1.  Several parent arrays are correct; depth (hop
 *     distance, -1 when unreachable) is unique.
 *   - Section 2.3: 32-bit vertex identifiers, more than 2^32 edges supported
 *     (64-bit offsets); duplicate edges and self-loops may be removed and
 *     neighbours reordered; graph building is untimed, every per-trial
 *     structure other than the graph is rebuilt per trial.
 *   - Section 3, BFS: the direction-optimizing search (top-down steps over a
 *     vertex list, bottom-up steps once the frontier is large), with each
 *     unvisited vertex's degree stored as a negative number in the parent
 *     array so the frontier's edge count accrues during top-down steps, and a
 *     final pass that turns every remaining negative value into -1.
 *
 * Conventions for every call:
 *   - Calls return a gap_status and never abort or throw; gap_last_error()
 *     gives a message for the calling thread's last failure.
 *   - "device" pointers are HIP device memory on the graph's device (for
 *     instance the data pointers of torch.cuda tensors); "host" pointers are
 *     ordinary process memory.
 *   - `stream` is a hipStream_t passed as void*; NULL means the legacy
 *     default stream.  Work is queued on it; outputs are complete once the
 *     caller synchronises that stream.  The library keeps scratch per
 *     (device, stream): calls on different streams may come from different
 *     host threads at once; calls that share a stream should come from one
 *     thread at a time.
 *   - Vertex IDs are int32 in [0, n); n <= 2^31 - 1.  Offsets and edge
 *     counts are int64.
 */
#ifndef GAPBFS_H
#define GAPBFS_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t gap_status;
#define GAP_OK 0
#define GAP_EINVAL (-1)    /* bad argument (NULL pointer, ID out of range) */
#define GAP_ENOMEM (-2)    /* device or host allocation failed */
#define GAP_EDEVICE (-3)   /* no HIP device, or a HIP runtime error */
#define GAP_EBUSY (-4)     /* the call cannot proceed now (a full request ring,
                              a server holding requests on another graph) */
#define GAP_EINTERNAL (-5) /* the device reported an inconsistent state */
#define GAP_ETIMEOUT (-6)  /* a bounded device-side wait gave up */

/* Opaque, immutable graph resident in device memory (CSR). */
typedef struct gap_graph gap_graph;

/* gap_build_csr flag: keep edge directions (Section 2.1 allows directed
 * graphs; a search then follows edges from tail to head only). */
#define GAP_BUILD_DIRECTED 1u

/*
 * gap_build_csr -- build the graph used by every search (Section 2.3: the
 * graph is loaded and built once, untimed).
 *   num_vertices  n, 1 <= n <= 2^31 - 1
 *   num_edges     number of raw pairs, >= 0
 *   src, dst      host int32[num_edges], each value in [0, n); copied, the
 *                 caller keeps ownership and may free them on return
 *   flags         0: undirected; GAP_BUILD_DIRECTED: the pair (src[i],
 *                 dst[i]) is the edge src[i] -> dst[i]; no other bit is
 *                 defined
 *   stream        stream used for the upload and build kernels
 *   out           receives the handle; release it with gap_free
 * Undirected: every pair is inserted in both directions.  Directed: the
 * handle holds the out-lists and also the in-lists (the transpose, read by
 * bottom-up steps), so it takes about twice the memory of one CSR.  In both
 * cases self-loops and duplicates are removed and each list is sorted
 * ascending; a CSR is an int64 row_ptr[n+1] and an int32 col[nnz] in device
 * memory owned by the handle.  The call returns after the build has
 * finished.
 * Errors: GAP_EINVAL (NULL out, n out of range, an ID out of range, an
 * unknown flag, more than 2^32 stored entries per call), GAP_ENOMEM,
 * GAP_EDEVICE.
 */
gap_status gap_build_csr(int64_t num_vertices, int64_t num_edges,
                         const int32_t *src, const int32_t *dst,
                         uint32_t flags, void *stream, gap_graph **out);

/*
 * gap_build_csr_weighted -- as gap_build_csr, with a weight per raw pair
 * for the shortest-path kernel (Section 2.1; Section 2.2 gives unweighted
 * graphs uniform integer weights 1..255).
 *   weights  host int32[num_edges], each >= 1; copied.  A pair given more
 *            than once keeps its smallest weight; for an undirected graph
 *            both directions of a pair carry its weight.
 * Other arguments and errors as gap_build_csr, plus GAP_EINVAL for NULL
 * weights or a weight below 1.  The weights are stored beside the out-lists
 * (4 bytes per entry).  Searches other than gap_sssp ignore them.
 */
gap_status gap_build_csr_weighted(int64_t num_vertices, int64_t num_edges,
                                  const int32_t *src, const int32_t *dst,
                                  const int32_t *weights, uint32_t flags,
                                  void *stream, gap_graph **out);

/* Copies the out-list weights (host int32[nnz], in gap_graph_export order).
 * GAP_EINVAL when the graph was built without weights.  Synchronous. */
gap_status gap_graph_export_weights(const gap_graph *g, int32_t *weights);

/* Vertex count n and stored adjacency entries nnz: 2|E| for an undirected
 * graph, |E| (out-list entries) for a directed one. */
gap_status gap_graph_info(const gap_graph *g, int64_t *n, int64_t *nnz);

/* 1 if g was built with GAP_BUILD_DIRECTED, 0 if not, GAP_EINVAL for NULL. */
gap_status gap_graph_directed(const gap_graph *g);

/*
 * gap_graph_export -- copy the CSR (the out-lists of a directed graph) to
 * host memory (for cross-checks and edge counting; not on the search
 * path).  row_ptr: host int64[n+1]; col: host int32[nnz] (either may be
 * NULL to skip it).  Synchronous.
 */
gap_status gap_graph_export(const gap_graph *g, int64_t *row_ptr,
                            int32_t *col);

/* As gap_graph_export, for the in-lists (the same arrays as the out-lists
 * when the graph is undirected). */
gap_status gap_graph_export_in(const gap_graph *g, int64_t *row_ptr,
                               int32_t *col);

/*
 * gap_bfs -- one direction-optimizing search (Section 2.1 output,
 * Section 3 method).
 *   g        graph from gap_build_csr
 *   source   vertex in [0, n); a degree-0 source is legal and reaches only
 *            itself
 *   parent   device int32[n], written: parent[source] = source, -1 for
 *            unreachable vertices, otherwise a vertex one level closer
 *            with an edge to this one (an in-neighbour when directed)
 *   depth    device int32[n] or NULL; written: hop distance, -1 when
 *            unreachable
 *   stream   queue for the work
 * Per-search scratch (queues, bitmaps, counters) comes from a pool the
 * library keeps per (device, stream); concurrent calls on different
 * streams are allowed, including on one graph.  With the default
 * (persistent-kernel) schedule the call only queues work; with the
 * host-driven schedule it waits on the stream between levels.
 * Errors: GAP_EINVAL (NULL g or parent, source out of range),
 * GAP_ENOMEM, GAP_EDEVICE, GAP_ETIMEOUT (a device-side wait that timed
 * out: reported by gap_bfs_ex with stats and by the host-driven schedule,
 * which wait for the search).  The default schedule returns before the
 * search runs: a search that fails on the device there leaves its outputs
 * undefined, does not affect later searches, and records its error in the
 * stream's sticky status word, which gap_stream_status returns.
 */
gap_status gap_bfs(const gap_graph *g, int32_t source, int32_t *parent,
                   int32_t *depth, void *stream);

/* Size in bytes of the per-device scratch array of gap_bfs_noalloc. */
#define GAP_NOALLOC_SCRATCH_BYTES (64ll << 20)

/*
 * gap_bfs_noalloc -- gap_bfs for callers that cannot allocate device
 * memory: work queued under stream capture, tight serving loops, harnesses
 * that forbid allocation.  Same arguments, outputs and errors as gap_bfs;
 * always the persistent schedule (one cooperative launch, after a small
 * kernel that clears the control block), whatever gap_set_params selected
 * for mode and grid_split; the other parameters apply.
 * Scratch: every per-search buffer (queues, bitmaps, control block, the
 * depth array when depth is NULL) lives in one file-scope device array of
 * GAP_NOALLOC_SCRATCH_BYTES, of which each GPU that runs the call holds its
 * own copy until the process ends.  The call allocates no device or pinned
 * memory and creates no event; its first call on a device records the
 * array's device address (and clears its status word on `stream`).  A
 * graph needs about 132 bytes per vertex (136 with a NULL depth) plus 2
 * bytes per adjacency entry (default hub_degree and chunk_edges), e.g. up
 * to 2^18 vertices with 2^23 entries; a larger one gets GAP_EINVAL and
 * nothing is queued.
 * Every call on a GPU shares that GPU's array, and it keeps the previous
 * call's contents (the call clears what must start at zero): calls that
 * overlap on one GPU -- on different streams, or from several host threads
 * -- race and give undefined results.  Serialise them (one stream, or
 * events).
 * A search that fails on the device (GAP_ETIMEOUT: a bounded wait gave up)
 * leaves its outputs undefined and records the error in a status word of
 * the array, which gap_stream_status returns (and clears) after waiting
 * for its stream.
 */
gap_status gap_bfs_noalloc(const gap_graph *g, int32_t source, int32_t *parent,
                           int32_t *depth, void *stream);

/*
 * gap_bfs_batch -- many searches in one multi-source launch.  Lane i
 * searches graph graphs[graph_of_source[i]] from sources[i]; each lane's
 * result is exactly what gap_bfs returns for that (graph, source) (same
 * depths; parents valid by the same definition).  Lanes of one graph share
 * 64-bit per-vertex visit/frontier words, so one traversal of the graph
 * serves up to 64 lanes per word.
 *   graphs            host array of num_graphs handles (all on one device)
 *   graph_of_source   host int32[num_sources], values in [0, num_graphs)
 *   sources           host int32[num_sources], each in [0, n of its graph);
 *                     repeats are allowed
 *   parents, depths   host arrays of num_sources device pointers; lane i
 *                     writes int32[n of its graph] at parents[i] and, when
 *                     depths is not NULL and depths[i] is not NULL, at
 *                     depths[i]
 *   stream            queue for the work
 * Undirected graphs only.
 * Errors: GAP_EINVAL (NULL arrays, counts <= 0, index or source out of
 * range, graphs on different devices, a directed graph), GAP_ENOMEM,
 * GAP_EDEVICE.  The call only queues the work.  A batch that fails on the
 * device (GAP_ETIMEOUT: a bounded wait gave up; GAP_EINTERNAL) writes
 * INT32_MIN to every entry of every lane's outputs and records the error
 * in the stream's sticky status word (gap_stream_status).
 */
gap_status gap_bfs_batch(const gap_graph *const *graphs, int32_t num_graphs,
                         const int32_t *graph_of_source,
                         const int32_t *sources, int32_t num_sources,
                         int32_t *const *parents, int32_t *const *depths,
                         void *stream);

/* ---- continuous batching (serving) -----------------------------------------
 * A server keeps one multi-source search running on the device for the
 * single-source queries of one graph at a time (Section 2.1 output per
 * query): up to 64 queries are the bits of a per-vertex 64-bit word; a query
 * submitted while the search runs joins it at the next level boundary
 * (its depths counted from that level) in a free lane, and a query whose
 * frontier is empty completes on its own, freeing its lane.  Every query's
 * result is exactly what gap_bfs returns for its (graph, source): the same
 * depths, valid parents.
 * Threading: one host thread at a time per server.  The server's launches
 * are queued on its stream, which they keep busy while they run; read a
 * completed query's outputs on another stream.
 */
typedef struct gap_server gap_server;

/*
 * gap_serve_open -- a server for graphs of at most max_vertices vertices
 * and max_entries adjacency entries, launching on `stream` (of the current
 * device).  Allocates its device state (about 152 bytes per vertex plus
 * 2 bytes per entry at the default hub_degree/chunk_edges) and a pinned
 * request/completion ring shared with the device.
 * Errors: GAP_EINVAL (NULL out, sizes out of range), GAP_ENOMEM,
 * GAP_EDEVICE.
 */
gap_status gap_serve_open(int64_t max_vertices, int64_t max_entries,
                          void *stream, gap_server **out);

/*
 * gap_serve_submit -- queues one query: BFS of g (undirected, built on the
 * server's device, within the server's sizes) from `source`, writing
 * int32[n] parent and (when not NULL) depth on the device, as gap_bfs does.
 * The outputs are final once gap_serve_poll returns `qid`.  The query joins
 * a running launch at its next level boundary, or the call launches one.
 * Errors: GAP_EINVAL (NULL server, graph or parent, source out of range, a
 * directed or too large graph), GAP_EBUSY (256 queries in flight: poll
 * first; or the server still holds queries on another graph),
 * GAP_ENOMEM, GAP_EDEVICE.
 */
gap_status gap_serve_submit(gap_server *s, const gap_graph *g, int64_t qid,
                            int32_t source, int32_t *parent, int32_t *depth);

/*
 * gap_serve_poll -- stores the ids of up to `max` completed queries (in
 * completion order) at qids and their number at *count; does not wait.
 * Returns GAP_ETIMEOUT or GAP_EINTERNAL once if a launch failed on the
 * device (the queries it held are lost).  Launches again when requests are
 * waiting and no launch is left to take them.
 */
gap_status gap_serve_poll(gap_server *s, int64_t *qids, int32_t max,
                          int32_t *count);

/* Waits for the server's launches (queries in flight finish) and releases
 * it (NULL-safe). */
gap_status gap_serve_close(gap_server *s);

/* gap_bc flag: return the raw sums (no division by the largest score). */
#define GAP_BC_RAW 1u

/*
 * gap_bc -- approximate betweenness centrality from a set of sources
 * (Section 2.1, "Betweenness Centrality": the benchmark uses 4 sources and
 * scores normalised to one).
 *   g            graph from gap_build_csr (undirected or directed)
 *   sources      host int32[num_sources], each in [0, n); a repeated source
 *                contributes twice
 *   num_sources  >= 1
 *   scores       device double[n], written: score[v] = sum over the sources
 *                s != v and all targets t != s, v of sigma_st(v) / sigma_st
 *                (sigma_st: number of shortest s-t paths, sigma_st(v): those
 *                through v; unweighted, along edge directions), then divided
 *                by the largest score unless flags has GAP_BC_RAW (all-zero
 *                scores stay zero)
 *   flags        0 or GAP_BC_RAW
 *   stream       queue for the work
 * fp64 throughout.  Sums are formed in an order that depends on scheduling,
 * so results may differ from run to run in the last bits.  Per-call scratch
 * (about 30 bytes per vertex, 34 when directed, plus 0.08 bytes per
 * adjacency entry) comes from the per-stream pool.  The call waits on the stream once per source
 * (to size the per-depth arrays) and returns with the last source's work
 * queued.
 * Errors: GAP_EINVAL (NULL argument, no sources, a source out of range, an
 * unknown flag), GAP_ENOMEM, GAP_EDEVICE, GAP_EINTERNAL.
 */
gap_status gap_bc(const gap_graph *g, const int32_t *sources,
                  int32_t num_sources, double *scores, uint32_t flags,
                  void *stream);

/*
 * gap_sssp -- single-source shortest paths (Section 2.1: distances, the
 * sentinel for unreachable vertices; Section 3: Delta-stepping).
 *   g       graph from gap_build_csr_weighted (a graph built without weights
 *           is searched with every weight 1, so the distances are the BFS
 *           depths); edges are followed along their direction
 *   source  vertex in [0, n)
 *   dist    device uint32[n], written: dist[source] = 0, 0xFFFFFFFF for
 *           unreachable vertices, otherwise the least total weight of a path
 *   delta   bucket width of Delta-stepping; 0 picks 16 * max weight / mean
 *           list length, rounded down to a power of two.  Any delta >= 1
 *           gives the same distances (the answer is unique); delta is the
 *           one parameter the paper lets depend on the graph (Section 2.3)
 *   stream  queue for the work; the call only queues it
 * Scratch (about 32 bytes per vertex plus 1 byte per adjacency entry) comes
 * from the per-stream pool.
 * Errors: GAP_EINVAL (NULL argument, source out of range, (n - 1) times
 * the largest weight not below 2^32 - 1), GAP_ENOMEM, GAP_EDEVICE,
 * GAP_ETIMEOUT (reported by gap_sssp_ex).
 */
gap_status gap_sssp(const gap_graph *g, int32_t source, uint32_t *dist,
                    uint32_t delta, void *stream);

/* gap_sssp with a statistics output: when phases is not NULL the call
 * waits for the search and stores the number of relaxation phases run
 * there, and reports a timed-out device-side wait as GAP_ETIMEOUT. */
gap_status gap_sssp_ex(const gap_graph *g, int32_t source, uint32_t *dist,
                       uint32_t delta, void *stream, int32_t *phases);

/*
 * gap_cc -- connected components (Section 2.1: two vertices share a label
 * if and only if an undirected path joins them; for a directed graph the
 * weak components; a vertex without edges is alone).
 *   g       graph from gap_build_csr or gap_build_csr_weighted
 *   labels  device int32[n], written: the smallest vertex of each vertex's
 *           component (so the labelling is unique)
 *   stream  queue for the work; the call only queues it
 * Scratch (about 0.3 bytes per adjacency entry) comes from the per-stream
 * pool.  Errors: GAP_EINVAL (NULL argument), GAP_ENOMEM, GAP_EDEVICE.
 */
gap_status gap_cc(const gap_graph *g, int32_t *labels, void *stream);

/* Releases the graph (NULL-safe).  Waits for the device to finish any work
 * queued on it before freeing. */
void gap_free(gap_graph *g);

/*
 * gap_stream_status -- waits for every call queued on `stream` and returns
 * GAP_OK, or the first error a kernel of gap_bfs, gap_bfs_batch or gap_sssp
 * recorded on the device since the previous gap_stream_status call on that
 * stream: GAP_ETIMEOUT (a bounded device-side wait gave up) or
 * GAP_EINTERNAL (an inconsistent search state).  Such a failure is kept in
 * a sticky status word of the stream's scratch, which no later search
 * clears; this call clears it.  The default schedules queue a search and
 * return before it runs, so this is where their device-side failures are
 * reported.  GAP_EDEVICE for a HIP runtime error.
 */
gap_status gap_stream_status(void *stream);

/*
 * gap_shutdown -- waits for every device the library has used, then
 * releases every per-stream scratch pool, event and captured graph it holds
 * (graph handles stay valid; a later call allocates scratch again).  For
 * process exit: the Python binding calls it at interpreter exit.
 */
void gap_shutdown(void);

/* Message for the calling thread's most recent failure ("" if none). */
const char *gap_last_error(void);

/* ---- schedule and tuning ------------------------------------------------
 * Tuning parameters are properties of the hardware, identical for every
 * graph (Section 2.3: one implementation and one parameter set for all
 * input graphs).  They never change results: depths are unique and every
 * schedule returns valid parents.
 */
#define GAP_MODE_PERSISTENT 0 /* one cooperative kernel, grid barriers */
#define GAP_MODE_LEVELS 1     /* one launch per step, host reads counters */
#define GAP_MODE_GRAPH 2      /* hipGraph chunks of levels, device-decided */

#define GAP_DIR_AUTO 0    /* edge/vertex-count switching heuristic */
#define GAP_DIR_TOPDOWN 1 /* top-down steps only */
#define GAP_DIR_BOTTOMUP 2 /* bottom-up from the first level on */

typedef struct gap_params {
  int32_t mode;          /* GAP_MODE_* */
  int32_t direction;     /* GAP_DIR_* */
  int32_t alpha;         /* top-down -> bottom-up when m_f > m_u / alpha */
  int32_t beta;          /* bottom-up -> top-down when n_f < n / beta and
                            the frontier shrank (default 128: a switch
                            back costs a pass over the frontier bitmap,
                            and a late bottom-up step is cheap) */
  int32_t block;         /* threads per workgroup: 256, 512 or 1024 */
  int32_t blocks_per_cu; /* persistent grid: workgroups per compute unit
                            (0 = as many as fit) */
  int32_t hub_degree;    /* top-down: vertices of larger degree are split
                            into chunk work items */
  int32_t chunk_edges;   /* edges per chunk work item (multiple of 64) */
  int32_t graph_chunk;   /* GAP_MODE_GRAPH: levels per captured graph */
  int32_t batch_mode;    /* multi-source schedule: 0 = persistent kernel */
  int32_t batch_alpha;   /* multi-source: top-down -> bottom-up threshold */
  int32_t batch_beta;    /* multi-source: bottom-up -> top-down threshold */
  int32_t grid_split;    /* k >= 1: a persistent launch takes 1/k of the CUs
                            and at most k of them run at once (so searches
                            queued on different streams can overlap) */
  int32_t small_frontier; /* persistent single-source schedule: a top-down
                            level whose frontier and frontier edges are both
                            at most this runs on 32 workgroups while the
                            rest wait (0 = every level on the whole grid) */
  int32_t lds_bitmap;    /* persistent single-source schedule: 1 = bottom-up
                            steps copy the frontier bitmap (n/8 bytes) into
                            each workgroup's LDS, the whole of it when it
                            fits, else its low words up to the LDS left
                            beside the kernel's own (probes of higher
                            vertex ids read the global copy); 0 = never */
  int32_t wait_limit_us; /* bound of one device-side wait without progress
                            (a grid barrier, or a parked workgroup waiting
                            for the small group), in microseconds; 0 = the
                            built-in bounds (3 s per barrier wait, 10 s
                            without a finished small level).  A wait that
                            gives up ends the search with GAP_ETIMEOUT; every
                            kernel still exits. */
  int32_t bu_mapping;    /* persistent single-source schedule, bottom-up
                            steps: 0 = each workgroup owns a contiguous range
                            of vertices and its lanes are refilled with new
                            vertices as held ones finish (when the range fits
                            the workgroup's LDS bitmap: up to 4096 64-vertex
                            words per workgroup), 1 = each wave keeps a fixed
                            set of 4 words until all their vertices finish */
  int32_t batch_words;   /* multi-source tile shape: 64-bit words per vertex
                            of one graph segment (1, 2 or 4); a graph with
                            more lanes than 64 * batch_words gets several
                            segments, each a pass of its own over the graph */
  int32_t serve_window_us; /* gap_serve_*: a serving launch takes new
                            requests into free lanes at level boundaries for
                            this long after it starts, then finishes the
                            searches it holds and exits (0 = it takes
                            requests at its first boundary only) */
  int32_t td_plain;      /* persistent single-source schedule: a top-down
                            level whose frontier edges exceed n / td_plain
                            claims vertices with plain stores of parent and
                            depth instead of compare-and-swap (any frontier
                            neighbour is a valid parent), and F_{d+1} and its
                            totals are then read back from the depths by one
                            pass over the vertices; 0 = every level claims by
                            compare-and-swap.  Default 8. */
  int32_t coop_launch;   /* grid-barrier kernels (persistent searches,
                            batches, serving, shortest paths): 0 = ordinary
                            launches sized to be resident, ordered by the
                            library's per-device launch ring so that at most
                            grid_split of them run at once (the default;
                            ~15 us less between consecutive searches), 1 =
                            cooperative launches (the runtime checks
                            residency; use when other software on the same
                            GPU launches its own grid-barrier kernels).  A
                            broken residency assumption ends in GAP_ETIMEOUT
                            from the bounded waits, not in a hang. */
} gap_params;

/* Process-wide parameters (copied).  Invalid values -> GAP_EINVAL. */
gap_status gap_set_params(const gap_params *p);
gap_status gap_get_params(gap_params *p);

/* Per-level record of one search, for measurement and tests. */
typedef struct gap_level_stat {
  int32_t level;        /* depth d of the frontier expanded at this step */
  int32_t direction;    /* 1 top-down, 2 bottom-up */
  int64_t frontier;     /* |F_d| */
  int64_t frontier_edges; /* sum of degrees over F_d */
  int64_t claimed;      /* |F_{d+1}| */
  int64_t scanned;      /* adjacency entries read by the step */
  int64_t unvisited;    /* bottom-up: vertices still searching a parent */
  int64_t time_ns;      /* device time from the level's start to the end of
                           its barrier (real-time clock, 10 ns resolution) */
} gap_level_stat;

/*
 * gap_bfs_ex -- gap_bfs with an explicit parameter set (NULL = process-wide)
 * and, when `stats` is not NULL, per-level records (synchronous: waits for
 * the search, then copies at most max_levels records and writes the level
 * count to *num_levels).  Counting adds device atomics; timed runs pass NULL.
 */
gap_status gap_bfs_ex(const gap_graph *g, int32_t source, int32_t *parent,
                      int32_t *depth, void *stream, const gap_params *params,
                      gap_level_stat *stats, int32_t max_levels,
                      int32_t *num_levels);

/* gap_bfs_batch with per-level records when `stats` is not NULL (waits for
 * the batch; copies at most max_levels records and writes the level count
 * to *num_levels).  A record aggregates the lanes of every graph: frontier =
 * vertices with some lane's frontier bit, frontier_edges = their degrees,
 * claimed = the next level's frontier, direction = that of the first
 * graph's lanes; a bottom-up level counts in `unvisited` the vertices some
 * lane still needed and in `scanned` the adjacency entries read (a top-down
 * level reads frontier_edges entries).  At most 128 levels are recorded.
 * Counting adds device atomics; timed runs pass NULL.  Errors as
 * gap_bfs_batch, plus GAP_ETIMEOUT / GAP_EINTERNAL from the device. */
gap_status gap_bfs_batch_ex(const gap_graph *const *graphs, int32_t num_graphs,
                            const int32_t *graph_of_source,
                            const int32_t *sources, int32_t num_sources,
                            int32_t *const *parents, int32_t *const *depths,
                            void *stream, gap_level_stat *stats,
                            int32_t max_levels, int32_t *num_levels);

/* Device facts used by the tuner and the benchmark. */
typedef struct gap_device_info {
  int32_t device;
  int32_t compute_units;
  int32_t lds_per_cu;      /* bytes */
  int32_t l2_bytes;
  int32_t wave_size;
  int32_t clock_khz;
  int64_t total_mem;
  char arch[64];
} gap_device_info;

gap_status gap_device_query(gap_device_info *info);

/*
 * gap_stream_copy -- HBM bandwidth probe: copies `bytes` (multiple of 16)
 * from src to dst (device pointers, non-overlapping) with the library's
 * streaming-copy kernel on `stream`.
 */
gap_status gap_stream_copy(void *dst, const void *src, int64_t bytes,
                           void *stream);

#ifdef __cplusplus
}
#endif

#endif /* GAPBFS_H */
