// Multi-source BFS (batch of searches).  Placeholder schedule: one
// single-source search per lane on the device.
#include "runtime.h"

namespace gap {

gap_status run_bfs_batch(const gap_graph *const *graphs, int32_t num_graphs,
                         const int32_t *graph_of_source, const int32_t *sources,
                         int32_t num_sources, int32_t *const *parents, int32_t *const *depths,
                         hipStream_t stream, const gap_params &p) {
  (void)num_graphs;
  for (int32_t i = 0; i < num_sources; ++i) {
    const gap_graph *g = graphs[graph_of_source[i]];
    gap_status st = run_bfs(g, sources[i], parents[i], depths ? depths[i] : nullptr, stream, p,
                            nullptr, 0, nullptr);
    if (st != GAP_OK) return st;
  }
  return GAP_OK;
}

}  // namespace gap
