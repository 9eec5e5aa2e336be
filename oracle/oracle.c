/*
 * CPU ORACLE FOR BREADTH-FIRST SEARCH, BETWEENNESS CENTRALITY,
 * SINGLE-SOURCE SHORTEST PATHS AND CONNECTED COMPONENTS -- TEST
 * INFRASTRUCTURE ONLY.
 *
 * Only the test suite, the smoke check and the benchmark's CPU-baseline leg
 * use this file.  It shares no code with the GPU library: it builds its own
 * adjacency from the raw edge list and runs a plain serial FIFO search.
 *
 * What it computes (paper, Section 2.1, "Breadth-First Search"):
 *   a parent array from a source with parent[source] = source,
 *   parent[v] = -1 for unreachable v, and for reachable v with parent u an
 *   edge u-v and depth[v] = depth[u] + 1.  Depth = hop distance from the
 *   source, -1 when unreachable.
 * How it is checked (paper, Section 3, BFS verifier): the parent of the
 * source is the source, every parent is joined to its child by an edge, and
 * depths from a trivial serial search show each parent one level above its
 * child.
 * Graph clean-up (paper, Section 2.3): removing duplicate edges and
 * self-loops and reordering neighbours are legal.  Undirected graphs insert
 * every raw pair in both directions; directed graphs (Section 2.2: some of
 * the paper's inputs are directed) keep each pair's direction.
 *
 * Betweenness centrality (Section 2.1): Brandes' dependency accumulation
 * from a set of sources, normalised by the largest score; see oracle_bc.
 * Shortest paths (Section 2.1): distances by Dijkstra's algorithm (the
 * paper's verifier for this kernel, Section 3) over a weighted adjacency
 * in which a repeated pair keeps its smallest weight; see oracle_sssp.
 * Connected components (Section 2.1): union-find over the raw pairs taken
 * as undirected (weak components of a directed graph), each vertex
 * labelled with the smallest vertex of its component (oracle_components),
 * and the paper's verifier for any labelling (oracle_cc_check).
 *
 * Pins (tests): exhaustive small graphs against Floyd-Warshall and boolean
 * matrix powers, random graphs against scipy's csgraph, closed forms (path,
 * cycle, star, complete, bipartite, hypercube, tree, grid), invariants and
 * union-find reachability on large runs.  Betweenness: every shortest path
 * enumerated on small graphs (the definition itself), closed forms (path,
 * star, cycle, complete graph), and the identity that a source's
 * dependencies sum to the total of (distance - 1) over the vertices it
 * reaches.  Shortest paths: Floyd-Warshall on small weighted graphs,
 * scipy's Dijkstra, unit weights against the BFS depths, closed forms, and
 * the two properties that define the answer (no edge can shorten a
 * distance; every reached vertex has an edge that attains it).
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ---- adjacency from the raw edge list --------------------------------- */

static int cmp_i32(const void *a, const void *b) {
  int32_t x = *(const int32_t *)a, y = *(const int32_t *)b;
  return (x > y) - (x < y);
}

/*
 * Symmetrised, self-loop-free, duplicate-free adjacency.
 *   offsets: caller-provided int64[n+1]
 *   adj:     caller-provided int32[2*m] (upper bound, compacted in place)
 * Returns the number of adjacency entries, or -1 on bad input.
 * Lists come out sorted ascending.
 */
int64_t oracle_build_adjacency(int64_t n, int64_t m, const int32_t *src,
                               const int32_t *dst, int64_t *offsets,
                               int32_t *adj) {
  if (n < 0 || m < 0 || !offsets || (m > 0 && (!src || !dst || !adj)))
    return -1;
  for (int64_t v = 0; v <= n; ++v) offsets[v] = 0;
  /* count both directions of every pair that is not a self-loop */
  for (int64_t e = 0; e < m; ++e) {
    int32_t u = src[e], v = dst[e];
    if (u < 0 || v < 0 || u >= n || v >= n) return -1;
    if (u == v) continue;
    offsets[u + 1] += 1;
    offsets[v + 1] += 1;
  }
  for (int64_t v = 0; v < n; ++v) offsets[v + 1] += offsets[v];
  int64_t *fill = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
  if (!fill) return -1;
  for (int64_t v = 0; v < n; ++v) fill[v] = offsets[v];
  for (int64_t e = 0; e < m; ++e) {
    int32_t u = src[e], v = dst[e];
    if (u == v) continue;
    adj[fill[u]++] = v;
    adj[fill[v]++] = u;
  }
  free(fill);
  /* sort each list, drop repeats, and pack the lists to the left */
  int64_t out = 0;
  int64_t start = 0;
  for (int64_t v = 0; v < n; ++v) {
    int64_t end = offsets[v + 1];
    int64_t len = end - start;
    if (len > 1) qsort(adj + start, (size_t)len, sizeof(int32_t), cmp_i32);
    int64_t row_begin = out;
    for (int64_t i = start; i < end; ++i) {
      if (i > start && adj[i] == adj[i - 1]) continue;
      adj[out++] = adj[i];
    }
    offsets[v] = row_begin;
    start = end;
  }
  offsets[n] = out;
  return out;
}

/*
 * Directed variant: out-lists only (u -> v for every raw pair (u, v),
 * u != v), sorted and duplicate-free.  A search over these lists follows
 * edges in their direction; the validator's edge test (is v in the list of
 * parent[v]?) then checks the directed edge parent[v] -> v.
 *   adj: caller-provided int32[m] (upper bound, compacted in place)
 */
int64_t oracle_build_out_adjacency(int64_t n, int64_t m, const int32_t *src,
                                   const int32_t *dst, int64_t *offsets,
                                   int32_t *adj) {
  if (n < 0 || m < 0 || !offsets || (m > 0 && (!src || !dst || !adj)))
    return -1;
  for (int64_t v = 0; v <= n; ++v) offsets[v] = 0;
  for (int64_t e = 0; e < m; ++e) {
    int32_t u = src[e], v = dst[e];
    if (u < 0 || v < 0 || u >= n || v >= n) return -1;
    if (u != v) offsets[u + 1] += 1;
  }
  for (int64_t v = 0; v < n; ++v) offsets[v + 1] += offsets[v];
  int64_t *fill = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
  if (!fill) return -1;
  for (int64_t v = 0; v < n; ++v) fill[v] = offsets[v];
  for (int64_t e = 0; e < m; ++e) {
    int32_t u = src[e], v = dst[e];
    if (u != v) adj[fill[u]++] = v;
  }
  free(fill);
  int64_t out = 0, start = 0;
  for (int64_t v = 0; v < n; ++v) {
    int64_t end = offsets[v + 1];
    if (end - start > 1) qsort(adj + start, (size_t)(end - start), sizeof(int32_t), cmp_i32);
    int64_t row_begin = out;
    for (int64_t i = start; i < end; ++i) {
      if (i > start && adj[i] == adj[i - 1]) continue;  /* repeated pair */
      adj[out++] = adj[i];
    }
    offsets[v] = row_begin;
    start = end;
  }
  offsets[n] = out;
  return out;
}

/* ---- serial FIFO breadth-first search --------------------------------- */

/*
 * depth/parent: caller-provided int32[n].  Returns the number of vertices
 * reached (including the source), or -1 on bad input.  The queue holds every
 * vertex at most once; neighbours are visited in list order, so the parent
 * of v is its first discoverer.
 */
int64_t oracle_bfs(int64_t n, const int64_t *offsets, const int32_t *adj,
                   int32_t source, int32_t *depth, int32_t *parent) {
  if (n <= 0 || source < 0 || source >= n || !offsets || !depth || !parent)
    return -1;
  int32_t *queue = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
  if (!queue) return -1;
  for (int64_t v = 0; v < n; ++v) {
    depth[v] = -1;
    parent[v] = -1;
  }
  depth[source] = 0;
  parent[source] = source;
  int64_t head = 0, tail = 0;
  queue[tail++] = source;
  while (head < tail) {
    int32_t u = queue[head++];
    for (int64_t i = offsets[u]; i < offsets[u + 1]; ++i) {
      int32_t v = adj[i];
      if (depth[v] == -1) {
        depth[v] = depth[u] + 1;
        parent[v] = u;
        queue[tail++] = v;
      }
    }
  }
  free(queue);
  return tail;
}

/* ---- validator --------------------------------------------------------- */

static int has_edge(const int64_t *offsets, const int32_t *adj, int32_t a,
                    int32_t b) {
  int64_t lo = offsets[a], hi = offsets[a + 1];
  while (lo < hi) {
    int64_t mid = lo + (hi - lo) / 2;
    if (adj[mid] < b)
      lo = mid + 1;
    else
      hi = mid;
  }
  return lo < offsets[a + 1] && adj[lo] == b;
}

/*
 * Checks a result against the definition, using reference depths from
 * oracle_bfs:
 *   1  depth_test differs from depth_ref (skipped when depth_test is NULL)
 *   2  parent[source] != source
 *   3  reachability of parent disagrees with the reference, or a negative
 *      value other than -1 appears
 *   4  parent of a reached vertex is out of range or not a neighbour
 *   5  parent of a reached vertex is not exactly one level above it
 * Returns 0 when every check passes; otherwise the first failing check, with
 * the offending vertex in *bad.
 */
int oracle_check(int64_t n, const int64_t *offsets, const int32_t *adj,
                 int32_t source, const int32_t *depth_ref,
                 const int32_t *parent, const int32_t *depth_test,
                 int64_t *bad) {
  int64_t dummy;
  if (!bad) bad = &dummy;
  *bad = -1;
  if (n <= 0 || source < 0 || source >= n || !parent || !depth_ref) return -1;
  if (depth_test) {
    for (int64_t v = 0; v < n; ++v)
      if (depth_test[v] != depth_ref[v]) {
        *bad = v;
        return 1;
      }
  }
  if (parent[source] != source) {
    *bad = source;
    return 2;
  }
  for (int64_t v = 0; v < n; ++v) {
    if (v == source) continue;
    int32_t p = parent[v];
    int reached = depth_ref[v] >= 0;
    if (!reached) {
      if (p != -1) {
        *bad = v;
        return 3;
      }
      continue;
    }
    if (p < 0) {
      *bad = v;
      return 3;
    }
    if (p >= n || !has_edge(offsets, adj, p, (int32_t)v)) {
      *bad = v;
      return 4;
    }
    if (depth_ref[p] != depth_ref[v] - 1) {
      *bad = v;
      return 5;
    }
  }
  return 0;
}

/* ---- union-find reachability (an independent algorithm) --------------- */

static int32_t uf_find(int32_t *up, int32_t x) {
  while (up[x] != x) {
    up[x] = up[up[x]];
    x = up[x];
  }
  return x;
}

/*
 * label[v] = a representative of v's connected component, computed from the
 * raw edge list with union-find (no adjacency, no queue).  Returns 0, or -1
 * on bad input.
 */
int oracle_components(int64_t n, int64_t m, const int32_t *src,
                      const int32_t *dst, int32_t *label) {
  if (n <= 0 || m < 0 || !label || (m > 0 && (!src || !dst))) return -1;
  for (int64_t v = 0; v < n; ++v) label[v] = (int32_t)v;
  for (int64_t e = 0; e < m; ++e) {
    int32_t a = src[e], b = dst[e];
    if (a < 0 || b < 0 || a >= n || b >= n) return -1;
    int32_t ra = uf_find(label, a), rb = uf_find(label, b);
    if (ra != rb) {
      if (ra < rb)
        label[rb] = ra;
      else
        label[ra] = rb;
    }
  }
  for (int64_t v = 0; v < n; ++v) label[v] = uf_find(label, (int32_t)v);
  return 0;
}

/* ---- betweenness centrality (Section 2.1, "Betweenness Centrality") ----- */

/*
 * Approximate betweenness from a set of sources:
 *   score[v] = sum over sources s != v, and targets t != s, t != v, of
 *              sigma_st(v) / sigma_st,
 * where sigma_st counts shortest s-t paths and sigma_st(v) those through v.
 * Unweighted; edges followed along the adjacency given (out-lists for a
 * directed graph).  Brandes' method, one source at a time: a FIFO search
 * counts paths (sigma of a vertex is the sum of sigma over its neighbours
 * one level up), then vertices are taken in reverse discovery order and each
 * one's dependency is accumulated from its successors (neighbours one level
 * down), found by their depths -- no successor lists are recorded.
 * A source listed twice contributes twice.  With normalise != 0 every score
 * is divided by the largest one (scores "normalised to one"); all-zero
 * scores stay zero.  fp64 throughout.  Returns 0, or -1 on bad input.
 */
int oracle_bc(int64_t n, const int64_t *offsets, const int32_t *adj,
              int32_t num_sources, const int32_t *sources, int normalise,
              double *score) {
  if (n <= 0 || !offsets || !score || num_sources < 0 ||
      (num_sources > 0 && !sources))
    return -1;
  for (int32_t k = 0; k < num_sources; ++k)
    if (sources[k] < 0 || sources[k] >= n) return -1;
  int32_t *order = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
  int32_t *depth = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
  double *sigma = (double *)malloc(sizeof(double) * (size_t)n);
  double *delta = (double *)malloc(sizeof(double) * (size_t)n);
  if (!order || !depth || !sigma || !delta) {
    free(order);
    free(depth);
    free(sigma);
    free(delta);
    return -1;
  }
  for (int64_t v = 0; v < n; ++v) score[v] = 0.0;
  for (int32_t k = 0; k < num_sources; ++k) {
    const int32_t s = sources[k];
    for (int64_t v = 0; v < n; ++v) {
      depth[v] = -1;
      sigma[v] = 0.0;
      delta[v] = 0.0;
    }
    depth[s] = 0;
    sigma[s] = 1.0;
    int64_t head = 0, tail = 0;
    order[tail++] = s;
    while (head < tail) {
      const int32_t u = order[head++];
      for (int64_t i = offsets[u]; i < offsets[u + 1]; ++i) {
        const int32_t v = adj[i];
        if (depth[v] == -1) {
          depth[v] = depth[u] + 1;
          order[tail++] = v;
        }
        if (depth[v] == depth[u] + 1) sigma[v] += sigma[u];
      }
    }
    for (int64_t i = tail - 1; i >= 0; --i) {
      const int32_t w = order[i];
      for (int64_t e = offsets[w]; e < offsets[w + 1]; ++e) {
        const int32_t v = adj[e];
        if (depth[v] == depth[w] + 1)
          delta[w] += sigma[w] / sigma[v] * (1.0 + delta[v]);
      }
      if (w != s) score[w] += delta[w];
    }
  }
  if (normalise) {
    double top = 0.0;
    for (int64_t v = 0; v < n; ++v)
      if (score[v] > top) top = score[v];
    if (top > 0.0)
      for (int64_t v = 0; v < n; ++v) score[v] /= top;
  }
  free(order);
  free(depth);
  free(sigma);
  free(delta);
  return 0;
}

/* ---- single-source shortest paths (Section 2.1, "SSSP") ----------------- */

typedef struct {
  int32_t v;
  int32_t w;
} wentry;

static int cmp_wentry(const void *a, const void *b) {
  const wentry *x = (const wentry *)a, *y = (const wentry *)b;
  if (x->v != y->v) return (x->v > y->v) - (x->v < y->v);
  return (x->w > y->w) - (x->w < y->w);
}

/*
 * Weighted adjacency: undirected (every pair in both directions) or, with
 * directed != 0, out-lists; self-loops dropped; a pair given several times
 * keeps its smallest weight.  offsets: int64[n+1]; adj, wadj: capacity
 * 2*m (undirected) or m.  Weights must be >= 1.  Returns nnz, or -1.
 */
int64_t oracle_build_weighted_adjacency(int64_t n, int64_t m, const int32_t *src,
                                        const int32_t *dst, const int32_t *w,
                                        int directed, int64_t *offsets,
                                        int32_t *adj, int32_t *wadj) {
  if (n <= 0 || m < 0 || !offsets || (m > 0 && (!src || !dst || !w || !adj || !wadj)))
    return -1;
  for (int64_t v = 0; v <= n; ++v) offsets[v] = 0;
  for (int64_t e = 0; e < m; ++e) {
    int32_t u = src[e], v = dst[e];
    if (u < 0 || v < 0 || u >= n || v >= n || w[e] < 1) return -1;
    if (u == v) continue;
    offsets[u + 1] += 1;
    if (!directed) offsets[v + 1] += 1;
  }
  for (int64_t v = 0; v < n; ++v) offsets[v + 1] += offsets[v];
  wentry *tmp = (wentry *)malloc(sizeof(wentry) * (size_t)(offsets[n] > 0 ? offsets[n] : 1));
  int64_t *fill = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
  if (!tmp || !fill) {
    free(tmp);
    free(fill);
    return -1;
  }
  for (int64_t v = 0; v < n; ++v) fill[v] = offsets[v];
  for (int64_t e = 0; e < m; ++e) {
    int32_t u = src[e], v = dst[e];
    if (u == v) continue;
    tmp[fill[u]].v = v;
    tmp[fill[u]++].w = w[e];
    if (!directed) {
      tmp[fill[v]].v = u;
      tmp[fill[v]++].w = w[e];
    }
  }
  int64_t out = 0;
  for (int64_t v = 0; v < n; ++v) {
    const int64_t start = offsets[v], end = offsets[v + 1];
    qsort(tmp + start, (size_t)(end - start), sizeof(wentry), cmp_wentry);
    offsets[v] = out;
    for (int64_t i = start; i < end; ++i) {
      if (i > start && tmp[i].v == tmp[i - 1].v) continue; /* heavier repeat */
      adj[out] = tmp[i].v;
      wadj[out] = tmp[i].w;
      ++out;
    }
  }
  offsets[n] = out;
  free(tmp);
  free(fill);
  return out;
}

/* binary min-heap of (distance, vertex) with lazy deletion */
typedef struct {
  int64_t d;
  int32_t v;
} hitem;

static void heap_push(hitem *h, int64_t *size, int64_t d, int32_t v) {
  int64_t i = (*size)++;
  while (i > 0) {
    int64_t p = (i - 1) / 2;
    if (h[p].d <= d) break;
    h[i] = h[p];
    i = p;
  }
  h[i].d = d;
  h[i].v = v;
}

static hitem heap_pop(hitem *h, int64_t *size) {
  hitem top = h[0], last = h[--(*size)];
  int64_t i = 0;
  for (;;) {
    int64_t c = 2 * i + 1;
    if (c >= *size) break;
    if (c + 1 < *size && h[c + 1].d < h[c].d) ++c;
    if (h[c].d >= last.d) break;
    h[i] = h[c];
    i = c;
  }
  if (*size > 0) h[i] = last;
  return top;
}

/*
 * Dijkstra's algorithm from source over (offsets, adj, wadj): dist[v] is the
 * least total weight of a path from the source, -1 when v is unreachable.
 * Returns the number of reached vertices, or -1 on bad input.
 */
int64_t oracle_sssp(int64_t n, const int64_t *offsets, const int32_t *adj,
                    const int32_t *wadj, int32_t source, int64_t *dist) {
  if (n <= 0 || source < 0 || source >= n || !offsets || !dist) return -1;
  const int64_t nnz = offsets[n];
  hitem *h = (hitem *)malloc(sizeof(hitem) * (size_t)(nnz + 1));
  char *done = (char *)calloc((size_t)n, 1);
  if (!h || !done) {
    free(h);
    free(done);
    return -1;
  }
  for (int64_t v = 0; v < n; ++v) dist[v] = -1;
  int64_t size = 0, reached = 0;
  dist[source] = 0;
  heap_push(h, &size, 0, source);
  while (size > 0) {
    hitem it = heap_pop(h, &size);
    if (done[it.v]) continue;
    done[it.v] = 1;
    ++reached;
    for (int64_t i = offsets[it.v]; i < offsets[it.v + 1]; ++i) {
      const int32_t v = adj[i];
      const int64_t nd = it.d + wadj[i];
      if (!done[v] && (dist[v] < 0 || nd < dist[v])) {
        dist[v] = nd;
        heap_push(h, &size, nd, v);
      }
    }
  }
  free(h);
  free(done);
  return reached;
}

/* ---- connected components check (Section 3, CC verifier) ---------------- */

/*
 * Checks a component labelling against the equivalence of Section 2.1
 * (same label if and only if an undirected path joins the vertices) the way
 * the paper's verifier does: one traversal per label over the undirected
 * adjacency (offsets, adj), which must meet no other label, and no label
 * may start a second traversal.  Returns 0 if the labelling is valid, 1 if
 * a traversal met another label (*bad = that vertex), 2 if two components
 * share a label (*bad = first vertex of the second one), -1 on bad input.
 */
int oracle_cc_check(int64_t n, const int64_t *offsets, const int32_t *adj,
                    const int32_t *label, int64_t *bad) {
  if (n <= 0 || !offsets || !label) return -1;
  if (bad) *bad = -1;
  char *seen = (char *)calloc((size_t)n, 1);
  int32_t *queue = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
  /* labels are arbitrary int32 values: remember used ones in a hash set */
  int64_t cap = 1;
  while (cap < 2 * n) cap <<= 1;
  int64_t *used = (int64_t *)malloc(sizeof(int64_t) * (size_t)cap);
  if (!seen || !queue || !used) {
    free(seen);
    free(queue);
    free(used);
    return -1;
  }
  for (int64_t i = 0; i < cap; ++i) used[i] = INT64_MIN;
  int rc = 0;
  for (int64_t s = 0; s < n && rc == 0; ++s) {
    if (seen[s]) continue;
    const int32_t L = label[s];
    uint64_t h = ((uint64_t)(uint32_t)L * 0x9E3779B97F4A7C15ULL) & (uint64_t)(cap - 1);
    while (used[h] != INT64_MIN && used[h] != (int64_t)L) h = (h + 1) & (uint64_t)(cap - 1);
    if (used[h] == (int64_t)L) {
      rc = 2;
      if (bad) *bad = s;
      break;
    }
    used[h] = (int64_t)L;
    int64_t head = 0, tail = 0;
    queue[tail++] = (int32_t)s;
    seen[s] = 1;
    while (head < tail && rc == 0) {
      const int32_t u = queue[head++];
      for (int64_t i = offsets[u]; i < offsets[u + 1]; ++i) {
        const int32_t v = adj[i];
        if (label[v] != L) {
          rc = 1;
          if (bad) *bad = v;
          break;
        }
        if (!seen[v]) {
          seen[v] = 1;
          queue[tail++] = v;
        }
      }
    }
  }
  free(seen);
  free(queue);
  free(used);
  return rc;
}
