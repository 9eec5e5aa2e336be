/*
 * Host-only driver for the sanitizer test: runs the input generators and
 * every oracle routine over small graphs (generated, degenerate and invalid
 * inputs) so that AddressSanitizer and UndefinedBehaviorSanitizer see each
 * code path.  Built together with the generators and the oracle by
 * tests/test_sanitize.py; exits non-zero on any unexpected result (the
 * sanitizers abort on their own findings).
 */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

int64_t gapgen_rmat(int scale, int64_t edge_factor, double a, double b, double c, uint64_t seed,
                    int permute, int32_t *src, int32_t *dst);
int64_t gapgen_urand(int64_t n, int64_t m, uint64_t seed, int32_t *src, int32_t *dst);
int64_t gapgen_grid_lattice_edges(int w, int h);
int64_t gapgen_grid_num_shortcuts(int w, int h, double frac);
int64_t gapgen_grid(int w, int h, double p_delete, double shortcut_frac, int max_offset,
                    uint64_t seed, int32_t *src, int32_t *dst, int64_t cap);
int32_t gapgen_pick_sources(int64_t n, int64_t m, const int32_t *src, const int32_t *dst,
                            uint64_t seed, int32_t k, int32_t *out);
int32_t gapgen_pick_out_sources(int64_t n, int64_t m, const int32_t *src, const int32_t *dst,
                                uint64_t seed, int32_t k, int32_t *out);
int gapgen_weights(int64_t m, const int32_t *src, const int32_t *dst, uint64_t seed, int directed,
                   int32_t *w);

int64_t oracle_build_adjacency(int64_t n, int64_t m, const int32_t *src, const int32_t *dst,
                               int64_t *offsets, int32_t *adj);
int64_t oracle_build_out_adjacency(int64_t n, int64_t m, const int32_t *src, const int32_t *dst,
                                   int64_t *offsets, int32_t *adj);
int64_t oracle_bfs(int64_t n, const int64_t *offsets, const int32_t *adj, int32_t source,
                   int32_t *depth, int32_t *parent);
int oracle_check(int64_t n, const int64_t *offsets, const int32_t *adj, int32_t source,
                 const int32_t *depth_ref, const int32_t *parent, const int32_t *depth_test,
                 int64_t *bad);
int oracle_components(int64_t n, int64_t m, const int32_t *src, const int32_t *dst,
                      int32_t *label);
int oracle_bc(int64_t n, const int64_t *offsets, const int32_t *adj, int32_t num_sources,
              const int32_t *sources, int normalise, double *score);
int64_t oracle_build_weighted_adjacency(int64_t n, int64_t m, const int32_t *src,
                                        const int32_t *dst, const int32_t *w, int directed,
                                        int64_t *offsets, int32_t *adj, int32_t *wadj);
int64_t oracle_sssp(int64_t n, const int64_t *offsets, const int32_t *adj, const int32_t *wadj,
                    int32_t source, int64_t *dist);
int oracle_cc_check(int64_t n, const int64_t *offsets, const int32_t *adj, const int32_t *label,
                    int64_t *bad);

static int failures = 0;
#define EXPECT(cond)                                                   \
  do {                                                                 \
    if (!(cond)) {                                                     \
      fprintf(stderr, "%s:%d: expectation failed: %s\n", __FILE__, __LINE__, #cond); \
      ++failures;                                                      \
    }                                                                  \
  } while (0)

static void *xmalloc(size_t bytes) {
  void *p = malloc(bytes ? bytes : 1);
  if (!p) {
    fprintf(stderr, "out of memory\n");
    exit(2);
  }
  return p;
}

/* Every oracle routine over one raw edge list (undirected, then directed). */
static void exercise(const char *what, int64_t n, int64_t m, const int32_t *src,
                     const int32_t *dst) {
  for (int directed = 0; directed < 2; ++directed) {
    int64_t *off = xmalloc(sizeof(int64_t) * (size_t)(n + 1));
    int32_t *adj = xmalloc(sizeof(int32_t) * (size_t)(2 * m));
    const int64_t nnz = directed ? oracle_build_out_adjacency(n, m, src, dst, off, adj)
                                 : oracle_build_adjacency(n, m, src, dst, off, adj);
    EXPECT(nnz >= 0 && nnz <= 2 * m);
    int32_t *depth = xmalloc(sizeof(int32_t) * (size_t)n);
    int32_t *parent = xmalloc(sizeof(int32_t) * (size_t)n);
    int32_t *label = xmalloc(sizeof(int32_t) * (size_t)n);
    int32_t srcs[8];
    const int32_t k = directed ? gapgen_pick_out_sources(n, m, src, dst, 99, 8, srcs)
                               : gapgen_pick_sources(n, m, src, dst, 99, 8, srcs);
    EXPECT(k >= 0 && k <= 8);
    for (int32_t i = 0; i < k || (i == 0 && n > 0); ++i) {
      const int32_t s = k > 0 ? srcs[i] : (int32_t)(n - 1);
      const int64_t reached = oracle_bfs(n, off, adj, s, depth, parent);
      EXPECT(reached >= 1 && reached <= n);
      int64_t bad = -2;
      EXPECT(oracle_check(n, off, adj, s, depth, parent, depth, &bad) == 0);
      EXPECT(oracle_check(n, off, adj, s, depth, parent, NULL, &bad) == 0);
      /* a planted wrong parent is caught, and reported inside [0, n) */
      if (reached > 1) {
        int32_t *p2 = xmalloc(sizeof(int32_t) * (size_t)n);
        memcpy(p2, parent, sizeof(int32_t) * (size_t)n);
        for (int64_t v = 0; v < n; ++v)
          if (v != s && depth[v] > 0) {
            p2[v] = -3;
            break;
          }
        EXPECT(oracle_check(n, off, adj, s, depth, p2, depth, &bad) != 0 && bad >= 0 && bad < n);
        free(p2);
      }
      if (k == 0) break;
    }
    if (k > 0) {
      double *score = xmalloc(sizeof(double) * (size_t)n);
      EXPECT(oracle_bc(n, off, adj, k < 4 ? k : 4, srcs, 1, score) == 0);
      EXPECT(oracle_bc(n, off, adj, k < 4 ? k : 4, srcs, 0, score) == 0);
      free(score);
    }
    if (!directed) {
      EXPECT(oracle_components(n, m, src, dst, label) == 0);
      int64_t bad = -2;
      EXPECT(oracle_cc_check(n, off, adj, label, &bad) == 0);
    }
    /* weighted: weights 1..255, Dijkstra from every picked source */
    int32_t *w = xmalloc(sizeof(int32_t) * (size_t)(m ? m : 1));
    EXPECT(gapgen_weights(m, src, dst, 7, directed, w) == 0);
    int64_t *woff = xmalloc(sizeof(int64_t) * (size_t)(n + 1));
    int32_t *wadj = xmalloc(sizeof(int32_t) * (size_t)(2 * m));
    int32_t *wts = xmalloc(sizeof(int32_t) * (size_t)(2 * m));
    const int64_t wnnz = oracle_build_weighted_adjacency(n, m, src, dst, w, directed, woff, wadj, wts);
    EXPECT(wnnz >= 0);
    int64_t *dist = xmalloc(sizeof(int64_t) * (size_t)n);
    for (int32_t i = 0; i < k; ++i) EXPECT(oracle_sssp(n, woff, wadj, wts, srcs[i], dist) >= 1);
    free(dist);
    free(wts);
    free(wadj);
    free(woff);
    free(w);
    free(label);
    free(parent);
    free(depth);
    free(adj);
    free(off);
  }
  if (failures) fprintf(stderr, "  (in %s)\n", what);
}

int main(void) {
  /* R-MAT, relabelled and not */
  for (int permute = 0; permute < 2; ++permute) {
    const int scale = 9;
    const int64_t m = (int64_t)16 << scale;
    int32_t *s = xmalloc(sizeof(int32_t) * (size_t)m), *d = xmalloc(sizeof(int32_t) * (size_t)m);
    EXPECT(gapgen_rmat(scale, 16, 0.57, 0.19, 0.19, 5 + permute, permute, s, d) == m);
    exercise("rmat", (int64_t)1 << scale, m, s, d);
    free(s);
    free(d);
  }
  /* uniform */
  {
    const int64_t n = 777, m = 16 * 777;
    int32_t *s = xmalloc(sizeof(int32_t) * (size_t)m), *d = xmalloc(sizeof(int32_t) * (size_t)m);
    EXPECT(gapgen_urand(n, m, 11, s, d) == m);
    exercise("urand", n, m, s, d);
    free(s);
    free(d);
  }
  /* grids: a 1 x k line, a small grid, everything deleted */
  const int gw[3] = {1, 23, 9}, gh[3] = {40, 17, 9};
  const double pdel[3] = {0.1, 0.1, 1.0};
  for (int t = 0; t < 3; ++t) {
    const int64_t cap = gapgen_grid_lattice_edges(gw[t], gh[t]) +
                        gapgen_grid_num_shortcuts(gw[t], gh[t], 0.01);
    int32_t *s = xmalloc(sizeof(int32_t) * (size_t)(cap + 1));
    int32_t *d = xmalloc(sizeof(int32_t) * (size_t)(cap + 1));
    const int64_t got = gapgen_grid(gw[t], gh[t], pdel[t], 0.01, 3, 13 + t, s, d, cap);
    EXPECT(got >= 0 && got <= cap);
    if (got >= 0) exercise("grid", (int64_t)gw[t] * gh[t], got, s, d);
    /* too small an output buffer is refused, not overrun */
    if (cap > 1) EXPECT(gapgen_grid(gw[t], gh[t], 0.0, 0.01, 3, 1, s, d, 1) == -1);
    free(s);
    free(d);
  }
  /* degenerate: one vertex, no edges, only self-loops and duplicates */
  {
    int32_t s[6] = {0, 0, 2, 2, 2, 4}, d[6] = {0, 0, 2, 3, 3, 4};
    exercise("one vertex, self-loop", 1, 2, s, d);
    exercise("no edges", 6, 0, s, d);
    exercise("self-loops and duplicates", 6, 6, s, d);
  }
  /* invalid arguments come back as -1 */
  {
    int64_t off[4];
    int32_t adj[4], dep[3], par[3], lab[3];
    double sc[3];
    EXPECT(gapgen_rmat(0, 16, 0.57, 0.19, 0.19, 1, 1, adj, adj) == -1);
    EXPECT(gapgen_rmat(4, 16, 0.6, 0.3, 0.3, 1, 1, adj, adj) == -1);
    EXPECT(gapgen_urand(0, 1, 1, adj, adj) == -1);
    EXPECT(gapgen_grid(0, 3, 0.1, 0.01, 3, 1, adj, adj, 4) == -1);
    EXPECT(gapgen_pick_sources(-1, 0, NULL, NULL, 1, 4, adj) < 0);
    EXPECT(gapgen_weights(3, NULL, NULL, 1, 0, NULL) == -1);
    EXPECT(oracle_build_adjacency(-1, 0, NULL, NULL, off, adj) == -1);
    EXPECT(oracle_build_adjacency(3, 2, NULL, NULL, off, adj) == -1);
    EXPECT(oracle_build_out_adjacency(3, 0, NULL, NULL, NULL, adj) == -1);
    EXPECT(oracle_build_adjacency(3, 0, NULL, NULL, off, adj) == 0);
    EXPECT(oracle_bfs(3, off, adj, 3, dep, par) == -1);
    EXPECT(oracle_bfs(3, off, adj, -1, dep, par) == -1);
    EXPECT(oracle_bfs(3, off, adj, 0, NULL, par) == -1);
    EXPECT(oracle_components(0, 0, NULL, NULL, lab) == -1);
    EXPECT(oracle_bc(3, off, adj, 1, NULL, 1, sc) == -1);
    EXPECT(oracle_sssp(3, off, adj, adj, 5, (int64_t *)off) == -1);
    EXPECT(oracle_cc_check(0, off, adj, lab, NULL) == -1);
  }
  if (failures) {
    fprintf(stderr, "%d expectation(s) failed\n", failures);
    return 1;
  }
  printf("sanitize driver: all checks passed\n");
  return 0;
}
