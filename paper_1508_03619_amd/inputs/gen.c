/*
 * Seeded synthetic graph generators (raw edge lists) and the trial-source
 * picker.  This module feeds both the GPU library and the CPU oracle, so it
 * holds no breadth-first-search arithmetic: it only draws edges and vertices.
 *
 * Workloads stand in for the paper's input graphs (Section 2.2):
 *   - Kron: Kronecker/R-MAT generator with the Graph 500 quadrant
 *     probabilities A=0.57, B=C=0.19, D=0.05, edge factor 16.
 *   - Urand: Erdos-Renyi uniform random endpoints, |E| = 16 |V|.
 *   - Road: high-diameter stand-in, a 2D 4-neighbour lattice with random edge
 *     deletions and short diagonal shortcuts.
 * The paper asks for generators that produce the same graph regardless of the
 * thread count (Section 3, reference-code infrastructure).  Every draw here is
 * a pure function of (seed, stream, counter), so any OpenMP schedule gives the
 * same output.
 *
 * Random numbers: SplitMix64 (Steele, Lea and Flood, "Fast splittable
 * pseudorandom number generators", OOPSLA 2014).  Draw i of a keyed stream is
 * the SplitMix64 finaliser applied to key + (i+1)*golden_gamma, which is the
 * i-th output of a SplitMix64 generator seeded with `key`.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define GOLDEN_GAMMA 0x9E3779B97F4A7C15ULL

static inline uint64_t mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}

/* Key of an independent stream derived from a user seed and a stream tag. */
static inline uint64_t stream_key(uint64_t seed, uint64_t tag) {
  return mix64(seed ^ mix64(tag * GOLDEN_GAMMA + 0x632BE59BD9B4E019ULL));
}

static inline uint64_t draw(uint64_t key, uint64_t i) {
  return mix64(key + (i + 1) * GOLDEN_GAMMA);
}

/* Unbiased-enough bounded integer from 32 random bits (multiply-shift). */
static inline uint32_t bounded32(uint32_t r, uint32_t bound) {
  return (uint32_t)(((uint64_t)r * (uint64_t)bound) >> 32);
}

enum { TAG_RMAT = 1, TAG_PERM = 2, TAG_URAND = 3, TAG_GRID_DEL = 4,
       TAG_GRID_SC = 5, TAG_SOURCES = 6, TAG_WEIGHTS = 7 };

void gapgen_set_threads(int t) {
#ifdef _OPENMP
  if (t > 0) omp_set_num_threads(t);
#else
  (void)t;
#endif
}

int gapgen_max_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

/* Bijective scramble of [0, 2^scale): odd multiplies, adds and xor-shifts are
 * each invertible modulo 2^scale, so the composition relabels vertices
 * without collisions.  It removes the locality R-MAT gives low vertex IDs,
 * as Graph 500 does with its random relabelling. */
typedef struct { uint64_t mul[4], add[4]; uint64_t mask; int shift; } perm_t;

static void perm_init(perm_t *p, int scale, uint64_t seed) {
  uint64_t key = stream_key(seed, TAG_PERM);
  for (int r = 0; r < 4; ++r) {
    p->mul[r] = draw(key, 2 * (uint64_t)r) | 1ULL;
    p->add[r] = draw(key, 2 * (uint64_t)r + 1);
  }
  p->mask = (scale >= 64) ? ~0ULL : ((1ULL << scale) - 1ULL);
  p->shift = (scale + 1) / 2;
  if (p->shift < 1) p->shift = 1;
}

static inline uint64_t perm_apply(const perm_t *p, uint64_t x) {
  for (int r = 0; r < 4; ++r) {
    x = (x * p->mul[r] + p->add[r]) & p->mask;
    x ^= x >> p->shift;
  }
  return x;
}

/* R-MAT / Kronecker: edge_factor * 2^scale tuples.  Each tuple takes one
 * quadrant draw per bit level: (0,0) with prob a, (0,1) with b, (1,0) with c,
 * (1,1) with the rest.  Probabilities are compared as 32-bit fixed point so
 * the output does not depend on floating-point evaluation order.
 * Returns the number of tuples written, or -1 on bad arguments. */
int64_t gapgen_rmat(int scale, int64_t edge_factor, double a, double b,
                    double c, uint64_t seed, int permute, int32_t *src,
                    int32_t *dst) {
  if (scale < 1 || scale > 31 || edge_factor < 1 || !src || !dst) return -1;
  if (a < 0 || b < 0 || c < 0 || a + b + c > 1.0) return -1;
  const int64_t m = edge_factor << scale;
  const uint64_t ta = (uint64_t)(a * 4294967296.0);
  const uint64_t tab = (uint64_t)((a + b) * 4294967296.0);
  const uint64_t tabc = (uint64_t)((a + b + c) * 4294967296.0);
  const uint64_t key = stream_key(seed, TAG_RMAT);
  const int words = (scale + 1) / 2; /* two 32-bit draws per 64-bit output */
  perm_t pm;
  perm_init(&pm, scale, seed);
#pragma omp parallel for schedule(static)
  for (int64_t e = 0; e < m; ++e) {
    uint64_t u = 0, v = 0;
    for (int w = 0; w < words; ++w) {
      uint64_t r64 = draw(key, (uint64_t)e * (uint64_t)words + (uint64_t)w);
      for (int h = 0; h < 2; ++h) {
        int bit = 2 * w + h;
        if (bit >= scale) break;
        uint64_t r = h ? (r64 >> 32) : (r64 & 0xFFFFFFFFULL);
        if (r < ta) {
        } else if (r < tab) {
          v |= 1ULL << bit;
        } else if (r < tabc) {
          u |= 1ULL << bit;
        } else {
          u |= 1ULL << bit;
          v |= 1ULL << bit;
        }
      }
    }
    if (permute) {
      u = perm_apply(&pm, u);
      v = perm_apply(&pm, v);
    }
    src[e] = (int32_t)u;
    dst[e] = (int32_t)v;
  }
  return m;
}

/* Uniform random (Erdos-Renyi style) endpoints: m independent pairs drawn
 * uniformly from [0,n) x [0,n). */
int64_t gapgen_urand(int64_t n, int64_t m, uint64_t seed, int32_t *src,
                     int32_t *dst) {
  if (n < 1 || n > 2147483647LL || m < 0 || !src || !dst) return -1;
  const uint64_t key = stream_key(seed, TAG_URAND);
#pragma omp parallel for schedule(static)
  for (int64_t e = 0; e < m; ++e) {
    uint64_t r = draw(key, (uint64_t)e);
    src[e] = (int32_t)bounded32((uint32_t)(r >> 32), (uint32_t)n);
    dst[e] = (int32_t)bounded32((uint32_t)r, (uint32_t)n);
  }
  return m;
}

/* Number of 4-neighbour lattice edges of a w x h grid. */
int64_t gapgen_grid_lattice_edges(int w, int h) {
  if (w < 1 || h < 1) return 0;
  return (int64_t)(w - 1) * h + (int64_t)w * (h - 1);
}

/* Number of shortcut edges for a grid: round(frac * lattice edges). */
int64_t gapgen_grid_num_shortcuts(int w, int h, double frac) {
  double s = frac * (double)gapgen_grid_lattice_edges(w, h);
  return (int64_t)(s + 0.5);
}

/* Lattice edge e -> endpoints.  Horizontal edges first, row by row, then
 * vertical ones.  Vertex id = y*w + x. */
static inline void lattice_edge(int64_t e, int w, int h, int32_t *u,
                                int32_t *v) {
  const int64_t nh = (int64_t)(w - 1) * h;
  if (e < nh) {
    int64_t y = e / (w - 1), x = e % (w - 1);
    *u = (int32_t)(y * w + x);
    *v = (int32_t)(y * w + x + 1);
  } else {
    int64_t f = e - nh;
    int64_t y = f / w, x = f % w;
    *u = (int32_t)(y * w + x);
    *v = (int32_t)((y + 1) * w + x);
  }
  (void)h;
}

/* Road-like grid: w x h lattice, each lattice edge deleted independently with
 * probability p_delete, then round(shortcut_frac * lattice edges) diagonal
 * shortcuts (x,y)-(x+dx,y+dy) with dx,dy uniform in {-max..max}\{0}; draws
 * that leave the grid are redrawn (up to 64 times, else the shortcut is
 * dropped).  Kept lattice edges come first in lattice order, then shortcuts.
 * `cap` is the capacity of src/dst; returns the edge count, or -1 if the
 * arguments are bad or the output does not fit. */
int64_t gapgen_grid(int w, int h, double p_delete, double shortcut_frac,
                    int max_offset, uint64_t seed, int32_t *src, int32_t *dst,
                    int64_t cap) {
  if (w < 1 || h < 1 || (int64_t)w * h > 2147483647LL || !src || !dst)
    return -1;
  if (p_delete < 0 || p_delete > 1 || shortcut_frac < 0 || max_offset < 1)
    return -1;
  const int64_t ne = gapgen_grid_lattice_edges(w, h);
  const int64_t ns = gapgen_grid_num_shortcuts(w, h, shortcut_frac);
  const uint64_t kdel = stream_key(seed, TAG_GRID_DEL);
  const uint64_t ksc = stream_key(seed, TAG_GRID_SC);
  /* p_delete as a 64-bit threshold; p=1 deletes everything. */
  const long double pd = (long double)p_delete;
  const uint64_t tdel =
      (p_delete >= 1.0) ? ~0ULL : (uint64_t)(pd * 18446744073709551616.0L);
  const int64_t chunk = 1 << 16;
  const int64_t nchunks = (ne + chunk - 1) / chunk;
  int64_t *cnt = (int64_t *)calloc((size_t)nchunks + 1, sizeof(int64_t));
  if (!cnt) return -1;
#pragma omp parallel for schedule(static)
  for (int64_t k = 0; k < nchunks; ++k) {
    int64_t lo = k * chunk, hi = lo + chunk < ne ? lo + chunk : ne, c = 0;
    for (int64_t e = lo; e < hi; ++e)
      if (p_delete < 1.0 && draw(kdel, (uint64_t)e) >= tdel) ++c;
    cnt[k + 1] = c;
  }
  for (int64_t k = 0; k < nchunks; ++k) cnt[k + 1] += cnt[k];
  const int64_t kept = cnt[nchunks];
  if (kept + ns > cap) {
    free(cnt);
    return -1;
  }
#pragma omp parallel for schedule(static)
  for (int64_t k = 0; k < nchunks; ++k) {
    int64_t lo = k * chunk, hi = lo + chunk < ne ? lo + chunk : ne;
    int64_t o = cnt[k];
    for (int64_t e = lo; e < hi; ++e) {
      if (p_delete < 1.0 && draw(kdel, (uint64_t)e) >= tdel) {
        lattice_edge(e, w, h, &src[o], &dst[o]);
        ++o;
      }
    }
  }
  free(cnt);
  const uint32_t span = 2u * (uint32_t)max_offset; /* nonzero offsets */
  int64_t dropped = 0;
#pragma omp parallel for schedule(static) reduction(+ : dropped)
  for (int64_t s = 0; s < ns; ++s) {
    int ok = 0;
    int32_t a = 0, bb = 0;
    for (int t = 0; t < 64 && !ok; ++t) {
      uint64_t r0 = draw(ksc, (uint64_t)s * 128 + 2 * (uint64_t)t);
      uint64_t r1 = draw(ksc, (uint64_t)s * 128 + 2 * (uint64_t)t + 1);
      int x = (int)bounded32((uint32_t)r0, (uint32_t)w);
      int y = (int)bounded32((uint32_t)(r0 >> 32), (uint32_t)h);
      int dx = (int)bounded32((uint32_t)r1, span) - max_offset;
      int dy = (int)bounded32((uint32_t)(r1 >> 32), span) - max_offset;
      if (dx >= 0) dx += 1; /* skip 0: {-max..-1} U {1..max} */
      if (dy >= 0) dy += 1;
      int x2 = x + dx, y2 = y + dy;
      if (x2 >= 0 && x2 < w && y2 >= 0 && y2 < h) {
        a = (int32_t)((int64_t)y * w + x);
        bb = (int32_t)((int64_t)y2 * w + x2);
        ok = 1;
      }
    }
    if (ok) {
      src[kept + s] = a;
      dst[kept + s] = bb;
    } else {
      src[kept + s] = -1; /* marked, compacted below */
      dst[kept + s] = -1;
      dropped += 1;
    }
  }
  int64_t total = kept + ns;
  if (dropped) {
    int64_t o = kept;
    for (int64_t s = kept; s < total; ++s)
      if (src[s] >= 0) {
        src[o] = src[s];
        dst[o] = dst[s];
        ++o;
      }
    total = o;
  }
  return total;
}

/* Trial sources: uniform draws from [0,n), keeping vertices that touch at
 * least one non-self-loop edge (non-zero degree once the graph is
 * symmetrised and cleaned) and that were not picked before.  Writes up to k
 * sources, returns how many were found (fewer only if the graph has fewer
 * non-zero-degree vertices, or after 64*n + 1024 draws). */
static int32_t pick_sources(int64_t n, int64_t m, const int32_t *src,
                            const int32_t *dst, uint64_t seed, int32_t k,
                            int32_t *out, int out_only) {
  if (n < 1 || m < 0 || k < 0 || !out || (m > 0 && (!src || !dst))) return -1;
  uint8_t *touch = (uint8_t *)calloc((size_t)n, 1);
  if (!touch) return -1;
  for (int64_t e = 0; e < m; ++e) {
    int32_t a = src[e], b = dst[e];
    if (a == b || a < 0 || b < 0 || a >= n || b >= n) continue;
    touch[a] = 1;
    if (!out_only) touch[b] = 1;
  }
  const uint64_t key = stream_key(seed, TAG_SOURCES);
  int32_t got = 0;
  const uint64_t limit = 64ULL * (uint64_t)n + 1024ULL;
  for (uint64_t i = 0; i < limit && got < k; ++i) {
    uint64_t r = draw(key, i);
    int64_t v = (int64_t)(((r >> 32) * (uint64_t)n) >> 32);
    if (touch[v] == 1) {
      out[got++] = (int32_t)v;
      touch[v] = 2; /* picked */
    }
  }
  free(touch);
  return got;
}

int32_t gapgen_pick_sources(int64_t n, int64_t m, const int32_t *src,
                            const int32_t *dst, uint64_t seed, int32_t k,
                            int32_t *out) {
  return pick_sources(n, m, src, dst, seed, k, out, 0);
}

/* As gapgen_pick_sources for a directed graph (pair e is the edge
 * src[e] -> dst[e]): only vertices with an out-edge qualify. */
int32_t gapgen_pick_out_sources(int64_t n, int64_t m, const int32_t *src,
                                const int32_t *dst, uint64_t seed, int32_t k,
                                int32_t *out) {
  return pick_sources(n, m, src, dst, seed, k, out, 1);
}


/* Edge weights for the shortest-path kernel (Section 2.2: the unweighted
 * graphs get uniform integer weights 1..255).  The weight of pair e is a
 * function of its endpoints only -- of the unordered pair when undirected,
 * of (src, dst) when directed -- so repeated pairs and the two directions
 * of an undirected edge agree.  Returns 0, or -1 on bad input. */
int gapgen_weights(int64_t m, const int32_t *src, const int32_t *dst,
                   uint64_t seed, int directed, int32_t *w) {
  if (m < 0 || (m > 0 && (!src || !dst || !w))) return -1;
  const uint64_t key = stream_key(seed, TAG_WEIGHTS);
#pragma omp parallel for schedule(static)
  for (int64_t e = 0; e < m; ++e) {
    uint32_t a = (uint32_t)src[e], b = (uint32_t)dst[e];
    if (!directed && a > b) {
      uint32_t t = a;
      a = b;
      b = t;
    }
    const uint64_t r = draw(key, ((uint64_t)a << 32) | b);
    w[e] = 1 + (int32_t)bounded32((uint32_t)(r >> 32), 255u);
  }
  return 0;
}
