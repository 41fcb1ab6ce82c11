/*
 * Seeded synthetic inputs for the flow-refinement path: random geometric
 * graphs in the unit square / cube, recursive coordinate bisection, and the
 * two boundary-noise recipes.  These build INPUTS only; nothing here takes
 * part in the refinement arithmetic, so the CPU oracle and the GPU library
 * may both be fed from it.
 *
 * Random numbers: splitmix64 (Steele, Lea, Flood, "Fast splittable
 * pseudorandom number generators", OOPSLA 2014): state += 0x9E3779B97F4A7C15,
 * then the output mix z ^= z>>30, z *= 0xBF58476D1CE4E5B9, z ^= z>>27,
 * z *= 0x94D049BB133111EB, z ^= z>>31.
 *
 * The random geometric graph follows the family shape of the paper's rggX
 * instances (uniform points in the unit square, an edge iff the Euclidean
 * distance is below a radius; Section 6, "Instances"), with the radius set by
 * a target mean degree instead of the paper's connectivity threshold.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define GOLDEN 0x9E3779B97F4A7C15ULL

static uint64_t mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}

uint64_t gen_splitmix64_next(uint64_t *state) {
  *state += GOLDEN;
  return mix64(*state);
}

/* Weight hash of an undirected edge {u,v}, u < v: one splitmix64 step keyed
 * by the pair, then one more keyed by the seed. */
uint64_t gen_edge_hash(uint64_t seed, int32_t u, int32_t v) {
  uint64_t key = ((uint64_t)(uint32_t)u << 32) | (uint64_t)(uint32_t)v;
  return mix64(seed ^ mix64(key + GOLDEN) + GOLDEN);
}

typedef struct {
  int32_t n;
  int32_t dim;
  int64_t narcs;
  double radius;
  int32_t *xadj;   /* [n+1] */
  int32_t *adjncy; /* [narcs] */
  int32_t *adjwgt; /* [narcs] */
  double *coords;  /* [n*dim], row per vertex */
} gen_graph;

void gen_free(gen_graph *g) {
  free(g->xadj);
  free(g->adjncy);
  free(g->adjwgt);
  free(g->coords);
  memset(g, 0, sizeof(*g));
}

/* Random geometric graph.  Points are drawn in generation order i = 0..n-1,
 * coordinate by coordinate, each as the top 53 bits of one splitmix64 output
 * scaled to [0,1).  The unit square/cube is cut into nc^dim cells of side
 * 1/nc >= r; vertex ids follow the cells in row-major order (x fastest) and,
 * inside a cell, the generation order.  An edge joins u != v iff their squared
 * distance is < r^2.  Adjacency lists come out sorted by id.
 * Edge weight = wlo + hash(seed, min, max) mod (whi - wlo + 1).
 * Returns 0, or -1 on bad arguments / allocation failure / arc overflow. */
int gen_rgg(int32_t n, int32_t dim, double mean_degree, uint64_t seed,
            int32_t wlo, int32_t whi, gen_graph *out) {
  memset(out, 0, sizeof(*out));
  if (n <= 0 || (dim != 2 && dim != 3) || mean_degree <= 0 || wlo < 1 || whi < wlo)
    return -1;
  const double PI = 3.14159265358979323846;
  double r = dim == 2 ? sqrt(mean_degree / (PI * (double)n))
                      : cbrt(3.0 * mean_degree / (4.0 * PI * (double)n));
  int64_t nc = (int64_t)floor(1.0 / r);
  if (nc < 1) nc = 1;
  int64_t ncells = dim == 2 ? nc * nc : nc * nc * nc;
  double *raw = (double *)malloc(sizeof(double) * (size_t)n * dim);
  int64_t *cell = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
  int64_t *cstart = (int64_t *)calloc((size_t)ncells + 1, sizeof(int64_t));
  int32_t *order = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
  if (!raw || !cell || !cstart || !order) goto fail0;
  uint64_t st = seed;
  for (int32_t i = 0; i < n; i++)
    for (int d = 0; d < dim; d++)
      raw[(size_t)i * dim + d] = (double)(gen_splitmix64_next(&st) >> 11) * 0x1.0p-53;
  for (int32_t i = 0; i < n; i++) {
    int64_t c[3];
    for (int d = 0; d < dim; d++) {
      int64_t q = (int64_t)(raw[(size_t)i * dim + d] * (double)nc);
      if (q >= nc) q = nc - 1;
      c[d] = q;
    }
    cell[i] = dim == 2 ? c[1] * nc + c[0] : (c[2] * nc + c[1]) * nc + c[0];
    cstart[cell[i] + 1]++;
  }
  for (int64_t c = 0; c < ncells; c++) cstart[c + 1] += cstart[c];
  {
    int64_t *fill = (int64_t *)malloc(sizeof(int64_t) * (size_t)ncells);
    if (!fill) goto fail0;
    memcpy(fill, cstart, sizeof(int64_t) * (size_t)ncells);
    for (int32_t i = 0; i < n; i++) order[fill[cell[i]]++] = i; /* stable */
    free(fill);
  }
  out->coords = (double *)malloc(sizeof(double) * (size_t)n * dim);
  out->xadj = (int32_t *)malloc(sizeof(int32_t) * ((size_t)n + 1));
  if (!out->coords || !out->xadj) goto fail1;
  for (int32_t v = 0; v < n; v++)
    for (int d = 0; d < dim; d++)
      out->coords[(size_t)v * dim + d] = raw[(size_t)order[v] * dim + d];
  /* cell of each new id: cells are contiguous id ranges now */
  int64_t *vcell = cell; /* reuse storage */
  for (int64_t c = 0; c < ncells; c++)
    for (int64_t v = cstart[c]; v < cstart[c + 1]; v++) vcell[v] = c;
  double r2 = r * r;
  const double *P = out->coords;
  /* two passes: count, then fill */
  for (int pass = 0; pass < 2; pass++) {
    int64_t pos = 0;
    if (pass == 1) {
      out->adjncy = (int32_t *)malloc(sizeof(int32_t) * (size_t)(out->narcs ? out->narcs : 1));
      out->adjwgt = (int32_t *)malloc(sizeof(int32_t) * (size_t)(out->narcs ? out->narcs : 1));
      if (!out->adjncy || !out->adjwgt) goto fail1;
    }
    for (int32_t u = 0; u < n; u++) {
      if (pass == 0) out->xadj[u] = (int32_t)pos;
      int64_t c = vcell[u];
      int64_t cx = c % nc, cy = (c / nc) % nc, cz = dim == 3 ? c / (nc * nc) : 0;
      for (int64_t dz = (dim == 3 ? -1 : 0); dz <= (dim == 3 ? 1 : 0); dz++) {
        int64_t zz = cz + dz;
        if (zz < 0 || zz >= nc) continue;
        for (int64_t dy = -1; dy <= 1; dy++) {
          int64_t yy = cy + dy;
          if (yy < 0 || yy >= nc) continue;
          for (int64_t dx = -1; dx <= 1; dx++) {
            int64_t xx = cx + dx;
            if (xx < 0 || xx >= nc) continue;
            int64_t cc = dim == 2 ? yy * nc + xx : (zz * nc + yy) * nc + xx;
            for (int64_t v = cstart[cc]; v < cstart[cc + 1]; v++) {
              if (v == u) continue;
              double s = 0.0;
              for (int d = 0; d < dim; d++) {
                double t = P[(size_t)u * dim + d] - P[(size_t)v * dim + d];
                s += t * t;
              }
              if (s < r2) {
                if (pass == 1) {
                  int32_t lo = u < v ? u : (int32_t)v, hi = u < v ? (int32_t)v : u;
                  out->adjncy[pos] = (int32_t)v;
                  out->adjwgt[pos] = wlo + (int32_t)(gen_edge_hash(seed, lo, hi) %
                                                     (uint64_t)(whi - wlo + 1));
                }
                pos++;
                if (pos >= 0x7fffffffLL) goto fail1;
              }
            }
          }
        }
      }
    }
    if (pass == 0) {
      out->xadj[n] = (int32_t)pos;
      out->narcs = pos;
    }
  }
  out->n = n;
  out->dim = dim;
  out->radius = r;
  free(raw);
  free(cell);
  free(cstart);
  free(order);
  return 0;
fail1:
  gen_free(out);
fail0:
  free(raw);
  free(cell);
  free(cstart);
  free(order);
  return -1;
}

/* ---- recursive coordinate bisection ------------------------------------ */

static const double *rcb_coords;
static int rcb_dim, rcb_axis;

/* strict total order: (coordinate on the axis, vertex id) */
static int rcb_less(int32_t a, int32_t b) {
  double x = rcb_coords[(size_t)a * rcb_dim + rcb_axis];
  double y = rcb_coords[(size_t)b * rcb_dim + rcb_axis];
  if (x != y) return x < y;
  return a < b;
}

/* Rearrange ids[lo,hi) so that its kth smallest (0-based, under rcb_less)
 * sits at lo+k with everything smaller before it.  Any correct selection
 * yields the same SET below position k because the order is total. */
static void rcb_select(int32_t *ids, int64_t lo, int64_t hi, int64_t k) {
  int64_t L = lo, R = hi - 1, target = lo + k;
  while (L < R) {
    int64_t mid = L + (R - L) / 2;
    /* median of three into ids[R] as the pivot */
    if (rcb_less(ids[mid], ids[L])) { int32_t t = ids[mid]; ids[mid] = ids[L]; ids[L] = t; }
    if (rcb_less(ids[R], ids[L])) { int32_t t = ids[R]; ids[R] = ids[L]; ids[L] = t; }
    if (rcb_less(ids[mid], ids[R])) { int32_t t = ids[mid]; ids[mid] = ids[R]; ids[R] = t; }
    int32_t pivot = ids[R];
    int64_t store = L;
    for (int64_t i = L; i < R; i++) {
      if (rcb_less(ids[i], pivot)) { int32_t t = ids[i]; ids[i] = ids[store]; ids[store] = t; store++; }
    }
    { int32_t t = ids[store]; ids[store] = ids[R]; ids[R] = t; }
    if (store == target) return;
    if (store < target) L = store + 1; else R = store - 1;
  }
}

static void rcb_rec(int32_t *ids, int64_t lo, int64_t hi, int32_t b0, int32_t kk,
                    int32_t force_axis, int32_t *part) {
  if (kk <= 1 || hi - lo <= 1) {
    for (int64_t i = lo; i < hi; i++) part[ids[i]] = b0;
    return;
  }
  int axis = force_axis;
  if (axis < 0) {
    double best = -1.0;
    for (int d = 0; d < rcb_dim; d++) {
      double mn = INFINITY, mx = -INFINITY;
      for (int64_t i = lo; i < hi; i++) {
        double x = rcb_coords[(size_t)ids[i] * rcb_dim + d];
        if (x < mn) mn = x;
        if (x > mx) mx = x;
      }
      if (mx - mn > best) { best = mx - mn; axis = d; }
    }
  }
  int32_t k1 = kk / 2;
  int64_t nlow = (hi - lo) * (int64_t)k1 / kk;
  rcb_axis = axis;
  if (nlow > 0 && nlow < hi - lo) rcb_select(ids, lo, hi, nlow);
  rcb_rec(ids, lo, lo + nlow, b0, k1, -1, part);
  rcb_rec(ids, lo + nlow, hi, b0 + k1, kk - k1, -1, part);
}

/* Recursive coordinate bisection into k blocks: split the current set at its
 * median along the longest bounding-box axis (ties by id), lower part gets the
 * lower block ids; the lower part holds floor(size * floor(kk/2) / kk)
 * vertices.  force_axis >= 0 fixes the axis of the top-level cut only. */
int gen_rcb(int32_t n, int32_t dim, const double *coords, int32_t k, int32_t force_axis,
            int32_t *part) {
  if (n <= 0 || k <= 0 || (dim != 2 && dim != 3) || force_axis >= dim) return -1;
  int32_t *ids = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
  if (!ids) return -1;
  for (int32_t i = 0; i < n; i++) ids[i] = i;
  rcb_coords = coords;
  rcb_dim = dim;
  rcb_rec(ids, 0, n, 0, k, force_axis, part);
  free(ids);
  return 0;
}

/* ---- boundary noise ----------------------------------------------------- */

static int64_t round_half_up(double x) { return (int64_t)floor(x + 0.5); }

/* Partial Fisher-Yates: move m uniformly chosen entries of a[0..N) to the front. */
static void partial_shuffle(int32_t *a, int64_t N, int64_t m, uint64_t *st) {
  for (int64_t i = 0; i < m && i < N; i++) {
    int64_t j = i + (int64_t)(gen_splitmix64_next(st) % (uint64_t)(N - i));
    int32_t t = a[i]; a[i] = a[j]; a[j] = t;
  }
}

/* Two-block noise: delta_0 / delta_1 = vertices of block 0 / 1 with a
 * neighbour in the other block, ascending.  round(frac*|delta_x|) of each are
 * chosen (side 0 first, one splitmix64 stream) and all chosen vertices switch
 * block simultaneously.  Returns the number of moved vertices. */
int64_t gen_pair_swap_noise(int32_t n, const int32_t *xadj, const int32_t *adjncy,
                            int32_t *part, double frac, uint64_t seed) {
  int32_t *d0 = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
  int32_t *d1 = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
  if (!d0 || !d1) { free(d0); free(d1); return -1; }
  int64_t n0 = 0, n1 = 0;
  for (int32_t u = 0; u < n; u++) {
    if (part[u] != 0 && part[u] != 1) continue;
    int other = 1 - part[u], hit = 0;
    for (int32_t e = xadj[u]; e < xadj[u + 1]; e++)
      if (part[adjncy[e]] == other) { hit = 1; break; }
    if (hit) { if (part[u] == 0) d0[n0++] = u; else d1[n1++] = u; }
  }
  uint64_t st = seed;
  int64_t m0 = round_half_up(frac * (double)n0), m1 = round_half_up(frac * (double)n1);
  partial_shuffle(d0, n0, m0, &st);
  partial_shuffle(d1, n1, m1, &st);
  for (int64_t i = 0; i < m0; i++) part[d0[i]] = 1;
  for (int64_t i = 0; i < m1; i++) part[d1[i]] = 0;
  free(d0);
  free(d1);
  return m0 + m1;
}

/* k-way noise: delta = vertices with a neighbour in another block, ascending;
 * round(frac*|delta|) chosen; each moves to the block of its smallest-id
 * foreign neighbour in the ORIGINAL partition, all simultaneously. */
int64_t gen_global_noise(int32_t n, const int32_t *xadj, const int32_t *adjncy,
                         int32_t *part, double frac, uint64_t seed) {
  int32_t *d = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
  if (!d) return -1;
  int64_t nd = 0;
  for (int32_t u = 0; u < n; u++) {
    for (int32_t e = xadj[u]; e < xadj[u + 1]; e++)
      if (part[adjncy[e]] != part[u]) { d[nd++] = u; break; }
  }
  uint64_t st = seed;
  int64_t m = round_half_up(frac * (double)nd);
  partial_shuffle(d, nd, m, &st);
  int32_t *target = (int32_t *)malloc(sizeof(int32_t) * (size_t)(m ? m : 1));
  if (!target) { free(d); return -1; }
  for (int64_t i = 0; i < m; i++) {
    int32_t u = d[i], best = -1;
    for (int32_t e = xadj[u]; e < xadj[u + 1]; e++) {
      int32_t v = adjncy[e];
      if (part[v] != part[u] && (best < 0 || v < best)) best = v;
    }
    target[i] = part[best];
  }
  for (int64_t i = 0; i < m; i++) part[d[i]] = target[i];
  free(target);
  free(d);
  return m;
}
