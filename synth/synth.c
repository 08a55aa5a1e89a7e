/*
 * Seeded synthetic inputs for the skew-symmetric SpMV library and its oracle.
 *
 * This module only builds inputs: sparsity patterns (2D/3D grid stencils,
 * random geometric graphs, Chung-Lu power-law graphs), a random relabelling
 * of the nodes, and i.i.d. values for the stored strictly-lower entries.  It
 * contains none of the method's arithmetic (no reordering, splitting or
 * products).  Because every stored value is drawn i.i.d. from a distribution
 * symmetric about zero, drawing the value of the stored entry (max, min) of
 * each edge directly is the same in law as drawing a_ij and setting
 * a_ji = -a_ij before the relabelling.
 *
 * Random numbers: SplitMix64 (Steele, Lea and Flood, OOPSLA 2014), one stream
 * per purpose (structure, relabelling, values) derived from the seed.
 * Uniforms use the top 53 bits; normals use the Box-Muller transform;
 * permutations use the Fisher-Yates shuffle.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define SYN_OK 0
#define SYN_EINVAL 1
#define SYN_ENOMEM 2

enum { VAL_UNIFORM = 0, VAL_NORMAL = 1, VAL_UNIFORM_F32 = 2, VAL_INT4 = 3, VAL_ONES = 4 };

static uint64_t sm_next(uint64_t *s) {
  uint64_t z = (*s += 0x9E3779B97F4A7C15ULL);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}
static double sm_u01(uint64_t *s) { return (double)(sm_next(s) >> 11) * 0x1.0p-53; }
static double sm_normal(uint64_t *s) {
  double u1 = sm_u01(s), u2 = sm_u01(s);
  if (u1 <= 0.0) u1 = 0x1.0p-53;
  return sqrt(-2.0 * log(u1)) * cos(6.283185307179586476925 * u2);
}
static uint64_t stream_seed(uint64_t seed, uint64_t k) {
  uint64_t s = seed ^ (0xD1B54A32D192ED03ULL * (k + 1));
  return sm_next(&s);
}

typedef struct {
  int64_t m, cap;
  int32_t *a, *b;
} edge_list;

static int el_push(edge_list *e, int32_t a, int32_t b) {
  if (e->m == e->cap) {
    int64_t nc = e->cap ? e->cap * 2 : 1024;
    int32_t *na = (int32_t *)realloc(e->a, (size_t)nc * sizeof(int32_t));
    if (!na) return SYN_ENOMEM;
    e->a = na;
    int32_t *nb = (int32_t *)realloc(e->b, (size_t)nc * sizeof(int32_t));
    if (!nb) return SYN_ENOMEM;
    e->b = nb;
    e->cap = nc;
  }
  e->a[e->m] = a;
  e->b[e->m] = b;
  e->m++;
  return SYN_OK;
}
static void el_free(edge_list *e) {
  free(e->a);
  free(e->b);
  e->a = e->b = NULL;
  e->m = e->cap = 0;
}

/* Output: strictly lower CSR (rows ascending, columns ascending within a row). */
typedef struct {
  int64_t n, nnz;
  int32_t *rowptr, *col;
  double *val;
} syn_matrix;

void syn_free(syn_matrix *m) {
  if (!m) return;
  free(m->rowptr);
  free(m->col);
  free(m->val);
  m->rowptr = m->col = NULL;
  m->val = NULL;
  m->n = m->nnz = 0;
}

static double draw_value(uint64_t *s, int kind) {
  switch (kind) {
    case VAL_NORMAL: return sm_normal(s);
    case VAL_UNIFORM_F32: return (double)(float)(2.0 * sm_u01(s) - 1.0);
    case VAL_INT4: return (double)((int)(sm_next(s) % 9) - 4);
    case VAL_ONES: return 1.0;
    default: return 2.0 * sm_u01(s) - 1.0;
  }
}

/* Random relabelling of the nodes (Fisher-Yates), orientation of every edge as
 * (larger label, smaller label), stable counting sorts to CSR order, then one
 * value per stored entry in CSR order.  Duplicate edges must not occur. */
static int finish(int64_t n, edge_list *e, uint64_t seed, int value_kind, int relabel,
                  syn_matrix *out) {
  memset(out, 0, sizeof(*out));
  int64_t m = e->m;
  int32_t *lab = (int32_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(int32_t));
  int32_t *r = (int32_t *)malloc((size_t)(m > 0 ? m : 1) * sizeof(int32_t));
  int32_t *c = (int32_t *)malloc((size_t)(m > 0 ? m : 1) * sizeof(int32_t));
  int32_t *tmp = (int32_t *)malloc((size_t)(m > 0 ? m : 1) * sizeof(int32_t));
  int64_t *cnt = (int64_t *)calloc((size_t)n + 1, sizeof(int64_t));
  out->rowptr = (int32_t *)calloc((size_t)n + 1, sizeof(int32_t));
  out->col = (int32_t *)malloc((size_t)(m > 0 ? m : 1) * sizeof(int32_t));
  out->val = (double *)malloc((size_t)(m > 0 ? m : 1) * sizeof(double));
  if (!lab || !r || !c || !tmp || !cnt || !out->rowptr || !out->col || !out->val) {
    free(lab); free(r); free(c); free(tmp); free(cnt);
    syn_free(out);
    return SYN_ENOMEM;
  }
  for (int64_t i = 0; i < n; i++) lab[i] = (int32_t)i;
  if (relabel) {
    uint64_t ps = stream_seed(seed, 1);
    for (int64_t i = n - 1; i > 0; i--) {
      int64_t j = (int64_t)(sm_u01(&ps) * (double)(i + 1));
      if (j > i) j = i;
      int32_t t = lab[i];
      lab[i] = lab[j];
      lab[j] = t;
    }
  }
  for (int64_t k = 0; k < m; k++) {
    int32_t p = lab[e->a[k]], q = lab[e->b[k]];
    r[k] = p > q ? p : q;
    c[k] = p > q ? q : p;
  }
  /* stable counting sort by column, then by row -> (row, col) order */
  int64_t *order = (int64_t *)malloc((size_t)(m > 0 ? m : 1) * sizeof(int64_t));
  int64_t *order2 = (int64_t *)malloc((size_t)(m > 0 ? m : 1) * sizeof(int64_t));
  if (!order || !order2) {
    free(lab); free(r); free(c); free(tmp); free(cnt); free(order); free(order2);
    syn_free(out);
    return SYN_ENOMEM;
  }
  memset(cnt, 0, (size_t)(n + 1) * sizeof(int64_t));
  for (int64_t k = 0; k < m; k++) cnt[c[k] + 1]++;
  for (int64_t i = 0; i < n; i++) cnt[i + 1] += cnt[i];
  for (int64_t k = 0; k < m; k++) order[cnt[c[k]]++] = k;
  memset(cnt, 0, (size_t)(n + 1) * sizeof(int64_t));
  for (int64_t k = 0; k < m; k++) cnt[r[k] + 1]++;
  for (int64_t i = 0; i < n; i++) cnt[i + 1] += cnt[i];
  for (int64_t i = 0; i <= n; i++) out->rowptr[i] = (int32_t)cnt[i];
  for (int64_t t = 0; t < m; t++) {
    int64_t k = order[t];
    order2[cnt[r[k]]++] = k;
  }
  for (int64_t t = 0; t < m; t++) out->col[t] = c[order2[t]];
  uint64_t vs = stream_seed(seed, 2);
  for (int64_t t = 0; t < m; t++) out->val[t] = draw_value(&vs, value_kind);
  out->n = n;
  out->nnz = m;
  free(lab); free(r); free(c); free(tmp); free(cnt); free(order); free(order2);
  return SYN_OK;
}

/* 2D grid k x k, node id r*k + c, edges to the right and downward neighbour
 * (five-point stencil graph): 2k(k-1) edges. */
int syn_grid2d(int32_t k, uint64_t seed, int value_kind, int relabel, syn_matrix *out) {
  if (k < 0) return SYN_EINVAL;
  int64_t n = (int64_t)k * k;
  edge_list e = {0};
  for (int32_t r = 0; r < k; r++)
    for (int32_t c = 0; c < k; c++) {
      int32_t id = r * k + c;
      if (c + 1 < k && el_push(&e, id, id + 1)) goto oom;
      if (r + 1 < k && el_push(&e, id, id + k)) goto oom;
    }
  {
    int rc = finish(n, &e, seed, value_kind, relabel, out);
    el_free(&e);
    return rc;
  }
oom:
  el_free(&e);
  return SYN_ENOMEM;
}

/* 3D grid k^3, node id x + k(y + k z), edges along +x, +y, +z (seven-point
 * stencil graph): 3k^2(k-1) edges. */
int syn_grid3d(int32_t k, uint64_t seed, int value_kind, int relabel, syn_matrix *out) {
  if (k < 0) return SYN_EINVAL;
  int64_t n = (int64_t)k * k * k;
  if (n > 0x7fffffffLL) return SYN_EINVAL;
  edge_list e = {0};
  for (int32_t z = 0; z < k; z++)
    for (int32_t y = 0; y < k; y++)
      for (int32_t x = 0; x < k; x++) {
        int32_t id = x + k * (y + k * z);
        if (x + 1 < k && el_push(&e, id, id + 1)) goto oom;
        if (y + 1 < k && el_push(&e, id, id + k)) goto oom;
        if (z + 1 < k && el_push(&e, id, id + k * k)) goto oom;
      }
  {
    int rc = finish(n, &e, seed, value_kind, relabel, out);
    el_free(&e);
    return rc;
  }
oom:
  el_free(&e);
  return SYN_ENOMEM;
}

/* Radius r such that (n-1) * P(|X - Y| < r) = deg for X, Y uniform in the unit
 * square, with P = pi r^2 - 8 r^3 / 3 + r^4 / 2 (valid for r <= 1). */
double syn_rgg2d_radius(int64_t n, double deg) {
  if (n < 2) return 0.0;
  double lo = 0.0, hi = 1.0, target = deg / (double)(n - 1);
  for (int it = 0; it < 200; it++) {
    double r = 0.5 * (lo + hi);
    double p = 3.141592653589793 * r * r - 8.0 * r * r * r / 3.0 + 0.5 * r * r * r * r;
    if (p < target) lo = r; else hi = r;
  }
  return 0.5 * (lo + hi);
}

/* Random geometric graph: n points uniform in [0,1)^2, an edge when the
 * Euclidean distance is strictly below r; cell-grid binning with cells no
 * smaller than r, each unordered pair examined once. */
int syn_rgg2d(int64_t n, double deg, uint64_t seed, int value_kind, int relabel, syn_matrix *out) {
  if (n < 0 || n > 0x7fffffffLL) return SYN_EINVAL;
  double r = syn_rgg2d_radius(n, deg);
  double r2 = r * r;
  double *px = (double *)malloc((size_t)(n > 0 ? n : 1) * sizeof(double));
  double *py = (double *)malloc((size_t)(n > 0 ? n : 1) * sizeof(double));
  uint64_t ss = stream_seed(seed, 0);
  int64_t nc = (r > 0.0) ? (int64_t)floor(1.0 / r) : 1;
  if (nc < 1) nc = 1;
  if (nc > 46340) nc = 46340;
  int64_t ncell = nc * nc;
  int64_t *cstart = (int64_t *)calloc((size_t)ncell + 1, sizeof(int64_t));
  int32_t *pts = (int32_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(int32_t));
  int64_t *cell = (int64_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(int64_t));
  edge_list e = {0};
  if (!px || !py || !cstart || !pts || !cell) goto oom;
  for (int64_t i = 0; i < n; i++) {
    px[i] = sm_u01(&ss);
    py[i] = sm_u01(&ss);
    int64_t cx = (int64_t)(px[i] * (double)nc), cy = (int64_t)(py[i] * (double)nc);
    if (cx >= nc) cx = nc - 1;
    if (cy >= nc) cy = nc - 1;
    cell[i] = cy * nc + cx;
    cstart[cell[i] + 1]++;
  }
  for (int64_t q = 0; q < ncell; q++) cstart[q + 1] += cstart[q];
  {
    int64_t *fill = (int64_t *)malloc((size_t)ncell * sizeof(int64_t));
    if (!fill) goto oom;
    memcpy(fill, cstart, (size_t)ncell * sizeof(int64_t));
    for (int64_t i = 0; i < n; i++) pts[fill[cell[i]]++] = (int32_t)i;
    free(fill);
  }
  {
    static const int dxs[4] = {1, -1, 0, 1}, dys[4] = {0, 1, 1, 1};
    for (int64_t cy = 0; cy < nc; cy++)
      for (int64_t cx = 0; cx < nc; cx++) {
        int64_t q = cy * nc + cx;
        for (int64_t s = cstart[q]; s < cstart[q + 1]; s++) {
          int32_t i = pts[s];
          for (int64_t t = s + 1; t < cstart[q + 1]; t++) {
            int32_t j = pts[t];
            double dx = px[i] - px[j], dy = py[i] - py[j];
            if (dx * dx + dy * dy < r2 && el_push(&e, i, j)) goto oom;
          }
          for (int d = 0; d < 4; d++) {
            int64_t ox = cx + dxs[d], oy = cy + dys[d];
            if (ox < 0 || ox >= nc || oy < 0 || oy >= nc) continue;
            int64_t o = oy * nc + ox;
            for (int64_t t = cstart[o]; t < cstart[o + 1]; t++) {
              int32_t j = pts[t];
              double dx = px[i] - px[j], dy = py[i] - py[j];
              if (dx * dx + dy * dy < r2 && el_push(&e, i, j)) goto oom;
            }
          }
        }
      }
  }
  free(px); free(py); free(cstart); free(pts); free(cell);
  {
    int rc = finish(n, &e, seed, value_kind, relabel, out);
    el_free(&e);
    return rc;
  }
oom:
  free(px); free(py); free(cstart); free(pts); free(cell);
  el_free(&e);
  return SYN_ENOMEM;
}

/* Radius r such that (n-1) * P(|X - Y| < r) = deg for X, Y uniform in the unit
 * cube, with P = 4 pi r^3 / 3 - 3 pi r^4 / 2 + 8 r^5 / 5 - r^6 / 6 (the
 * distribution function of the distance between two uniform points of the
 * unit cube, valid for r <= 1). */
double syn_rgg3d_radius(int64_t n, double deg) {
  if (n < 2) return 0.0;
  const double pi = 3.141592653589793;
  double lo = 0.0, hi = 1.0, target = deg / (double)(n - 1);
  for (int it = 0; it < 200; it++) {
    double r = 0.5 * (lo + hi);
    double r3 = r * r * r;
    double p = 4.0 * pi * r3 / 3.0 - 1.5 * pi * r3 * r + 1.6 * r3 * r * r - r3 * r3 / 6.0;
    if (p < target) lo = r; else hi = r;
  }
  return 0.5 * (lo + hi);
}

/* Random geometric graph in 3D: n points uniform in [0,1)^3, an edge when the
 * Euclidean distance is strictly below r; cell-grid binning with cells no
 * smaller than r, each unordered pair examined once (own cell, then the 13
 * neighbouring cells that come later in (z, y, x) order). */
int syn_rgg3d(int64_t n, double deg, uint64_t seed, int value_kind, int relabel, syn_matrix *out) {
  if (n < 0 || n > 0x7fffffffLL) return SYN_EINVAL;
  double r = syn_rgg3d_radius(n, deg);
  double r2 = r * r;
  double *px = (double *)malloc((size_t)(n > 0 ? n : 1) * sizeof(double));
  double *py = (double *)malloc((size_t)(n > 0 ? n : 1) * sizeof(double));
  double *pz = (double *)malloc((size_t)(n > 0 ? n : 1) * sizeof(double));
  uint64_t ss = stream_seed(seed, 0);
  int64_t nc = (r > 0.0) ? (int64_t)floor(1.0 / r) : 1;
  if (nc > (int64_t)cbrt((double)n) + 1) nc = (int64_t)cbrt((double)n) + 1;  /* about one cell per point at most */
  if (nc < 1) nc = 1;
  int64_t ncell = nc * nc * nc;
  int64_t *cstart = (int64_t *)calloc((size_t)ncell + 1, sizeof(int64_t));
  int32_t *pts = (int32_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(int32_t));
  int64_t *cell = (int64_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(int64_t));
  edge_list e = {0};
  if (!px || !py || !pz || !cstart || !pts || !cell) goto oom;
  for (int64_t i = 0; i < n; i++) {
    px[i] = sm_u01(&ss);
    py[i] = sm_u01(&ss);
    pz[i] = sm_u01(&ss);
    int64_t cx = (int64_t)(px[i] * (double)nc), cy = (int64_t)(py[i] * (double)nc),
            cz = (int64_t)(pz[i] * (double)nc);
    if (cx >= nc) cx = nc - 1;
    if (cy >= nc) cy = nc - 1;
    if (cz >= nc) cz = nc - 1;
    cell[i] = (cz * nc + cy) * nc + cx;
    cstart[cell[i] + 1]++;
  }
  for (int64_t q = 0; q < ncell; q++) cstart[q + 1] += cstart[q];
  {
    int64_t *fill = (int64_t *)malloc((size_t)ncell * sizeof(int64_t));
    if (!fill) goto oom;
    memcpy(fill, cstart, (size_t)ncell * sizeof(int64_t));
    for (int64_t i = 0; i < n; i++) pts[fill[cell[i]]++] = (int32_t)i;
    free(fill);
  }
  {
    /* the 13 of the 26 neighbouring cells that follow the own cell */
    int off[13][3], no = 0;
    for (int dz = -1; dz <= 1; dz++)
      for (int dy = -1; dy <= 1; dy++)
        for (int dx = -1; dx <= 1; dx++)
          if (dz > 0 || (dz == 0 && dy > 0) || (dz == 0 && dy == 0 && dx > 0)) {
            off[no][0] = dx;
            off[no][1] = dy;
            off[no][2] = dz;
            no++;
          }
    for (int64_t cz = 0; cz < nc; cz++)
      for (int64_t cy = 0; cy < nc; cy++)
        for (int64_t cx = 0; cx < nc; cx++) {
          int64_t q = (cz * nc + cy) * nc + cx;
          for (int64_t s = cstart[q]; s < cstart[q + 1]; s++) {
            int32_t i = pts[s];
            for (int64_t t = s + 1; t < cstart[q + 1]; t++) {
              int32_t j = pts[t];
              double dx = px[i] - px[j], dy = py[i] - py[j], dz = pz[i] - pz[j];
              if (dx * dx + dy * dy + dz * dz < r2 && el_push(&e, i, j)) goto oom;
            }
            for (int d = 0; d < no; d++) {
              int64_t ox = cx + off[d][0], oy = cy + off[d][1], oz = cz + off[d][2];
              if (ox < 0 || ox >= nc || oy < 0 || oy >= nc || oz < 0 || oz >= nc) continue;
              int64_t o = (oz * nc + oy) * nc + ox;
              for (int64_t t = cstart[o]; t < cstart[o + 1]; t++) {
                int32_t j = pts[t];
                double dx = px[i] - px[j], dy = py[i] - py[j], dz = pz[i] - pz[j];
                if (dx * dx + dy * dy + dz * dz < r2 && el_push(&e, i, j)) goto oom;
              }
            }
          }
        }
  }
  free(px); free(py); free(pz); free(cstart); free(pts); free(cell);
  {
    int rc = finish(n, &e, seed, value_kind, relabel, out);
    el_free(&e);
    return rc;
  }
oom:
  free(px); free(py); free(pz); free(cstart); free(pts); free(cell);
  el_free(&e);
  return SYN_ENOMEM;
}

/* Chung-Lu graph with expected degrees w_i = C (i + i0)^(-1/(gamma-1)),
 * i = 0..n-1 (non-increasing).  C makes the mean weight equal `deg`; i0 is
 * chosen so that w_0^2 = sum(w), which keeps every pair probability
 * min(1, w_u w_v / sum(w)) at most 1 up to rounding.  Edges are sampled with
 * the geometric skipping method of Miller and Hagberg (WAW 2011). */
int syn_chung_lu(int64_t n, double deg, double gamma, uint64_t seed, int value_kind, int relabel,
                 syn_matrix *out) {
  if (n < 0 || n > 0x7fffffffLL || !(gamma > 1.0) || !(deg >= 0.0)) return SYN_EINVAL;
  double a = 1.0 / (gamma - 1.0);
  double S = deg * (double)n;
  double *w = (double *)malloc((size_t)(n > 0 ? n : 1) * sizeof(double));
  edge_list e = {0};
  if (!w) return SYN_ENOMEM;
  if (n >= 2 && S > 0.0) {
    /* i0 from the integral approximation of sum (i + i0)^-a  (a != 1) */
    double lo = 1e-9, hi = (double)n;
    for (int it = 0; it < 200; it++) {
      double i0 = sqrt(lo * hi);
      double Z = (a == 1.0) ? log(((double)n + i0) / i0)
                            : (pow((double)n + i0, 1.0 - a) - pow(i0, 1.0 - a)) / (1.0 - a);
      double g = Z * pow(i0, a) - sqrt(S);
      if (g < 0.0) lo = i0; else hi = i0;
    }
    double i0 = sqrt(lo * hi), Z = 0.0;
    for (int64_t i = 0; i < n; i++) Z += pow((double)i + i0, -a);
    double C = S / Z;
    for (int64_t i = 0; i < n; i++) w[i] = C * pow((double)i + i0, -a);
    uint64_t ss = stream_seed(seed, 0);
    for (int64_t u = 0; u < n - 1; u++) {
      int64_t v = u + 1;
      double p = w[u] * w[v] / S;
      if (p > 1.0) p = 1.0;
      while (v < n && p > 0.0) {
        if (p != 1.0) {
          double rr = sm_u01(&ss);
          if (rr <= 0.0) rr = 0x1.0p-53;
          double skip = floor(log(rr) / log1p(-p));
          if (skip > (double)(n - v)) skip = (double)(n - v);
          v += (int64_t)skip;
        }
        if (v < n) {
          double q = w[u] * w[v] / S;
          if (q > 1.0) q = 1.0;
          double rr = sm_u01(&ss);
          if (rr < q / p && el_push(&e, (int32_t)u, (int32_t)v)) goto oom;
          p = q;
          v++;
        }
      }
    }
  }
  free(w);
  {
    int rc = finish(n, &e, seed, value_kind, relabel, out);
    el_free(&e);
    return rc;
  }
oom:
  free(w);
  el_free(&e);
  return SYN_ENOMEM;
}

/* Build a matrix from a caller-given undirected edge list (no duplicates, no
 * self loops). */
int syn_from_edges(int64_t n, int64_t m, const int32_t *a, const int32_t *b, uint64_t seed,
                   int value_kind, int relabel, syn_matrix *out) {
  if (n < 0 || m < 0) return SYN_EINVAL;
  edge_list e = {0};
  for (int64_t k = 0; k < m; k++) {
    if (a[k] < 0 || b[k] < 0 || a[k] >= n || b[k] >= n || a[k] == b[k]) {
      el_free(&e);
      return SYN_EINVAL;
    }
    if (el_push(&e, a[k], b[k])) {
      el_free(&e);
      return SYN_ENOMEM;
    }
  }
  int rc = finish(n, &e, seed, value_kind, relabel, out);
  el_free(&e);
  return rc;
}

/* m values from distribution `kind` (stream 3 of the seed). */
void syn_values(int64_t m, uint64_t seed, int kind, double *outv) {
  uint64_t s = stream_seed(seed, 3);
  for (int64_t i = 0; i < m; i++) outv[i] = draw_value(&s, kind);
}
