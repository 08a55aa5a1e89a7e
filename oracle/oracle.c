/*
 * Oracle for the skew-symmetric SpMV path.
 *
 * TEST INFRASTRUCTURE ONLY.  Plain, slow, single-threaded host C that states
 * what the path computes (or_csr_spmv_par alone shares its rows among the
 * host's threads, for the all-core CPU baseline, with the same sums).  Only the tests, the smoke check and the benchmark's
 * CPU-baseline leg load it; the library never does, and it shares no code,
 * header or constant with the GPU path.  Built with -O2 -fno-fast-math
 * -ffp-contract=off so that every product and sum is rounded as written.
 *
 * Conventions.  The input is the strictly lower triangle L of a skew-symmetric
 * S (S = -S^T, zero diagonal) in CSR: rowptr[n+1], col[nnz], val[nnz].  The
 * stored entry l_ij (i > j) stands for S_ij = l_ij and S_ji = -l_ij (the
 * symmetric-pair rule of eqs. (2)-(6), Section 3.1.2).  The system matrix is
 * A = alpha*I + S (shifted skew-symmetric form, Section 1).  The "_ex" and
 * "_sign" variants also cover the symmetric case (S_ji = +l_ij, the sign
 * parameter tsign = +1) and a diagonal array D held beside the triangle as in
 * SSS storage (Section 1), for A = alpha*I + D + S.
 *
 * Parity notes: every function here is pinned by the CPU tests against
 * closed forms, dense products, brute force or hand-derived cases.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ------------------------------------------------------------------------ */
/* Input validation (storage of one triangle, Sections 1 and 3).
 * Returns 0 when (rowptr, col) is a strictly lower CSR with strictly
 * increasing columns in every row; 1 for malformed sizes or row pointers;
 * 2 for an entry outside the strictly lower triangle; 3 for unsorted or
 * duplicate columns.  Rows are checked in order, entries in order; the first
 * violation decides the code. */
int or_validate(int64_t n, int64_t nnz, const int32_t *rowptr, const int32_t *col) {
  if (n < 0 || nnz < 0 || n > 0x7fffffffLL || nnz > 0x7fffffffLL) return 1;
  if (!rowptr) return 1;
  if (nnz > 0 && !col) return 1;
  if (rowptr[0] != 0 || rowptr[n] != nnz) return 1;
  for (int64_t i = 0; i < n; i++)
    if (rowptr[i + 1] < rowptr[i]) return 1;
  for (int64_t i = 0; i < n; i++) {
    for (int64_t e = rowptr[i]; e < rowptr[i + 1]; e++) {
      if (col[e] < 0 || col[e] >= i) return 2;
      if (e > rowptr[i] && col[e] <= col[e - 1]) return 3;
    }
  }
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Graph of S: N(v) = {j : (v,j) stored} U {i : (i,v) stored}. */
typedef struct {
  int32_t n;
  int32_t *deg, *ptr, *adj;
} graph;

static int graph_build(int32_t n, const int32_t *rowptr, const int32_t *col, graph *g) {
  g->n = n;
  g->deg = (int32_t *)calloc((size_t)n + 1, sizeof(int32_t));
  g->ptr = (int32_t *)calloc((size_t)n + 1, sizeof(int32_t));
  int64_t m = n > 0 ? rowptr[n] : 0;
  g->adj = (int32_t *)malloc((size_t)(2 * m + 1) * sizeof(int32_t));
  int32_t *fill = (int32_t *)calloc((size_t)n + 1, sizeof(int32_t));
  if (!g->deg || !g->ptr || !g->adj || !fill) {
    free(fill);
    return 1;
  }
  for (int32_t i = 0; i < n; i++)
    for (int32_t e = rowptr[i]; e < rowptr[i + 1]; e++) {
      g->deg[i]++;
      g->deg[col[e]]++;
    }
  for (int32_t i = 0; i < n; i++) g->ptr[i + 1] = g->ptr[i] + g->deg[i];
  for (int32_t i = 0; i < n; i++) fill[i] = g->ptr[i];
  for (int32_t i = 0; i < n; i++)
    for (int32_t e = rowptr[i]; e < rowptr[i + 1]; e++) {
      int32_t j = col[e];
      g->adj[fill[i]++] = j;
      g->adj[fill[j]++] = i;
    }
  free(fill);
  return 0;
}
static void graph_free(graph *g) {
  free(g->deg);
  free(g->ptr);
  free(g->adj);
}

/* (deg, index) order used by every tie-break of the reordering. */
static const int32_t *g_cmp_deg;
static int less_deg_idx(int32_t a, int32_t b) {
  return g_cmp_deg[a] < g_cmp_deg[b] || (g_cmp_deg[a] == g_cmp_deg[b] && a < b);
}
static int cmp_deg_idx(const void *pa, const void *pb) {
  int32_t a = *(const int32_t *)pa, b = *(const int32_t *)pb;
  if (a == b) return 0;
  return less_deg_idx(a, b) ? -1 : 1;
}

/* Level structure of a BFS from s inside its component.  Returns the
 * eccentricity (number of levels - 1) and the nodes of the last level in
 * last[0..*nlast).  `stamp`/`id` mark visited nodes without clearing. */
static int32_t bfs_levels(const graph *g, int32_t s, int32_t *queue, int32_t *stamp, int32_t id,
                          int32_t *last, int32_t *nlast) {
  int32_t head = 0, tail = 0;
  queue[tail++] = s;
  stamp[s] = id;
  int32_t level = 0, level_start = 0, level_end = 1;
  for (;;) {
    while (head < level_end) {
      int32_t v = queue[head++];
      for (int32_t e = g->ptr[v]; e < g->ptr[v + 1]; e++) {
        int32_t u = g->adj[e];
        if (stamp[u] != id) {
          stamp[u] = id;
          queue[tail++] = u;
        }
      }
    }
    if (tail == level_end) break; /* no next level */
    level++;
    level_start = level_end;
    level_end = tail;
  }
  *nlast = level_end - level_start;
  memcpy(last, queue + level_start, (size_t)(*nlast) * sizeof(int32_t));
  return level;
}

/* Reverse Cuthill-McKee with fixed tie-breaking (the reordering that turns
 * the matrix into a band, Sections 1 and 3.1.2; Cuthill-McKee, Section 2).
 *   (a) s = the unvisited node minimising (deg, index);
 *   (b) George-Liu pseudo-peripheral search from s: build the BFS level
 *       structure; take u of minimum (deg, index) in the last level; if u has
 *       a larger eccentricity, move to u and repeat, else stop;
 *   (c) Cuthill-McKee BFS from s: pop v, append v to the order, push the
 *       unvisited neighbours of v in ascending (deg, index);
 *   repeat (a)-(c) until every node is ordered; finally reverse the whole
 *   concatenated order: perm[k] = order[n-1-k] (new position k holds old node
 *   perm[k]).  Returns 0, or 1 when out of memory. */
int or_rcm(int32_t n, const int32_t *rowptr, const int32_t *col, int32_t *perm) {
  if (n <= 0) return 0;
  graph g;
  if (graph_build(n, rowptr, col, &g)) {
    graph_free(&g);
    return 1;
  }
  int32_t *order = (int32_t *)malloc((size_t)n * sizeof(int32_t));
  int32_t *byrank = (int32_t *)malloc((size_t)n * sizeof(int32_t));
  int32_t *queue = (int32_t *)malloc((size_t)n * sizeof(int32_t));
  int32_t *stamp = (int32_t *)calloc((size_t)n, sizeof(int32_t));
  int32_t *last = (int32_t *)malloc((size_t)n * sizeof(int32_t));
  int32_t *nb = (int32_t *)malloc((size_t)n * sizeof(int32_t));
  char *visited = (char *)calloc((size_t)n, 1);
  if (!order || !byrank || !queue || !stamp || !last || !nb || !visited) {
    free(order); free(byrank); free(queue); free(stamp); free(last); free(nb); free(visited);
    graph_free(&g);
    return 1;
  }
  g_cmp_deg = g.deg;
  /* all nodes in ascending (deg, index): step (a) scans this list */
  for (int32_t v = 0; v < n; v++) byrank[v] = v;
  qsort(byrank, (size_t)n, sizeof(int32_t), cmp_deg_idx);

  int32_t nord = 0, scan = 0, bfs_id = 0;
  while (nord < n) {
    /* (a) */
    while (visited[byrank[scan]]) scan++;
    int32_t s = byrank[scan];
    /* (b) */
    int32_t nlast;
    int32_t ecc_s = bfs_levels(&g, s, queue, stamp, ++bfs_id, last, &nlast);
    for (;;) {
      int32_t u = last[0];
      for (int32_t t = 1; t < nlast; t++)
        if (less_deg_idx(last[t], u)) u = last[t];
      if (u == s) break;
      int32_t nlast_u;
      int32_t ecc_u = bfs_levels(&g, u, queue, stamp, ++bfs_id, nb, &nlast_u);
      if (ecc_u > ecc_s) {
        s = u;
        ecc_s = ecc_u;
        nlast = nlast_u;
        memcpy(last, nb, (size_t)nlast * sizeof(int32_t));
      } else {
        break;
      }
    }
    /* (c): the order array doubles as the FIFO queue */
    int32_t head = nord;
    visited[s] = 1;
    order[nord++] = s;
    while (head < nord) {
      int32_t v = order[head++];
      int32_t k = 0;
      for (int32_t e = g.ptr[v]; e < g.ptr[v + 1]; e++)
        if (!visited[g.adj[e]]) nb[k++] = g.adj[e];
      qsort(nb, (size_t)k, sizeof(int32_t), cmp_deg_idx);
      for (int32_t t = 0; t < k; t++) {
        visited[nb[t]] = 1;
        order[nord++] = nb[t];
      }
    }
  }
  for (int32_t k = 0; k < n; k++) perm[k] = order[n - 1 - k];
  free(order); free(byrank); free(queue); free(stamp); free(last); free(nb); free(visited);
  graph_free(&g);
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Symmetric permutation B = P A P^T, B[k,l] = S[perm[k], perm[l]], stored as
 * its strictly lower triangle.  A stored l_ij (i > j) lands at
 * (p, q) = (iperm[i], iperm[j]); if p > q it is stored as l_ij at (p, q),
 * otherwise as -l_ij at (q, p), because S_ji = -S_ij (eq. (2)).  Rows are
 * sorted by column.  Output arrays have n+1 and nnz entries. */
typedef struct {
  int32_t c;
  double v;
} cv_pair;
int or_permute_sign(int32_t n, const int32_t *rowptr, const int32_t *col, const double *val,
                    const int32_t *perm, double tsign, int32_t *orow, int32_t *ocol, double *oval);

static int cmp_cv(const void *a, const void *b) {
  int32_t x = ((const cv_pair *)a)->c, y = ((const cv_pair *)b)->c;
  return (x > y) - (x < y);
}

int or_permute(int32_t n, const int32_t *rowptr, const int32_t *col, const double *val,
               const int32_t *perm, int32_t *orow, int32_t *ocol, double *oval) {
  return or_permute_sign(n, rowptr, col, val, perm, -1.0, orow, ocol, oval);
}

/* The same with the sign of the transposed entry: tsign = -1 for a
 * skew-symmetric matrix (A_ji = -A_ij), +1 for a symmetric one. */
int or_permute_sign(int32_t n, const int32_t *rowptr, const int32_t *col, const double *val,
                    const int32_t *perm, double tsign, int32_t *orow, int32_t *ocol, double *oval) {
  if (n < 0) return 1;
  int32_t nnz = n > 0 ? rowptr[n] : 0;
  int32_t *iperm = (int32_t *)malloc((size_t)(n + 1) * sizeof(int32_t));
  int32_t *fill = (int32_t *)malloc((size_t)(n + 1) * sizeof(int32_t));
  cv_pair *tmp = (cv_pair *)malloc((size_t)(nnz + 1) * sizeof(cv_pair));
  if (!iperm || !fill || !tmp) {
    free(iperm); free(fill); free(tmp);
    return 1;
  }
  for (int32_t k = 0; k < n; k++) iperm[perm[k]] = k;
  memset(orow, 0, (size_t)(n + 1) * sizeof(int32_t));
  for (int32_t i = 0; i < n; i++)
    for (int32_t e = rowptr[i]; e < rowptr[i + 1]; e++) {
      int32_t p = iperm[i], q = iperm[col[e]];
      orow[(p > q ? p : q) + 1]++;
    }
  for (int32_t i = 0; i < n; i++) orow[i + 1] += orow[i];
  for (int32_t i = 0; i < n; i++) fill[i] = orow[i];
  for (int32_t i = 0; i < n; i++)
    for (int32_t e = rowptr[i]; e < rowptr[i + 1]; e++) {
      int32_t p = iperm[i], q = iperm[col[e]];
      if (p > q) {
        tmp[fill[p]].c = q;
        tmp[fill[p]++].v = val[e];
      } else {
        tmp[fill[q]].c = p;
        tmp[fill[q]++].v = tsign * val[e];
      }
    }
  for (int32_t r = 0; r < n; r++) qsort(tmp + orow[r], (size_t)(orow[r + 1] - orow[r]), sizeof(cv_pair), cmp_cv);
  for (int32_t e = 0; e < nnz; e++) {
    ocol[e] = tmp[e].c;
    oval[e] = tmp[e].v;
  }
  free(iperm); free(fill); free(tmp);
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Three-way split of the band (Sections 1 and 3.1.2).  For a stored entry at
 * distance d = i - j: inner if d <= w_in, middle if w_in < d <= t_out, outer if
 * d > t_out.  beta = max d (0 when nnz = 0).  Negative parameters select the
 * defaults: w_in = 0 (the "inner bandwidth of size 1" is the main diagonal,
 * which for S is the shift alone) and t_out = max(beta - 3, 0) (the "outer
 * bandwidth = 3" read as the three outermost diagonals).  part[e] is 0, 1 or
 * 2; cnt[0..2] the part sizes; params[0..2] = (w_in, t_out, beta) as used.
 * Returns 1 when w_in > t_out. */
int or_split(int32_t n, const int32_t *rowptr, const int32_t *col, int32_t w_in, int32_t t_out,
             int8_t *part, int64_t *cnt, int32_t *params) {
  int32_t beta = 0;
  for (int32_t i = 0; i < n; i++)
    for (int32_t e = rowptr[i]; e < rowptr[i + 1]; e++)
      if (i - col[e] > beta) beta = i - col[e];
  if (w_in < 0) w_in = 0;
  if (t_out < 0) t_out = beta - 3 > 0 ? beta - 3 : 0;
  if (w_in > t_out) return 1;
  cnt[0] = cnt[1] = cnt[2] = 0;
  for (int32_t i = 0; i < n; i++)
    for (int32_t e = rowptr[i]; e < rowptr[i + 1]; e++) {
      int32_t d = i - col[e];
      int8_t p = d <= w_in ? 0 : (d <= t_out ? 1 : 2);
      part[e] = p;
      cnt[p]++;
    }
  params[0] = w_in;
  params[1] = t_out;
  params[2] = beta;
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Full CSR of A = alpha*I + D + S with ascending columns in every row, for
 * S = L + tsign L^T (tsign = -1: skew-symmetric, the paper's case; +1:
 * symmetric).  Row i holds l_ij for stored (i, j), then alpha + d_i at (i, i)
 * when that is nonzero (diag may be NULL: D = 0), then tsign l_ki for every
 * stored (k, i), k > i.  frow[n+1]; fcol/fval sized 2*nnz + n. */
int64_t or_full_csr_ex(int32_t n, const int32_t *rowptr, const int32_t *col, const double *val,
                       double alpha, const double *diag, double tsign, int32_t *frow, int32_t *fcol,
                       double *fval) {
  int32_t *cnt = (int32_t *)calloc((size_t)n + 1, sizeof(int32_t));
  int32_t *fill = (int32_t *)malloc((size_t)(n + 1) * sizeof(int32_t));
  if (!cnt || !fill) {
    free(cnt); free(fill);
    return -1;
  }
  for (int32_t i = 0; i < n; i++)
    for (int32_t e = rowptr[i]; e < rowptr[i + 1]; e++) {
      cnt[i]++;
      cnt[col[e]]++;
    }
  frow[0] = 0;
  for (int32_t i = 0; i < n; i++) {
    double a = alpha + (diag ? diag[i] : 0.0);
    frow[i + 1] = frow[i] + cnt[i] + (a != 0.0 ? 1 : 0);
  }
  for (int32_t i = 0; i < n; i++) {
    int32_t f = frow[i];
    for (int32_t e = rowptr[i]; e < rowptr[i + 1]; e++) {
      fcol[f] = col[e];
      fval[f++] = val[e];
    }
    double a = alpha + (diag ? diag[i] : 0.0);
    if (a != 0.0) {
      fcol[f] = i;
      fval[f++] = a;
    }
    fill[i] = f;
  }
  for (int32_t k = 0; k < n; k++)
    for (int32_t e = rowptr[k]; e < rowptr[k + 1]; e++) {
      int32_t i = col[e];
      fcol[fill[i]] = k;
      fval[fill[i]++] = tsign * val[e];
    }
  int64_t total = frow[n];
  free(cnt); free(fill);
  return total;
}

/* Full CSR of A = alpha*I + S, S skew-symmetric. */
int64_t or_full_csr(int32_t n, const int32_t *rowptr, const int32_t *col, const double *val,
                    double alpha, int32_t *frow, int32_t *fcol, double *fval) {
  return or_full_csr_ex(n, rowptr, col, val, alpha, NULL, -1.0, frow, fcol, fval);
}

/* y_i = sum_j a_ij x_j over row i in ascending column order. */
void or_csr_spmv(int32_t n, const int32_t *frow, const int32_t *fcol, const double *fval,
                 const double *x, double *y) {
  for (int32_t i = 0; i < n; i++) {
    double s = 0.0;
    for (int32_t e = frow[i]; e < frow[i + 1]; e++) s += fval[e] * x[fcol[e]];
    y[i] = s;
  }
}

/* The same full-CSR product with the rows shared among the host's threads
 * (OpenMP, static schedule).  Each row is still summed alone in ascending
 * column order, so the result equals or_csr_spmv bit for bit; this is the
 * all-core CPU baseline. */
void or_csr_spmv_par(int32_t n, const int32_t *frow, const int32_t *fcol, const double *fval,
                     const double *x, double *y) {
#pragma omp parallel for schedule(static)
  for (int32_t i = 0; i < n; i++) {
    double s = 0.0;
    for (int32_t e = frow[i]; e < frow[i + 1]; e++) s += fval[e] * x[fcol[e]];
    y[i] = s;
  }
}

/* Threads the parallel product uses (OpenMP's limit for this process). */
int or_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

/* Serial SSS skew SpMV (the paper's baseline, Section 3.1.1, adapted to skew
 * symmetry with the pair rule of eqs. (2)-(6)): y = alpha*x; then for every
 * stored l = l_ij in row order: y_i += l * x_j and y_j -= l * x_i. */
void or_sss_spmv(int32_t n, const int32_t *rowptr, const int32_t *col, const double *val,
                 double alpha, const double *x, double *y) {
  for (int32_t i = 0; i < n; i++) y[i] = alpha * x[i];
  for (int32_t i = 0; i < n; i++)
    for (int32_t e = rowptr[i]; e < rowptr[i + 1]; e++) {
      int32_t j = col[e];
      double l = val[e];
      y[i] += l * x[j];
      y[j] -= l * x[i];
    }
}

/* The serial SSS product with the diagonal array of SSS storage (Section 1)
 * and the sign of the transposed update: y = alpha*x + d .* x (diag may be
 * NULL); then y_i += l * x_j and y_j += tsign * l * x_i per stored l_ij
 * (tsign = -1 skew-symmetric, +1 symmetric). */
void or_sss_spmv_ex(int32_t n, const int32_t *rowptr, const int32_t *col, const double *val,
                    double alpha, const double *diag, double tsign, const double *x, double *y) {
  for (int32_t i = 0; i < n; i++) y[i] = alpha * x[i] + (diag ? diag[i] * x[i] : 0.0);
  for (int32_t i = 0; i < n; i++)
    for (int32_t e = rowptr[i]; e < rowptr[i + 1]; e++) {
      int32_t j = col[e];
      double l = val[e];
      y[i] += l * x[j];
      y[j] += tsign * l * x[i];
    }
}

/* ------------------------------------------------------------------------ */
/* Precision rounding.  FP64 -> FP32: IEEE round to nearest even (the C
 * conversion in the default rounding mode).  FP32 -> BF16: round to nearest
 * even on the upper 16 bits; NaN becomes a quiet NaN with the same sign. */
void or_round_f32(int64_t m, const double *in, float *out) {
  for (int64_t i = 0; i < m; i++) out[i] = (float)in[i];
}
void or_round_bf16(int64_t m, const float *in, uint16_t *out) {
  for (int64_t i = 0; i < m; i++) {
    uint32_t u;
    memcpy(&u, &in[i], 4);
    if ((u & 0x7fffffffu) > 0x7f800000u) {
      out[i] = (uint16_t)((u >> 16) | 0x0040u);
    } else {
      uint32_t lsb = (u >> 16) & 1u;
      out[i] = (uint16_t)((u + 0x7fffu + lsb) >> 16);
    }
  }
}
void or_bf16_to_f64(int64_t m, const uint16_t *in, double *out) {
  for (int64_t i = 0; i < m; i++) {
    uint32_t u = (uint32_t)in[i] << 16;
    float f;
    memcpy(&f, &u, 4);
    out[i] = (double)f;
  }
}

/* ------------------------------------------------------------------------ */
/* MRS: minimal residual iteration for (alpha*I + S) x = b (Section 1 cites
 * it: one product with S and one inner product per iteration).  x_k minimises
 * ||b - A x|| over x_0 + K_k(S, r_0).  Skew Lanczos: w = S v_j + beta_j
 * v_{j-1}, beta_{j+1} = ||w||, v_{j+1} = w / beta_{j+1}; then
 * (alpha*I + S) V_k = V_{k+1} H_k with column j of H_k holding -beta_j in row
 * j-1, alpha in row j and beta_{j+1} in row j+1.  H_k is reduced by Givens
 * rotations as in MINRES (Paige and Saunders, 1975); |eta| is the residual
 * norm of x_k.
 *   info[0] = iterations, info[1] = status (0 converged, 1 maxit,
 *   2 breakdown), info[2] = |eta|/||b||, info[3] = true ||b - A x||/||b||.
 * hist (may be NULL) receives |eta_j| / ||b|| for j = 1..iterations. */
static double dot(int32_t n, const double *a, const double *b) {
  double s = 0.0;
  for (int32_t i = 0; i < n; i++) s += a[i] * b[i];
  return s;
}

int or_mrs(int32_t n, const int32_t *rowptr, const int32_t *col, const double *val, double alpha,
           const double *b, double *x, double tol, int32_t maxit, double *hist, double *info) {
  size_t sz = (size_t)(n > 0 ? n : 1) * sizeof(double);
  double *r = (double *)malloc(sz), *v = (double *)malloc(sz), *vp = (double *)calloc((size_t)(n > 0 ? n : 1), sizeof(double));
  double *w = (double *)malloc(sz), *p = (double *)malloc(sz);
  double *p1 = (double *)calloc((size_t)(n > 0 ? n : 1), sizeof(double));
  double *p2 = (double *)calloc((size_t)(n > 0 ? n : 1), sizeof(double));
  if (!r || !v || !vp || !w || !p || !p1 || !p2) {
    free(r); free(v); free(vp); free(w); free(p); free(p1); free(p2);
    return 1;
  }
  double bnorm = sqrt(dot(n, b, b));
  int32_t it = 0, status = 1;
  double eta = 0.0;
  /* r0 = b - A x0 */
  or_sss_spmv(n, rowptr, col, val, alpha, x, r);
  for (int32_t i = 0; i < n; i++) r[i] = b[i] - r[i];
  double beta1 = sqrt(dot(n, r, r));
  if (bnorm == 0.0) bnorm = 1.0;
  eta = beta1;
  if (beta1 == 0.0 || beta1 <= tol * bnorm) {
    status = 0;
  } else {
    for (int32_t i = 0; i < n; i++) v[i] = r[i] / beta1;
    double beta_j = 0.0; /* coefficient of v_{j-1}; v_0 = 0 */
    double c1 = 1.0, s1 = 0.0, c2 = 1.0, s2 = 0.0; /* G_{j-1}, G_{j-2} */
    for (it = 1; it <= maxit; it++) {
      or_sss_spmv(n, rowptr, col, val, 0.0, v, w);
      for (int32_t i = 0; i < n; i++) w[i] += beta_j * vp[i];
      double beta_n = sqrt(dot(n, w, w));
      double eps = s2 * (-beta_j);
      double dbar = c2 * (-beta_j);
      double delta = c1 * dbar + s1 * alpha;
      double gbar = -s1 * dbar + c1 * alpha;
      double gamma = sqrt(gbar * gbar + beta_n * beta_n);
      if (gamma == 0.0) {
        status = 2;
        break;
      }
      double c = gbar / gamma, s = beta_n / gamma;
      for (int32_t i = 0; i < n; i++) p[i] = (v[i] - delta * p1[i] - eps * p2[i]) / gamma;
      for (int32_t i = 0; i < n; i++) x[i] += (c * eta) * p[i];
      eta = -s * eta;
      if (hist) hist[it - 1] = fabs(eta) / bnorm;
      c2 = c1; s2 = s1; c1 = c; s1 = s;
      double *t = p2; p2 = p1; p1 = p; p = t;
      if (fabs(eta) <= tol * bnorm || beta_n == 0.0) {
        status = 0;
        break;
      }
      for (int32_t i = 0; i < n; i++) {
        vp[i] = v[i];
        v[i] = w[i] / beta_n;
      }
      beta_j = beta_n;
    }
    if (it > maxit) it = maxit;
  }
  /* true residual of the returned x, with the full-CSR product of
   * alpha*I + S (the definition, not the recurrence) */
  {
    int64_t nnz = n > 0 ? rowptr[n] : 0;
    size_t m = (size_t)(2 * nnz + n + 1);
    int32_t *frow = (int32_t *)malloc((size_t)(n + 1) * sizeof(int32_t));
    int32_t *fcol = (int32_t *)malloc(m * sizeof(int32_t));
    double *fval = (double *)malloc(m * sizeof(double));
    if (!frow || !fcol || !fval) {
      free(frow); free(fcol); free(fval);
      free(r); free(v); free(vp); free(w); free(p); free(p1); free(p2);
      return 1;
    }
    or_full_csr(n, rowptr, col, val, alpha, frow, fcol, fval);
    or_csr_spmv(n, frow, fcol, fval, x, r);
    free(frow); free(fcol); free(fval);
  }
  for (int32_t i = 0; i < n; i++) r[i] = b[i] - r[i];
  if (info) {
    info[0] = (double)it;
    info[1] = (double)status;
    info[2] = fabs(eta) / bnorm;
    info[3] = sqrt(dot(n, r, r)) / bnorm;
  }
  free(r); free(v); free(vp); free(w); free(p); free(p1); free(p2);
  return 0;
}

/* ------------------------------------------------------------------------ */
/* 32 sparsity features of a lower CSR (the band's bandwidth and density
 * characteristics that Section 3.1.2 suggests for choosing the outer split).
 * Row lower bandwidth b_i = i - min col(i) (0 for an empty row); d = i - j per
 * entry; beta = max d; row length l_i.  Quantiles are nearest-rank on the
 * sorted b_i (rank ceil(p n), 1-based).  Ratios with a zero denominator are 0.
 *  f0  log2 n              f1  log2 nnz          f2  nnz / n
 *  f3  beta / n            f4  log2(beta + 1)
 *  f5..f9   b quantiles p10, p50, p90, p99, max, each / beta
 *  f10 nnz / sum b_i (envelope fill)
 *  f11..f18 fraction of entries with d <= 1, 2, 4, ..., 128
 *  f19..f21 fraction with d/beta > 1/2, 3/4, 9/10
 *  f22..f28 fraction of rows with length 0, 1, 2, 3-4, 5-8, 9-16, >= 17
 *  f29 max l / mean l      f30 std(l) / mean(l) (population)
 *  f31 fraction of 256-row tiles whose window r0 + 256 - lo_t (lo_t = the
 *      smallest column in the tile, r0 + 256 clipped to n) fits 160 KiB of
 *      FP64 x and y (16 bytes per row). */
static int cmp_i32(const void *a, const void *b) {
  int32_t x = *(const int32_t *)a, y = *(const int32_t *)b;
  return (x > y) - (x < y);
}

int or_features(int32_t n, const int32_t *rowptr, const int32_t *col, double *f) {
  for (int k = 0; k < 32; k++) f[k] = 0.0;
  if (n <= 0) return 0;
  int64_t nnz = rowptr[n];
  int32_t *bw = (int32_t *)malloc((size_t)n * sizeof(int32_t));
  if (!bw) return 1;
  int64_t beta = 0, sumb = 0, maxl = 0, s1 = 0, s2 = 0;
  int64_t dle[8] = {0}, dfar[3] = {0}, lenh[7] = {0};
  for (int32_t i = 0; i < n; i++) {
    int64_t l = rowptr[i + 1] - rowptr[i];
    bw[i] = l > 0 ? i - col[rowptr[i]] : 0;
    sumb += bw[i];
    if (l > maxl) maxl = l;
    s1 += l;
    s2 += l * l;
    int h = l == 0 ? 0 : l == 1 ? 1 : l == 2 ? 2 : l <= 4 ? 3 : l <= 8 ? 4 : l <= 16 ? 5 : 6;
    lenh[h]++;
    for (int32_t e = rowptr[i]; e < rowptr[i + 1]; e++) {
      int64_t d = i - col[e];
      if (d > beta) beta = d;
    }
  }
  for (int32_t i = 0; i < n; i++)
    for (int32_t e = rowptr[i]; e < rowptr[i + 1]; e++) {
      int64_t d = i - col[e];
      for (int k = 0; k < 8; k++)
        if (d <= (1 << k)) dle[k]++;
      if (2 * d > beta) dfar[0]++;
      if (4 * d > 3 * beta) dfar[1]++;
      if (10 * d > 9 * beta) dfar[2]++;
    }
  qsort(bw, (size_t)n, sizeof(int32_t), cmp_i32);
  f[0] = log2((double)n);
  f[1] = nnz > 0 ? log2((double)nnz) : 0.0;
  f[2] = (double)nnz / (double)n;
  f[3] = (double)beta / (double)n;
  f[4] = log2((double)(beta + 1));
  if (beta > 0) {
    static const int64_t pct[4] = {10, 50, 90, 99};
    for (int k = 0; k < 4; k++) {
      int64_t rank = (pct[k] * (int64_t)n + 99) / 100;
      f[5 + k] = (double)bw[rank - 1] / (double)beta;
    }
    f[9] = (double)bw[n - 1] / (double)beta;
  }
  f[10] = sumb > 0 ? (double)nnz / (double)sumb : 0.0;
  if (nnz > 0) {
    for (int k = 0; k < 8; k++) f[11 + k] = (double)dle[k] / (double)nnz;
    for (int k = 0; k < 3; k++) f[19 + k] = (double)dfar[k] / (double)nnz;
  }
  for (int k = 0; k < 7; k++) f[22 + k] = (double)lenh[k] / (double)n;
  if (s1 > 0) {
    f[29] = (double)(maxl * (int64_t)n) / (double)s1;
    f[30] = sqrt((double)((int64_t)n * s2 - s1 * s1)) / (double)s1;
  }
  int64_t tiles = (n + 255) / 256, fit = 0;
  for (int64_t t = 0; t < tiles; t++) {
    int64_t r0 = t * 256, r1 = r0 + 256 < n ? r0 + 256 : n;
    int64_t lo = r0;
    for (int64_t i = r0; i < r1; i++)
      if (rowptr[i + 1] > rowptr[i] && col[rowptr[i]] < lo) lo = col[rowptr[i]];
    if ((r1 - lo) * 16 <= 160 * 1024) fit++;
  }
  f[31] = (double)fit / (double)tiles;
  free(bw);
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Conflict map of a block-row distribution (Section 3, Fig. 2).  Block p owns
 * the rows [R_p, R_{p+1}) of the (reordered) matrix and the stored lower
 * entries of those rows.  An entry (i, j) of block p is safe (R1) when its
 * column j is also a row of block p: both of its products land in the block's
 * own outputs.  It is conflicting (R2) when j < R_p: its transposed product
 * writes y_j, which another block owns, and it reads x_j from there.  Block 0
 * never has conflicting entries.
 * bounds: nb + 1 nondecreasing row boundaries from 0 to n, or NULL for the
 * balanced R_p = floor(p n / nb).  part: the split class of every entry
 * (0 inner, 1 middle, 2 outer).  out: 11 values per block:
 *   [0] R_p  [1] rows  [2..4] safe entries per part  [5..7] conflicting
 *   entries per part  [8] reach = smallest column of a conflicting entry (R_p
 *   when there is none)  [9] partners = distinct other blocks owning such a
 *   column  [10] halo = distinct such columns (the x values the block reads
 *   from others, and the partial sums it sends back).
 * Returns 1 for nb < 1 or bad bounds, -1 when out of memory. */
int or_conflict_map(int32_t n, const int32_t *rowptr, const int32_t *col, const int8_t *part, int32_t nb,
                    const int64_t *bounds, int64_t *out) {
  if (nb < 1) return 1;
  int64_t *R = (int64_t *)malloc(((size_t)nb + 1) * sizeof(int64_t));
  int32_t *owner = (int32_t *)malloc(((size_t)n + 1) * sizeof(int32_t));
  int32_t *seen_col = (int32_t *)malloc(((size_t)n + 1) * sizeof(int32_t));
  int32_t *seen_blk = (int32_t *)malloc((size_t)nb * sizeof(int32_t));
  if (!R || !owner || !seen_col || !seen_blk) {
    free(R); free(owner); free(seen_col); free(seen_blk);
    return -1;
  }
  int bad = 0;
  for (int32_t p = 0; p <= nb; p++) R[p] = bounds ? bounds[p] : ((int64_t)p * n) / nb;
  if (R[0] != 0 || R[nb] != n) bad = 1;
  for (int32_t p = 0; p < nb && !bad; p++)
    if (R[p + 1] < R[p]) bad = 1;
  if (bad) {
    free(R); free(owner); free(seen_col); free(seen_blk);
    return 1;
  }
  for (int32_t p = 0; p < nb; p++)
    for (int64_t i = R[p]; i < R[p + 1]; i++) owner[i] = p;
  for (int32_t i = 0; i < n; i++) seen_col[i] = -1;
  for (int32_t p = 0; p < nb; p++) seen_blk[p] = -1;
  for (int32_t p = 0; p < nb; p++) {
    int64_t *o = out + (size_t)11 * p;
    for (int k = 0; k < 11; k++) o[k] = 0;
    o[0] = R[p];
    o[1] = R[p + 1] - R[p];
    o[8] = R[p];
    for (int64_t i = R[p]; i < R[p + 1]; i++) {
      for (int32_t e = rowptr[i]; e < rowptr[i + 1]; e++) {
        int32_t j = col[e];
        int k = part[e];
        if (j >= R[p]) {
          o[2 + k]++;
          continue;
        }
        o[5 + k]++;
        if (j < o[8]) o[8] = j;
        if (seen_col[j] != p) {
          seen_col[j] = p;
          o[10]++;
        }
        if (seen_blk[owner[j]] != p) {
          seen_blk[owner[j]] = p;
          o[9]++;
        }
      }
    }
  }
  free(R); free(owner); free(seen_col); free(seen_blk);
  return 0;
}

/* Conflict features of a block-row distribution over nb balanced blocks
 * (Section 3, Fig. 2: the R2 entries whose column lies in an earlier block;
 * the closing remarks of Section 4.1 propose finding such races ahead of time
 * for a given number of processors).  From the conflict map (part only
 * splits the counts, so none is needed here):
 *   f[0] = (R2 entries of all blocks) / nnz            (0 when nnz = 0)
 *   f[1] = max over blocks of halo / rows               (rows >= 1 counted)
 *   f[2] = max over blocks of (first_row - reach) / rows
 * Each is a ratio of integers in IEEE double division.  Returns 0, 1 for a
 * bad block count, -1 when out of memory. */
int or_conflict_features(int32_t n, const int32_t *rowptr, const int32_t *col, int32_t nb, double *f) {
  f[0] = f[1] = f[2] = 0.0;
  if (nb < 1) return 1;
  const int64_t nnz = rowptr[n];
  int8_t *part = (int8_t *)calloc((size_t)nnz + 1, 1);
  int64_t *map = (int64_t *)malloc((size_t)nb * 11 * sizeof(int64_t));
  if (!part || !map) {
    free(part); free(map);
    return -1;
  }
  const int r = or_conflict_map(n, rowptr, col, part, nb, NULL, map);
  if (r != 0) {
    free(part); free(map);
    return r;
  }
  int64_t conf = 0;
  for (int32_t p = 0; p < nb; p++) {
    const int64_t *o = map + (size_t)11 * p;
    conf += o[5] + o[6] + o[7];
    const int64_t rows = o[1] > 0 ? o[1] : 1;
    const double halo = (double)o[10] / (double)rows;
    const double reach = (double)(o[0] - o[8]) / (double)rows;
    if (halo > f[1]) f[1] = halo;
    if (reach > f[2]) f[2] = reach;
  }
  f[0] = nnz > 0 ? (double)conf / (double)nnz : 0.0;
  free(part); free(map);
  return 0;
}
